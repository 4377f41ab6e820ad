#!/usr/bin/env python3
"""Benchmark of the flow classify/aggregate path on one MI355X.

Workload (plain-large): windows of 10,000,000 synthetic NetFlow-style records
against a registry of 1,000 collaboration sites / 20,000 CIDR prefixes
(/8../28, /24 dominant) and 8 local /16 prefixes, 70 % of site-bound records
going to the 10 most popular sites.  One step = one plain window: accumulator
initialisation, the classify/aggregate kernel over the window, and the
sub-optimal-site flag kernel.  Inputs are resident in HBM before timing and
the timed steps rotate over distinct windows (8 x 280 MB of read fields,
well above twice the 256 MB Infinity Cache) so every step streams from HBM.

Beside the headline line the batched form is measured: the same 8 windows in
one persistent launch.  The CPU oracle is timed on the host's cores on one
full window and the GPU tables of that window are compared with it bit for
bit.  Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "flow records/sec + HBM GB/s (batched vs plain, bit-exact); p99 window latency"
ALG_BYTES_PER_RECORD = 28  # src_ip, dst_ip, bytes, packets, first_ms, last_ms
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E peak
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_classify_plain_large.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "gnm_internal.h"):
        with open(os.path.join(ROOT, "paper_1108_1785_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic():
    """HBM bytes per launch from committed rocprofv3 counter runs, if current.

    The summary file holds `key: value` lines; `kernel_source_hash` must match
    the kernels as built now, else the counters are stale and traffic is null.
    """
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return float(kv["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--windows", type=int, default=8, help="distinct 10M-record windows to rotate")
    ap.add_argument("--batched-steps", type=int, default=10)
    ap.add_argument("--records-per-thread", type=int, default=0)
    ap.add_argument("--grid-blocks", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg (profiling runs)")
    ap.add_argument("--no-workspace", action="store_true", help="merge tables with atomics only")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this many MiB first (scale for FETCH/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this path has no multi-GPU launch (records shard with no "
              "exchange; see the design notes). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    import flowgen
    import paper_1108_1785_amd as gnm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    torch.cuda.set_device(0)
    gnm.lib()  # fail loudly if the HIP library is missing

    if args.calib_copy_mib:
        src = torch.ones(args.calib_copy_mib << 18, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy of %d MiB done" % args.calib_copy_mib)

    t_gen = time.time()
    reg_h = flowgen.registry_for(flowgen.PLAIN_LARGE)
    parts = []
    for k in range(args.windows):
        parts.append(flowgen.records_for(flowgen.PLAIN_LARGE, reg=reg_h, stream=k))
        log("generated window %d/%d (%.1fs)" % (k + 1, args.windows, time.time() - t_gen))
    n_win = parts[0].n
    big = flowgen.concat(parts)
    d = {}
    for f in ("src_ip", "dst_ip", "packets", "first_ms", "last_ms"):
        d[f] = torch.from_numpy(getattr(big, f).view(np.int32)).to(dev)
    d["bytes"] = torch.from_numpy(big.bytes.view(np.int64)).to(dev)
    off_dev = torch.from_numpy(big.window_offsets.view(np.int64)).to(dev)
    torch.cuda.synchronize()
    log("uploaded %d records (%.2f GB of read fields)" % (big.n, big.n * ALG_BYTES_PER_RECORD / 1e9))

    t_reg = time.time()
    reg = gnm.Registry.from_generated(reg_h)
    t_reg = time.time() - t_reg
    info = reg.info()
    rows, n_sites = reg.rows, reg_h.n_sites
    log("registry built in %.3fs: %s" % (t_reg, info))

    views = [{f: t[k * n_win:(k + 1) * n_win] for f, t in d.items()} for k in range(args.windows)]
    structs = [gnm.records_struct(v, n_win) for v in views]
    acc = torch.empty((1, rows, 8), dtype=torch.int64, device=dev)
    flags = torch.empty(n_sites, dtype=torch.uint8, device=dev)
    ws = None if args.no_workspace else gnm.make_workspace(reg, args.grid_blocks, device=dev)
    kw = dict(records_per_thread=args.records_per_thread, grid_blocks=args.grid_blocks, workspace=ws)

    def plain_step(k, ev=None):
        # one call: (table initialisation,) classify kernel, (workspace reduce)
        if ev is not None:
            ev[0].record()
        gnm.classify_aggregate(reg, structs[k], acc, **kw)
        if ev is not None:
            ev[1].record()
        gnm.flag_suboptimal(reg, acc, 1, flags)

    for s in range(args.warmup):
        plain_step(s % args.windows)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        plain_step(s % args.windows, evs[s])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    kms = [a.elapsed_time(b) for a, b in evs]
    k_avg = float(np.mean(kms))
    value = args.steps * n_win / wall
    log("plain: %.2f ms/step, kernel avg %.4f ms (min %.4f) -> %.1f GB/s" %
        (wall / args.steps * 1e3, k_avg, min(kms), n_win * ALG_BYTES_PER_RECORD / (k_avg * 1e-3) / 1e9))

    # batched form: all windows in one persistent launch
    nb = args.windows
    acc_b = torch.empty((nb, rows, 8), dtype=torch.int64, device=dev)
    flags_b = torch.empty(nb * n_sites, dtype=torch.uint8, device=dev)
    bstruct = gnm.records_struct(d, big.n)

    def batched_step(ev=None):
        if ev is not None:
            ev[0].record()
        gnm.classify_aggregate(reg, bstruct, acc_b, window_offsets=off_dev, n_windows=nb, **kw)
        if ev is not None:
            ev[1].record()
        gnm.flag_suboptimal(reg, acc_b, nb, flags_b)

    for _ in range(2):
        batched_step()
    bevs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in range(args.batched_steps)]
    torch.cuda.synchronize()
    tb0 = time.perf_counter()
    for s in range(args.batched_steps):
        batched_step(bevs[s])
    torch.cuda.synchronize()
    tb1 = time.perf_counter()
    bk = float(np.mean([a.elapsed_time(b) for a, b in bevs]))
    b_rate = args.batched_steps * big.n / (tb1 - tb0)
    log("batched: %.2f ms/step, kernel avg %.4f ms -> %.1f GB/s" %
        ((tb1 - tb0) / args.batched_steps * 1e3, bk, big.n * ALG_BYTES_PER_RECORD / (bk * 1e-3) / 1e9))

    # parity of window 0, plain and batched, against the oracle
    plain_step(0)
    torch.cuda.synchronize()
    got_plain = gnm.acc_to_numpy(acc)[0].copy()
    got_batched = gnm.acc_to_numpy(acc_b)[0].copy()
    got_flags = flags.cpu().numpy().copy()

    cpu = None
    parity = "not checked (--no-cpu)"
    if not args.no_cpu:
        import oracle
        orc = oracle.Registry.from_generated(reg_h)
        reps, t_cpu, exp = 0, 0.0, None
        while reps < 400 and (reps == 0 or t_cpu < 10.0):
            tc = time.perf_counter()
            exp = orc.classify_aggregate(parts[0])
            t_cpu += time.perf_counter() - tc
            reps += 1
            if reps == 1 or reps % 20 == 0:
                log("oracle rep %d: %.2fs" % (reps, t_cpu))
        cpu = {"value": reps * n_win / t_cpu, "unit": "records/s", "cores": oracle.max_threads(),
               "kind": "oracle",
               "sample": "%d x one full %d-record plain-large window (OpenMP over records)" % (reps, n_win)}
        ok = (got_plain == exp).all() and (got_batched == exp).all() and \
            (got_flags == oracle.flags(exp, n_sites)).all()
        parity = "bit-exact" if ok else "MISMATCH"
        if not ok:
            log("PARITY FAILURE: plain %d fields, batched %d fields differ" %
                (int((got_plain != exp).sum()), int((got_batched != exp).sum())))

    achieved = n_win * ALG_BYTES_PER_RECORD / (k_avg * 1e-3) / 1e9
    traffic = load_traffic()
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "records/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": "plain-large: one 10,000,000-record window per step, 1,000 sites / 20,000 prefixes, "
                        "8 local /16; rotating over %d distinct resident windows" % args.windows,
            "records_per_window": n_win,
            "alg_bytes_per_record": ALG_BYTES_PER_RECORD,
            "lds_bytes": info["lds_bytes"], "root_bits": info["root_bits"],
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
            "kernel": "classify_kernel + reduce_partials_kernel (one classify call)",
            "kernel_ms_avg": k_avg,
        },
        "cpu_baseline": cpu,
        "parity": parity,
        "forms": {
            "plain": {"records_per_s": value, "kernel_gb_s": achieved},
            "batched": {"windows": nb, "records": big.n, "records_per_s": b_rate,
                        "kernel_ms_avg": bk,
                        "kernel_gb_s": big.n * ALG_BYTES_PER_RECORD / (bk * 1e-3) / 1e9},
        },
        "registry_build_s": t_reg,
    }
    print(json.dumps(out), flush=True)
    if parity == "MISMATCH":
        sys.exit(1)


if __name__ == "__main__":
    main()
