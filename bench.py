#!/usr/bin/env python3
"""Benchmark of the flow classify/aggregate path on one MI355X.

Headline (plain-large): windows of 10,000,000 synthetic NetFlow-style records
against a registry of 1,000 collaboration sites / 20,000 CIDR prefixes
(/8../28, /24 dominant) and 8 local /16 prefixes, 70 % of site-bound records
going to the 10 most popular sites.  One step = one plain window: the
classify/aggregate call (classify kernel and its table merge) and the
sub-optimal-site flag kernel.  Inputs are resident in HBM before timing and
the timed steps rotate over distinct windows (8 x 280 MB of read fields,
well above twice the 256 MB Infinity Cache) so every step streams from HBM.

Beside the headline line, the other forms:
* batched, 8 x 10 M: the same 8 windows in one persistent launch, first with
  the default launch shape, then autotuned and replayed as a HIP graph;
* batched-256: 256 windows of uniform 10 k..2 M records (64-site registry) in
  one autotuned, graph-replayed launch;
* large-table: 10 windows of 10 M records against 1,000,000 prefixes /
  20,000 sites (lookup structure and tables beyond LDS), autotuned and
  graph-replayed;
* median: the same plain and 8-window batched steps with the rate
  histograms filled by the classify pass (keys staged in the workspace and
  counted by the histogram kernels), then the lower medians and the
  two-window warning (the paper's warning criterion);
* filtered: the plain step with the paper's exclusion filters on (average
  packet size >= 100 B, >= 1,000 packets, >= 5 s), the thresholds being this
  benchmark's choice (the paper gives none);
* ingest: a 10 M-record plain-large window as NetFlow v5 export datagrams
  (30 records per datagram, some partial), resident in HBM, decoded into the
  record arrays; then the same decode followed by classify/aggregate and the
  flag kernel on the decoded window;
* hosts: the plain step with per-host statistics and median rate buckets
  for the remote hosts of the registered sites (staged by the classify
  kernel, then partitioned by host and reduced in LDS);
* served: open-loop Poisson arrivals (200 windows/s, lognormal sizes with
  median 300 k records, capped at 5 M) through the request loop, host records
  copied in over PCIe; p50/p99 latency from scheduled arrival to result;
  then the same with the record pool already in device memory, a burst of
  2,000 windows, and 1 s runs at rising arrival rates up to the knee.

The CPU oracle is timed on the host's cores on one full window; the GPU
tables are compared with it bit for bit (plain, batched, sampled batched-256,
large-table and served windows).  Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "flow records/sec + HBM GB/s (batched vs plain, bit-exact); p99 window latency"
ALG_BYTES_PER_RECORD = 28  # src_ip, dst_ip, bytes, packets, first_ms, last_ms
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E peak


EVENT_GROUP = 5  # consecutive plain steps between one pair of HIP events


def event_period(windows: int) -> int:
    """Plain steps from one event-bracketed group to the next: the smallest prime above
    EVENT_GROUP that does not divide the window count, so the groups visit every window."""
    return next((c for c in (7, 11, 13, 17) if windows % c), EVENT_GROUP)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_classify_plain_large.txt")
POOL_STREAMS = 5           # 64-site record pool: 5 x 10 M records
POOL_STREAM_BASE = 100
TABLE_WINDOWS = 10         # large-table: 10 x 10 M records
TABLE_STREAM_BASE = 200


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def code_only(text: str) -> str:
    """C++ source without comments or blank space, so that edits to comments
    do not mark measured counters as stale (the compiled code is the same)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "gnm_internal.h"):
        with open(os.path.join(ROOT, "paper_1108_1785_amd", "csrc", f)) as fh:
            h.update(code_only(fh.read()).encode())
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


def _gen(job):
    import flowgen
    workload, n, stream = job
    return flowgen.records_for(workload, reg=flowgen.registry_for(workload), n=n, stream=stream)


def generate(jobs, workers):
    """Seeded record runs, generated on a thread pool (numpy releases the GIL
    in its bulk kernels, and each run has its own generator)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        return list(ex.map(_gen, jobs))


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def pct(a, q):
    return float(np.percentile(np.asarray(a, dtype=np.float64), q)) if len(a) else None


def timed_events(fn, steps, torch):
    """Run fn() `steps` times between HIP events on the current stream; (wall s, [ms])."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, [a.elapsed_time(b) for a, b in evs]


def served_run(gnm, serve, reg, pool_views, pool_n, seconds, rate_hz, seed, log_every=2.0, resident=False,
               burst=0):
    """Open-loop Poisson driver; latency = completion - scheduled arrival.

    burst > 0: that many windows all arrive at once instead (saturation)."""
    import flowgen
    rng = np.random.Generator(np.random.PCG64(seed))
    arr = np.zeros(burst) if burst else flowgen.poisson_arrivals(rng, rate_hz, seconds)
    sizes = flowgen.served_sizes(rng, len(arr))
    offs = (rng.random(len(arr)) * (pool_n - sizes + 1)).astype(np.int64)
    ex = serve.GpuExecutor(reg, mem_budget_bytes=4 << 30, max_batch_windows=1024, max_inflight=2)
    srv = serve.Server(ex)
    futs = []
    t0 = time.perf_counter() + 0.05
    next_log = log_every
    for i in range(len(arr)):
        t_sched = t0 + float(arr[i])
        dt = t_sched - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        o, n = int(offs[i]), int(sizes[i])
        futs.append(srv.submit({f: v[o:o + n] for f, v in pool_views.items()}, n=n, t_arrival=t_sched))
        if arr[i] >= next_log:
            log("  served%s: %.0f s, %d windows submitted" % (" (resident)" if resident else "", arr[i], i + 1))
            next_log += log_every
    res = [f.result(timeout=120) for f in futs]
    t_end = max(r_.latency_s + t0 + float(a) for r_, a in zip(res, arr)) if res else t0
    srv.close()
    lat = [r_.latency_s * 1e3 for r_ in res]
    total = int(sizes.sum())
    out = {
        "windows": len(res), "records": total, "seconds": seconds if not burst else t_end - t0,
        "arrival_rate_hz": rate_hz if not burst else None,
        "records_per_s": total / max(t_end - t0, 1e-9),
        "offered_records_per_s": total / seconds if not burst else None,
        "latency_ms_p50": pct(lat, 50), "latency_ms_p99": pct(lat, 99), "latency_ms_max": max(lat) if lat else None,
        "launches": int(srv.stats["launches"]),
        "windows_per_launch": len(res) / max(int(srv.stats["launches"]), 1),
        "admission_waits": int(srv.stats["admission_waits"]),
        "arena_records": ex.capacity,
        "host_to_device": "device-to-device staging" if resident else "pinned host -> HBM over PCIe",
    }
    return out, res, offs, sizes


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
    ap.add_argument("--no-forms", action="store_true",
                    help="plain and default batched launches only (profiling runs)")
    ap.add_argument("--no-workspace", action="store_true", help="merge tables with atomics only")
    ap.add_argument("--served-seconds", type=float, default=60.0,
                    help="length of the served run (the served-stream workload is 60 s)")
    ap.add_argument("--served-rate", type=float, default=200.0)
    ap.add_argument("--gen-workers", type=int, default=12)
    ap.add_argument("--no-large-table", action="store_true", help="skip the 1,000,000-prefix leg")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this many MiB first (scale for FETCH/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: windows would shard across GPUs with no exchange, and this "
              "path has no multi-GPU launch. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import flowgen

    # ---------------------------------------------------------------- data
    t_gen = time.time()
    jobs = [(flowgen.PLAIN_LARGE, None, k) for k in range(args.windows)]
    if not args.no_forms:
        jobs += [(flowgen.PLAIN_SMALL, 10_000_000, POOL_STREAM_BASE + k) for k in range(POOL_STREAMS)]
        if not args.no_large_table:
            jobs += [(flowgen.LARGE_TABLE, 10_000_000, TABLE_STREAM_BASE + k) for k in range(TABLE_WINDOWS)]
    runs = generate(jobs, args.gen_workers)
    parts = runs[:args.windows]
    pool_parts = runs[args.windows:args.windows + POOL_STREAMS]
    table_parts = runs[args.windows + POOL_STREAMS:]
    log("generated %d record runs in %.1fs" % (len(runs), time.time() - t_gen))
    t_gen = time.time()
    v5_rec = flowgen.v5_records(flowgen.PLAIN_LARGE, 10_000_000, stream=1)
    v5_buf, v5_off = flowgen.encode_netflow_v5(v5_rec, np.random.Generator(np.random.PCG64(flowgen.SEED_BASE + 500)))
    log("encoded %d records into %d NetFlow v5 datagrams (%.0f MB) in %.1fs" %
        (v5_rec.n, len(v5_off) - 1, v5_buf.size / 1e6, time.time() - t_gen))

    import torch

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

    reg_h = flowgen.registry_for(flowgen.PLAIN_LARGE)
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

    # ---------------------------------------------------------------- plain
    views = [{f: t[k * n_win:(k + 1) * n_win] for f, t in d.items()} for k in range(args.windows)]
    structs = [gnm.records_struct(v, n_win) for v in views]
    acc = torch.empty((1, rows, 8), dtype=torch.int64, device=dev)
    flags = torch.empty(n_sites, dtype=torch.uint8, device=dev)
    ws = None if args.no_workspace else gnm.make_workspace(reg, args.grid_blocks, device=dev)
    kw = dict(records_per_thread=args.records_per_thread, grid_blocks=args.grid_blocks, workspace=ws)

    def plain_step(k, ev=None):
        # one call: classify kernel, then the workspace reduce with the flag test
        # (or the flag kernel, without a workspace)
        if ev is not None:
            ev[0].record()
        gnm.classify_flag(reg, structs[k], acc, flags, **kw)
        if ev is not None:
            ev[1].record()

    for s in range(args.warmup):
        plain_step(s % args.windows)
    torch.cuda.synchronize()
    # A HIP event pair costs about 7 us of GPU time per step here (a 10 M window
    # takes 102.9 us per step without events, 110.1 us with a pair around every
    # step), and part of it falls inside the interval it measures.  So one pair
    # brackets each group of `group` back-to-back steps (EVENT_GROUP, or all
    # of a shorter run), a group starting every `period` steps, and a call's
    # time is the group's interval divided by `group`.
    if args.steps < 1:
        raise SystemExit("--steps must be at least 1")
    group = min(EVENT_GROUP, args.steps)
    period = max(event_period(args.windows), group)
    starts = [s for s in range(0, args.steps - group + 1, period)]
    evs = {s: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for s in starts}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        g = s - (s % period)
        if g in evs and s == g:
            evs[g][0].record()
        plain_step(s % args.windows)
        if g in evs and s == g + group - 1:
            evs[g][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = [a.elapsed_time(b) / group for a, b in evs.values()]
    k_avg = float(np.mean(kms))
    value = args.steps * n_win / wall
    log("plain: %.3f ms/step, classify call avg %.4f ms (min %.4f) -> %.1f GB/s" %
        (wall / args.steps * 1e3, k_avg, min(kms), n_win * ALG_BYTES_PER_RECORD / (k_avg * 1e-3) / 1e9))

    # ---------------------------------------------------------------- batched 8 x 10 M
    nb = args.windows
    acc_b = torch.empty((nb, rows, 8), dtype=torch.int64, device=dev)
    flags_b = torch.empty(nb * n_sites, dtype=torch.uint8, device=dev)
    bstruct = gnm.records_struct(d, big.n)

    def batched_step(ev=None):
        if ev is not None:
            ev[0].record()
        gnm.classify_flag(reg, bstruct, acc_b, flags_b, window_offsets=off_dev, n_windows=nb, **kw)
        if ev is not None:
            ev[1].record()

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
    log("batched (default shape): %.3f ms/step, classify call avg %.4f ms -> %.1f GB/s" %
        ((tb1 - tb0) / args.batched_steps * 1e3, bk, big.n * ALG_BYTES_PER_RECORD / (bk * 1e-3) / 1e9))
    got_batched = gnm.acc_to_numpy(acc_b)[0].copy()

    forms = {
        "plain": {"records_per_s": value, "call_ms_avg": k_avg,
                  "kernel_gb_s": n_win * ALG_BYTES_PER_RECORD / (k_avg * 1e-3) / 1e9},
        "batched_default": {"windows": nb, "records": big.n, "records_per_s": b_rate, "call_ms_avg": bk,
                            "kernel_gb_s": big.n * ALG_BYTES_PER_RECORD / (bk * 1e-3) / 1e9},
    }
    parity_notes = {}
    graph_batched_ok = True

    # ---------------------------------------------------------------- median statistic
    hist_bytes = gnm.rate_hist_words(reg) * 4
    hist1 = gnm.make_rate_hist(reg, 1, device=dev)
    med1 = torch.empty(2 * n_sites, dtype=torch.int32, device=dev)
    mflags1 = torch.empty(n_sites, dtype=torch.uint8, device=dev)

    # a workspace that also holds the staged histogram keys (histogram kernels
    # instead of the LDS cache, device atomics and the zeroing pass)
    kw_h = dict(kw, workspace=None if args.no_workspace else
                gnm.make_workspace(reg, args.grid_blocks, device=dev, n_records=n_win, hist=True))

    def median_step(k, ev=None):
        # classify call with histograms (classify, merge, histogram kernels), then medians + warning
        if ev is not None:
            ev[0].record()
        gnm.classify_aggregate(reg, structs[k], acc, rate_hist=hist1, **kw_h)
        if ev is not None:
            ev[1].record()
        gnm.median_flags(reg, hist1, 1, mflags1, median_bucket=med1)
        if ev is not None:
            ev[2].record()

    for s in range(args.warmup):
        median_step(s % args.windows)
    mev = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    tm0 = time.perf_counter()
    for s in range(args.steps):
        median_step(s % args.windows, mev[s])
    torch.cuda.synchronize()
    wall_m = time.perf_counter() - tm0
    mk = float(np.mean([a.elapsed_time(b) for a, b, _ in mev]))
    mm = float(np.mean([b.elapsed_time(c) for _, b, c in mev]))
    median_step(0)
    torch.cuda.synchronize()
    got_m = (hist1.cpu().numpy().view(np.uint32).copy(), med1.cpu().numpy().view(np.uint32).copy(),
             mflags1.cpu().numpy().copy())
    log("median (plain): %.3f ms/step; classify+histogram call %.4f ms (plain call %.4f), medians %.4f ms" %
        (wall_m / args.steps * 1e3, mk, k_avg, mm))
    hist_b = gnm.make_rate_hist(reg, nb, device=dev)
    med_b = torch.empty(nb * 2 * n_sites, dtype=torch.int32, device=dev)
    mflags_b = torch.empty(nb * n_sites, dtype=torch.uint8, device=dev)
    kw_hb = dict(kw, workspace=None if args.no_workspace else
                 gnm.make_workspace(reg, args.grid_blocks, device=dev, n_records=big.n, n_windows=nb, hist=True))

    def median_batched(ev=None):
        if ev is not None:
            ev[0].record()
        gnm.classify_aggregate(reg, bstruct, acc_b, window_offsets=off_dev, n_windows=nb, rate_hist=hist_b, **kw_hb)
        if ev is not None:
            ev[1].record()
        gnm.median_flags(reg, hist_b, nb, mflags_b, median_bucket=med_b)
        if ev is not None:
            ev[2].record()

    median_batched()
    mbev = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(args.batched_steps)]
    torch.cuda.synchronize()
    tmb0 = time.perf_counter()
    for s in range(args.batched_steps):
        median_batched(mbev[s])
    torch.cuda.synchronize()
    wall_mb = time.perf_counter() - tmb0
    mbk = float(np.mean([a.elapsed_time(b) for a, b, _ in mbev]))
    mbm = float(np.mean([b.elapsed_time(c) for _, b, c in mbev]))
    got_mb = (hist_b[[0, nb - 1]].cpu().numpy().view(np.uint32).copy(),
              med_b.cpu().numpy().view(np.uint32).reshape(nb, 2 * n_sites).copy(),
              mflags_b.cpu().numpy().reshape(nb, n_sites).copy())
    log("median (batched %d x 10M): %.3f ms/step; classify+histogram call %.4f ms, medians %.4f ms" %
        (nb, wall_mb / args.batched_steps * 1e3, mbk, mbm))
    # bytes each step must move at the least: the records' read fields, the
    # histograms written once and read once (medians)
    m_alg = n_win * ALG_BYTES_PER_RECORD + 2 * hist_bytes
    forms["median"] = {
        "records_per_s": args.steps * n_win / wall_m, "step_ms": wall_m / args.steps * 1e3,
        "classify_hist_call_ms_avg": mk, "median_call_ms_avg": mm, "plain_call_ms_avg": k_avg,
        "histogram_overhead": mk / k_avg - 1.0, "hist_bytes_per_window": hist_bytes,
        "alg_bytes_per_step": m_alg, "step_gb_s": m_alg / ((mk + mm) * 1e-3) / 1e9,
        "launch": "classify call with rate histograms, then gnm_median_flags (one window per step)"}
    forms["median_batched"] = {
        "windows": nb, "records": big.n, "records_per_s": args.batched_steps * big.n / wall_mb,
        "step_ms": wall_mb / args.batched_steps * 1e3, "classify_hist_call_ms_avg": mbk, "median_call_ms_avg": mbm,
        "histogram_overhead": mbk / bk - 1.0,
        "step_gb_s": (big.n * ALG_BYTES_PER_RECORD + 2 * nb * hist_bytes) / ((mbk + mbm) * 1e-3) / 1e9,
        "launch": "one persistent classify launch with histograms over %d windows, then medians and the "
                  "two-window warning over them" % nb}
    del hist_b, kw_hb

    # ---------------------------------------------------------------- NetFlow v5 ingest
    d_v5 = torch.from_numpy(v5_buf).to(dev)
    d_v5off = torch.from_numpy(v5_off.view(np.int64)).to(dev)
    n_v5 = v5_rec.n
    v5_out = gnm.make_records_out(n_v5, device=dev)
    v5_ws = torch.empty(gnm.netflow_v5_workspace_bytes(len(v5_off) - 1), dtype=torch.uint8, device=dev)
    v5_cnt = torch.empty(2, dtype=torch.int64, device=dev)
    v5_struct = gnm.records_struct(v5_out, n_v5)

    def ingest_call():
        gnm.netflow_v5_decode(d_v5, d_v5off, v5_out, workspace=v5_ws, counts=v5_cnt)

    for _ in range(args.warmup):
        ingest_call()
    wall_i, ims = timed_events(ingest_call, args.steps, torch)
    ik = float(np.mean(ims))

    def ingest_classify():
        ingest_call()
        gnm.classify_flag(reg, v5_struct, acc, flags, **kw)

    wall_ic, icms = timed_events(ingest_classify, args.steps, torch)
    torch.cuda.synchronize()
    got_v5 = {f: t.cpu().numpy() for f, t in v5_out.items()}
    got_v5_cnt = v5_cnt.cpu().numpy().tolist()
    got_v5_acc = gnm.acc_to_numpy(acc)[0].copy()
    v5_alg = v5_buf.size + v5_off.size * 8 + n_v5 * 33  # datagrams + offsets read, 33 B per record written
    # reference: a plain 1 GiB device-to-device copy (reads and writes, like the decode)
    cp_src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    cp_dst = torch.empty_like(cp_src)
    cp_dst.copy_(cp_src)
    _, cpms = timed_events(lambda: cp_dst.copy_(cp_src), 5, torch)
    copy_gbs = 2 * (1 << 30) / (float(np.mean(cpms)) * 1e-3) / 1e9
    del cp_src, cp_dst
    forms["ingest"] = {
        "records": n_v5, "datagrams": len(v5_off) - 1, "datagram_bytes": int(v5_buf.size),
        "decode_call_ms_avg": ik, "records_per_s": n_v5 / (ik * 1e-3),
        "alg_bytes_per_call": v5_alg, "decode_gb_s": v5_alg / (ik * 1e-3) / 1e9,
        "reference_copy_gb_s": copy_gbs,
        "ingest_classify_step_ms": float(np.mean(icms)), "ingest_classify_records_per_s": args.steps * n_v5 / wall_ic,
        "launch": "gnm_netflow_v5_decode (count, 3 scan passes, decode), then classify call + flag"}
    log("ingest: decode %.4f ms (%.1f G records/s, %.0f GB/s; a 1 GiB device copy runs at %.0f GB/s); "
        "decode + classify step %.4f ms" % (ik, n_v5 / (ik * 1e-3) / 1e9, v5_alg / (ik * 1e-3) / 1e9, copy_gbs,
                                            float(np.mean(icms))))
    del d_v5, v5_ws

    # ---------------------------------------------------------------- per-host statistics
    host_t = gnm.HostTable(reg, 1 << 20, n_win, device=dev)
    kw_h = dict(kw, hosts=host_t)
    hstep = [0]

    def hosts_call():
        gnm.classify_aggregate(reg, structs[hstep[0] % args.windows], acc, **kw_h)
        hstep[0] += 1

    for _ in range(args.warmup):
        hosts_call()
    wall_h, hms = timed_events(hosts_call, args.steps, torch)
    hk = float(np.mean(hms))
    gnm.classify_aggregate(reg, structs[0], acc, **kw_h)
    torch.cuda.synchronize()
    got_hosts = host_t.to_numpy()
    forms["hosts"] = {"records_per_s": args.steps * n_win / wall_h, "call_ms_avg": hk, "plain_call_ms_avg": k_avg,
                      "overhead_vs_plain": hk / k_avg - 1.0, "table_capacity": host_t.capacity,
                      "hosts_window0": got_hosts[3], "host_flows_window0": got_hosts[4],
                      "launch": "classify call staging the bulk flows of registered sites, then partition counts, "
                                "their scan, the scatter and the per-partition reduce (statistics and medians)"}
    log("hosts: classify call with per-host statistics and medians %.4f ms (plain %.4f), %d hosts in window 0" %
        (hk, k_avg, got_hosts[3]))
    del host_t

    # ---------------------------------------------------------------- exclusion filters
    filt = {"min_avg_packet_bytes": 100, "min_packets": 1000, "min_duration_ms": 5000}
    kw_f = dict(kw, filters=filt)
    for s in range(args.warmup):
        gnm.classify_aggregate(reg, structs[s % args.windows], acc, **kw_f)
    fstep = [0]

    def filtered_call():
        gnm.classify_aggregate(reg, structs[fstep[0] % args.windows], acc, **kw_f)
        fstep[0] += 1

    wall_f, fms = timed_events(filtered_call, args.steps, torch)
    fk = float(np.mean(fms))
    gnm.classify_aggregate(reg, structs[0], acc, **kw_f)
    torch.cuda.synchronize()
    got_f = gnm.acc_to_numpy(acc)[0].copy()
    forms["filtered"] = {"records_per_s": args.steps * n_win / wall_f, "call_ms_avg": fk,
                         "plain_call_ms_avg": k_avg, "filters": filt,
                         "kernel_gb_s": n_win * ALG_BYTES_PER_RECORD / (fk * 1e-3) / 1e9}
    log("filtered (plain window, %s): classify call %.4f ms (plain %.4f)" % (filt, fk, k_avg))

    if not args.no_forms:
        from paper_1108_1785_amd import serve, tune
        # ------------------------------------------------------------ batched, tuned + graph
        ws_tune = tune.tuning_workspace(reg, device=dev)
        tp = tune.tuned_params(reg, bstruct, acc_b, window_offsets=off_dev, n_windows=nb, n=big.n, workspace=ws_tune)
        del ws_tune
        log("autotune 8x10M: rpt=%d grid=%d (%.4f ms)%s" % (tp["records_per_thread"], tp["grid_blocks"],
                                                         tp["best_ms"], " cached" if tp["cached"] else ""))
        ws_t = gnm.make_workspace(reg, tp["grid_blocks"], device=dev)
        g = gnm.Graph(reg, bstruct, acc_b, window_offsets=off_dev, n_windows=nb, flags=flags_b,
                      records_per_thread=tp["records_per_thread"], grid_blocks=tp["grid_blocks"], workspace=ws_t)
        g.launch()
        wall_g, gms = timed_events(g.launch, args.batched_steps, torch)
        gk = float(np.mean(gms))
        graph_batched_ok = bool((gnm.acc_to_numpy(acc_b)[0] == got_batched).all())
        forms["batched"] = {"windows": nb, "records": big.n, "records_per_s": args.batched_steps * big.n / wall_g,
                            "step_ms_avg": gk, "kernel_gb_s": big.n * ALG_BYTES_PER_RECORD / (gk * 1e-3) / 1e9,
                            "launch": "hipGraph replay (classify + merge + flag)",
                            "records_per_thread": tp["records_per_thread"], "grid_blocks": tp["grid_blocks"],
                            "tune_candidates": len(tp["tried"])}
        log("batched (tuned, graph): %.4f ms/step -> %.1f GB/s" % (gk, forms["batched"]["kernel_gb_s"]))
        del g

        # ------------------------------------------------------------ batched-256
        reg1_h = flowgen.registry_for(flowgen.PLAIN_SMALL)
        reg1 = gnm.Registry.from_generated(reg1_h)
        pool = flowgen.concat(pool_parts)
        pool.window_offsets = None
        pool_dev = {}
        for f in ("src_ip", "dst_ip", "packets", "first_ms", "last_ms"):
            pool_dev[f] = torch.from_numpy(getattr(pool, f).view(np.int32)).to(dev)
        pool_dev["bytes"] = torch.from_numpy(pool.bytes.view(np.int64)).to(dev)
        rng = np.random.Generator(np.random.PCG64(flowgen.SEED_BASE + 256))
        sizes = flowgen.window_sizes(rng, 256, 10_000, 2_000_000)
        starts = (rng.random(256) * (pool.n - sizes + 1)).astype(np.int64)
        offs256 = np.zeros(257, dtype=np.int64)
        np.cumsum(sizes, out=offs256[1:])
        n256 = int(offs256[-1])
        d256 = {f: torch.empty(n256, dtype=t.dtype, device=dev) for f, t in pool_dev.items()}
        for w in range(256):
            for f, t in pool_dev.items():
                d256[f][offs256[w]:offs256[w + 1]].copy_(t[starts[w]:starts[w] + sizes[w]])
        off256_dev = torch.from_numpy(offs256).to(dev)
        s256 = gnm.records_struct(d256, n256)
        acc256 = torch.empty((256, reg1.rows, 8), dtype=torch.int64, device=dev)
        flags256 = torch.empty(256 * reg1_h.n_sites, dtype=torch.uint8, device=dev)
        ws1 = tune.tuning_workspace(reg1, device=dev)
        tp2 = tune.tuned_params(reg1, s256, acc256, window_offsets=off256_dev, n_windows=256, n=n256, workspace=ws1)
        del ws1
        ws1t = gnm.make_workspace(reg1, tp2["grid_blocks"], device=dev)
        g2 = gnm.Graph(reg1, s256, acc256, window_offsets=off256_dev, n_windows=256, flags=flags256,
                       records_per_thread=tp2["records_per_thread"], grid_blocks=tp2["grid_blocks"], workspace=ws1t)
        g2.launch()
        wall2, g2ms = timed_events(g2.launch, args.batched_steps, torch)
        g2k = float(np.mean(g2ms))
        forms["batched_256"] = {"windows": 256, "records": n256, "records_per_s": args.batched_steps * n256 / wall2,
                                "step_ms_avg": g2k, "kernel_gb_s": n256 * ALG_BYTES_PER_RECORD / (g2k * 1e-3) / 1e9,
                                "launch": "hipGraph replay (classify + merge + flag)",
                                "records_per_thread": tp2["records_per_thread"], "grid_blocks": tp2["grid_blocks"],
                                "registry": "64 sites / 512 prefixes",
                                "window_records": "uniform 10,000..2,000,000 (seeded)"}
        log("batched-256 (%d records): %.4f ms/step -> %.1f GB/s" % (n256, g2k, forms["batched_256"]["kernel_gb_s"]))
        acc256_h = gnm.acc_to_numpy(acc256).copy()
        flags256_h = flags256.cpu().numpy().reshape(256, reg1_h.n_sites).copy()
        del g2

        # ------------------------------------------------------------ plain-small (latency)
        # one 100,000-record window against the 64-site registry: a few
        # microseconds of work, so the launch and the synchronisation are the
        # cost; reported as per-call latency, not against the HBM roofline
        small_rec = flowgen.records_for(flowgen.PLAIN_SMALL, reg=reg1_h)
        d_small = {}
        for f in ("src_ip", "dst_ip", "packets", "first_ms", "last_ms"):
            d_small[f] = torch.from_numpy(getattr(small_rec, f).view(np.int32)).to(dev)
        d_small["bytes"] = torch.from_numpy(small_rec.bytes.view(np.int64)).to(dev)
        s_small = gnm.records_struct(d_small, small_rec.n)
        acc_s = torch.empty((1, reg1.rows, 8), dtype=torch.int64, device=dev)
        flags_s = torch.empty(reg1_h.n_sites, dtype=torch.uint8, device=dev)
        ws_s = gnm.make_workspace(reg1, device=dev)

        def small_call():
            gnm.classify_flag(reg1, s_small, acc_s, flags_s, workspace=ws_s)

        for _ in range(20):
            small_call()
        torch.cuda.synchronize()
        n_lat = 500
        host_ms = []
        for _ in range(n_lat):
            t_a = time.perf_counter()
            small_call()
            torch.cuda.synchronize()
            host_ms.append((time.perf_counter() - t_a) * 1e3)
        _, dev_ms = timed_events(small_call, n_lat, torch)
        wall_sb, _ = timed_events(small_call, n_lat, torch)
        acc_s_h = gnm.acc_to_numpy(acc_s)[0].copy()
        flags_s_h = flags_s.cpu().numpy().copy()
        forms["plain_small"] = {
            "records": small_rec.n, "calls": n_lat,
            "latency_ms_p50": pct(host_ms, 50), "latency_ms_p99": pct(host_ms, 99),
            "latency_from": "host clock around one call and a stream synchronisation",
            "device_ms_p50": pct(dev_ms, 50), "device_ms_p99": pct(dev_ms, 99),
            "device_from": "HIP events around each call (an event pair adds a few microseconds)",
            "records_per_s_back_to_back": n_lat * small_rec.n / wall_sb,
            "registry": "64 sites / 512 prefixes",
            "launch": "gnm_classify_flag with a workspace (classify kernel, reduce with the flag test)"}
        log("plain-small (100k): latency p50 %.4f ms p99 %.4f ms; device p50 %.4f ms; back to back %.3g records/s" %
            (forms["plain_small"]["latency_ms_p50"], forms["plain_small"]["latency_ms_p99"],
             forms["plain_small"]["device_ms_p50"], forms["plain_small"]["records_per_s_back_to_back"]))

        # ------------------------------------------------------------ large-table
        if table_parts:
            reg5_h = flowgen.registry_for(flowgen.LARGE_TABLE)
            t5 = time.time()
            reg5 = gnm.Registry.from_generated(reg5_h)
            t5 = time.time() - t5
            big5 = flowgen.concat(table_parts)
            d5 = {}
            for f in ("src_ip", "dst_ip", "packets", "first_ms", "last_ms"):
                d5[f] = torch.from_numpy(getattr(big5, f).view(np.int32)).to(dev)
            d5["bytes"] = torch.from_numpy(big5.bytes.view(np.int64)).to(dev)
            off5 = torch.from_numpy(big5.window_offsets.view(np.int64)).to(dev)
            s5 = gnm.records_struct(d5, big5.n)
            nw5 = len(table_parts)
            acc5 = torch.empty((nw5, reg5.rows, 8), dtype=torch.int64, device=dev)
            flags5 = torch.empty(nw5 * reg5_h.n_sites, dtype=torch.uint8, device=dev)
            ws5 = tune.tuning_workspace(reg5, device=dev, n_records=big5.n, n_windows=nw5)
            tp5 = tune.tuned_params(reg5, s5, acc5, window_offsets=off5, n_windows=nw5, n=big5.n, workspace=ws5)
            del ws5
            ws5 = gnm.make_workspace(reg5, tp5["grid_blocks"], device=dev, n_records=big5.n, n_windows=nw5)
            g5 = gnm.Graph(reg5, s5, acc5, window_offsets=off5, n_windows=nw5, flags=flags5,
                           records_per_thread=tp5["records_per_thread"], grid_blocks=tp5["grid_blocks"],
                           workspace=ws5)
            g5.launch()
            wall5, g5ms = timed_events(g5.launch, max(3, args.batched_steps // 2), torch)
            g5k = float(np.mean(g5ms))
            i5 = reg5.info()
            forms["large_table"] = {
                "windows": nw5, "records": big5.n, "records_per_s": len(g5ms) * big5.n / wall5,
                "step_ms_avg": g5k, "kernel_gb_s": big5.n * ALG_BYTES_PER_RECORD / (g5k * 1e-3) / 1e9,
                "launch": "hipGraph replay (classify + flag)", "records_per_thread": tp5["records_per_thread"],
                "grid_blocks": tp5["grid_blocks"], "registry": "20,000 sites / 1,000,000 prefixes",
                "registry_build_s": t5, "acc_in_lds": i5["acc_in_lds"], "lines_in_lds": i5["lines_in_lds"],
                "wide_nodes": i5["n_nodes"], "leaf_lines": i5["n_leaf_lines"], "device_bytes": i5["device_bytes"]}
            log("large-table (%d records): %.4f ms/step -> %.1f GB/s (registry build %.1fs)" %
                (big5.n, g5k, forms["large_table"]["kernel_gb_s"], t5))
            acc5_h = gnm.acc_to_numpy(acc5).copy()
            flags5_h = flags5.cpu().numpy().reshape(nw5, reg5_h.n_sites).copy()
            del g5, d5, s5

        # ------------------------------------------------------------ served
        pinned = {}
        for f in ("src_ip", "dst_ip", "packets", "first_ms", "last_ms", "bytes"):
            a = getattr(pool, f).view(np.int64 if f == "bytes" else np.int32)
            t = torch.empty(a.shape, dtype=torch.int64 if f == "bytes" else torch.int32, pin_memory=True)
            t.numpy()[:] = a
            pinned[f] = t
        log("served: %.0f s at %.0f windows/s from a %d-record pinned pool" %
            (args.served_seconds, args.served_rate, pool.n))
        sv, sv_res, sv_offs, sv_sizes = served_run(gnm, serve, reg1, pinned, pool.n, args.served_seconds,
                                                   args.served_rate, flowgen.SEED_BASE + 400)
        log("served: p50 %.3f ms p99 %.3f ms, %.3g records/s, %.1f windows/launch" %
            (sv["latency_ms_p50"], sv["latency_ms_p99"], sv["records_per_s"], sv["windows_per_launch"]))
        rs_seconds = max(args.served_seconds / 2, 1.0)
        svr, svr_res, svr_offs, svr_sizes = served_run(gnm, serve, reg1, pool_dev, pool.n, rs_seconds,
                                                       args.served_rate, flowgen.SEED_BASE + 401, resident=True)
        log("served (resident): p50 %.3f ms p99 %.3f ms" % (svr["latency_ms_p50"], svr["latency_ms_p99"]))
        forms["served"] = sv
        forms["served_device_resident"] = svr
        # saturation: a burst of windows at once, from device memory; the
        # request loop batches whatever has arrived whenever a launch slot frees
        sat, sat_res, sat_offs, sat_sizes = served_run(gnm, serve, reg1, pool_dev, pool.n, 0.0, 0.0,
                                                       flowgen.SEED_BASE + 402,
                                  resident=True, burst=2000)
        log("served (burst of 2000): %.3g records/s, %.1f windows/launch, p50 %.1f ms p99 %.1f ms" %
            (sat["records_per_s"], sat["windows_per_launch"], sat["latency_ms_p50"], sat["latency_ms_p99"]))
        forms["served_saturation"] = sat
        # capacity: open-loop device-resident runs of 1 s at rising arrival
        # rates, until the completed rate falls below 90 % of the offered one
        # or p99 passes 100 ms (the knee).  Same request loop and kernels as
        # the runs checked against the oracle above; these are not re-checked.
        if args.served_seconds >= 5:
            ramp, knee = [], None
            for k, rate in enumerate((500.0, 1000.0, 2000.0, 4000.0, 8000.0, 16000.0)):
                rr, _, _, _ = served_run(gnm, serve, reg1, pool_dev, pool.n, 1.0, rate,
                                         flowgen.SEED_BASE + 410 + k, resident=True, log_every=10.0)
                ramp.append({x: rr[x] for x in ("arrival_rate_hz", "windows", "records", "records_per_s",
                                                "offered_records_per_s", "latency_ms_p50", "latency_ms_p99",
                                                "windows_per_launch", "admission_waits")})
                log("served ramp %5.0f windows/s: %.3g of %.3g records/s offered, %.1f windows/launch, "
                    "p50 %.2f ms p99 %.2f ms" % (rate, rr["records_per_s"], rr["offered_records_per_s"],
                                                   rr["windows_per_launch"], rr["latency_ms_p50"],
                                                   rr["latency_ms_p99"]))
                if rr["records_per_s"] < 0.9 * rr["offered_records_per_s"] or rr["latency_ms_p99"] > 100.0:
                    knee = rate
                    break
            forms["served_ramp"] = {"runs": ramp, "knee_arrival_rate_hz": knee,
                                    "launch": "open-loop Poisson arrivals from device memory, 1 s per rate"}
        del pinned

    # ---------------------------------------------------------------- oracle
    plain_step(0)
    torch.cuda.synchronize()
    got_plain = gnm.acc_to_numpy(acc)[0].copy()
    got_flags = flags.cpu().numpy().copy()

    cpu = None
    parity = "not checked (--no-cpu)"
    if not args.no_cpu:
        import oracle
        t_orc_reg = time.perf_counter()
        orc = oracle.Registry.from_generated(reg_h)
        t_orc_reg = time.perf_counter() - t_orc_reg
        reps, t_cpu, exp = 0, 0.0, None
        while reps < 400 and (reps == 0 or t_cpu < 10.0):
            tc = time.perf_counter()
            exp = orc.classify_aggregate(parts[0])
            t_cpu += time.perf_counter() - tc
            reps += 1
            if reps == 1 or reps % 20 == 0:
                log("oracle rep %d: %.2fs" % (reps, t_cpu))
        t1 = time.perf_counter()
        orc.classify_aggregate(parts[0], threads=1)
        t1 = time.perf_counter() - t1
        cpu = {"value": reps * n_win / t_cpu, "unit": "records/s", "cores": oracle.max_threads(),
               "kind": "oracle",
               "sample": "%d x one full %d-record plain-large window (OpenMP over records)" % (reps, n_win),
               "single_thread_records_per_s": n_win / t1, "registry_build_s": t_orc_reg,
               "cpu_model": host_cpu_model(), "host_cpus_visible": os.cpu_count()}
        log("oracle: %.3g records/s on %d threads, %.3g on one; registry build %.2fs" %
            (cpu["value"], cpu["cores"], n_win / t1, t_orc_reg))
        bad = []
        if not (got_plain == exp).all():
            bad.append("plain")
        if not (got_batched == exp).all():
            bad.append("batched")
        if not graph_batched_ok:
            bad.append("batched graph")
        if not (got_flags == oracle.flags(exp, n_sites)).all():
            bad.append("flags")
        # median statistic: window 0 in full, the batched windows' medians and warnings
        S2 = 2 * n_sites
        mh = oracle.rate_histograms(orc, parts[0])[:, :S2]
        mmed, mcnt = oracle.rate_medians(orc, parts[0])
        if not (got_m[0] == mh).all():
            bad.append("median histogram")
        if not (got_m[1] == mmed[0, :S2]).all() or not (got_m[2] == oracle.median_flags(mmed, mcnt, n_sites)[0]).all():
            bad.append("median / warning")
        bmed, bcnt = oracle.rate_medians(orc, big)
        if not (got_mb[1] == bmed[:, :S2]).all() or not (got_mb[2] == oracle.median_flags(bmed, bcnt, n_sites)).all():
            bad.append("batched medians / warnings")
        if not (got_mb[0][0] == mh[0]).all() or \
                not (got_mb[0][1] == oracle.rate_histograms(orc, parts[nb - 1])[0, :S2]).all():
            bad.append("batched histograms")
        # ingest: every decoded record equals the one it was encoded from, the
        # oracle decoder agrees on 200 sampled datagrams, and the decoded
        # window's table equals the oracle's
        from oracle import netflow
        typ = {"src_port": np.uint16, "dst_port": np.uint16, "proto": np.uint8, "bytes": np.uint64}
        dec = {f: v.view(typ.get(f, np.uint32)) for f, v in got_v5.items()}
        if got_v5_cnt != [n_v5, 0] or any(not np.array_equal(dec[f], getattr(v5_rec, f)) for f in dec):
            bad.append("ingest decode")
        first = np.concatenate([[0], np.cumsum([netflow.datagram_count(v5_buf, int(v5_off[k]), int(v5_off[k + 1]))
                                                for k in range(len(v5_off) - 1)])])
        for k in np.random.default_rng(13).integers(0, len(v5_off) - 1, size=200):
            e, _ = netflow.decode_netflow_v5(v5_buf, v5_off[k:k + 2])
            lo = int(first[k])
            if any(not np.array_equal(dec[f][lo:lo + e[f].size], e[f]) for f in e):
                bad.append("ingest datagram %d" % k)
                break
        if not (got_v5_acc == orc.classify_aggregate(v5_rec)).all():
            bad.append("ingest + classify")
        parity_notes["ingest"] = "all 10M decoded records vs their source; 200 datagrams vs the oracle decoder; table"
        hk_, hs_ = oracle.host_stats(orc, parts[0])
        mk_, hm_ = oracle.host_medians(orc, parts[0])
        if got_hosts[3] != hk_.size or got_hosts[0].size != hk_.size or not (got_hosts[0] == hk_).all() or \
                not (got_hosts[1] == hs_).all() or not (mk_ == hk_).all() or not (got_hosts[2] == hm_).all() or \
                got_hosts[4] != int(hs_[:, 0].sum()):
            bad.append("hosts")
        parity_notes["hosts"] = "every host of window 0: statistics and median bucket"
        exp_f = orc.classify_aggregate(parts[0], filters=filt)
        if not (got_f == exp_f).all():
            bad.append("filtered")
        parity_notes["median_windows_checked"] = "histograms of windows 0 and %d; medians and warnings of all %d" % (
            nb - 1, nb)
        if not args.no_forms:
            orc1 = oracle.Registry.from_generated(reg1_h)
            t_chk = time.perf_counter()
            for w in range(256):
                e = orc1.classify_aggregate(pool.slice(int(starts[w]), int(starts[w] + sizes[w])))
                if not (acc256_h[w] == e).all() or not (flags256_h[w] == oracle.flags(e, reg1_h.n_sites)).all():
                    bad.append("batched-256 window %d" % w)
            parity_notes["batched_256_windows_checked"] = 256
            e = orc1.classify_aggregate(small_rec)
            if not (acc_s_h == e).all() or not (flags_s_h == oracle.flags(e, reg1_h.n_sites)).all():
                bad.append("plain-small")
            log("parity: all 256 batched-256 windows checked in %.1fs" % (time.perf_counter() - t_chk))
            if table_parts:
                t_chk = time.perf_counter()
                orc5 = oracle.Registry.from_generated(reg5_h)
                for w in range(len(table_parts)):
                    e = orc5.classify_aggregate(table_parts[w])
                    if not (acc5_h[w] == e).all() or not (flags5_h[w] == oracle.flags(e, reg5_h.n_sites)).all():
                        bad.append("large-table window %d" % w)
                parity_notes["large_table_windows_checked"] = len(table_parts)
                log("parity: all %d large-table windows checked in %.1fs" % (len(table_parts),
                                                                             time.perf_counter() - t_chk))
            # every served window, offline against the oracle
            for tag, res, offs_, sizes_ in (("served", sv_res, sv_offs, sv_sizes),
                                            ("served resident", svr_res, svr_offs, svr_sizes),
                                            ("served burst", sat_res, sat_offs, sat_sizes)):
                pick = range(len(res))
                t_chk = time.perf_counter()
                for i in pick:
                    o, n = int(offs_[i]), int(sizes_[i])
                    e = orc1.classify_aggregate(pool.slice(o, o + n))
                    if not (res[i].acc == e).all() or not (res[i].flags == oracle.flags(e, reg1_h.n_sites)).all():
                        bad.append("%s window %d" % (tag, i))
                    if (i + 1) % 2000 == 0:
                        log("parity: %s, %d of %d windows checked (%.0fs)" % (tag, i + 1, len(res),
                                                                             time.perf_counter() - t_chk))
                parity_notes["%s_windows_checked" % tag.replace(" ", "_")] = len(pick)
        parity = "bit-exact" if not bad else "MISMATCH: " + ", ".join(bad[:8])
        if bad:
            log("PARITY FAILURE: %s" % bad)

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
            "kernel": "classify_kernel + reduce_partials_kernel (one classify_flag call)",
            "kernel_ms_avg": k_avg,
            "kernel_ms_from": "HIP events around %d groups of %d consecutive timed steps (of %d), one group "
                              "every %d steps" % (len(kms), group, args.steps, period),
        },
        "cpu_baseline": cpu,
        "parity": parity,
        "parity_samples": parity_notes,
        "forms": forms,
        "registry_build_s": t_reg,
    }
    print(json.dumps(out), flush=True)
    if parity.startswith("MISMATCH"):
        sys.exit(1)


if __name__ == "__main__":
    main()
