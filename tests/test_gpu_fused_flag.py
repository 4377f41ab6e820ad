"""GPU parity of gnm_classify_flag: the classify call and the mean-rate flag
test in one call, the test fused into the reduce kernel when a workspace is
given.  Tables and flags must equal the oracle's, and equal what
gnm_classify_aggregate followed by gnm_flag_suboptimal gives, bit for bit:
single windows (the reduce kernel overwrites the table), many windows (some
own no workspace slot, so the reduce kernel reads their rows as the classify
kernel left them), accumulation, empty runs, registries whose row count is
not a multiple of the reduce tile, and thresholds at the flagged / not
flagged edge."""
import sys

import numpy as np
import pytest

import flowgen
import oracle
import paper_1108_1785_amd as gnm
from tests._gpu import DEV, diff, offsets_to_device, to_device
from tests._helpers import random_tiny_registry, soa

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def mean_rates(exp, n_sites):
    """floor(rate_sum / bulk_flows) of every registered (site, direction) with bulk flows."""
    rows = exp.reshape(-1, exp.shape[-2], 8)[:, :2 * n_sites]
    nb, rs = rows[..., 4], rows[..., 5]
    return sorted({int(s) // int(b) for b, s in zip(nb.ravel().tolist(), rs.ravel().tolist()) if b})


def fused(reg, rec, off, threshold, min_bulk, workspace, grid_blocks=0, accumulate=False, acc=None,
          records_per_thread=0):
    import torch
    nw = 1 if off is None else len(off) - 1
    if acc is None:
        acc = torch.empty((nw, reg.rows, 8), dtype=torch.int64, device=DEV)
    flags = torch.full((nw * reg.n_sites,), 0xA5, dtype=torch.uint8, device=DEV)
    gnm.classify_flag(reg, to_device(rec), acc, flags, threshold, min_bulk,
                      window_offsets=None if off is None else offsets_to_device(off), n_windows=nw,
                      n=rec.n, accumulate=accumulate, grid_blocks=grid_blocks,
                      records_per_thread=records_per_thread,
                      workspace=gnm.make_workspace(reg, grid_blocks) if workspace else None)
    torch.cuda.synchronize()
    return acc, gnm.acc_to_numpy(acc), flags.cpu().numpy().reshape(nw, reg.n_sites)


def separate(reg, rec, off, threshold, min_bulk, workspace, grid_blocks=0):
    import torch
    nw = 1 if off is None else len(off) - 1
    acc = torch.empty((nw, reg.rows, 8), dtype=torch.int64, device=DEV)
    flags = torch.empty(nw * reg.n_sites, dtype=torch.uint8, device=DEV)
    gnm.classify_aggregate(reg, to_device(rec), acc, window_offsets=None if off is None else offsets_to_device(off),
                           n_windows=nw, n=rec.n, grid_blocks=grid_blocks,
                           workspace=gnm.make_workspace(reg, grid_blocks) if workspace else None)
    gnm.flag_suboptimal(reg, acc, nw, flags, threshold, min_bulk)
    torch.cuda.synchronize()
    return gnm.acc_to_numpy(acc), flags.cpu().numpy().reshape(nw, reg.n_sites)


_S = {}


def _small():
    if not _S:
        r = flowgen.registry_for(flowgen.PLAIN_SMALL)
        rec = flowgen.records_for(flowgen.PLAIN_SMALL, reg=r)
        orc = oracle.Registry.from_generated(r)
        _S.update(reg=r, orc=orc, rec=rec, exp=orc.classify_aggregate(rec))
    return _S


def test_fused_flag_plain_small(torch_cuda):
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    exp, n_sites = s["exp"], s["reg"].n_sites
    means = mean_rates(exp, n_sites)
    assert len(means) > 10
    mid = means[len(means) // 2]
    # the mean itself is not below the threshold: sites at exactly `mid` flip
    # between mid and mid + 1
    for thr in (1_000_000, mid, mid + 1, 0, 2**64 - 1):
        for mb in (0, 2, 40):
            want = oracle.flags(exp, n_sites, thr, mb)
            for ws in (True, False):
                say("case: plain-small threshold", thr, "min_bulk", mb, "workspace", ws)
                _, got, fl = fused(reg, s["rec"], None, thr, mb, ws)
                assert (got[0] == exp).all(), diff(got[0], exp)
                assert (fl[0] == want).all(), np.argwhere(fl[0] != want)[:5].tolist()
    assert (oracle.flags(exp, n_sites, mid) != oracle.flags(exp, n_sites, mid + 1)).any()


def test_fused_flag_windows_without_slots(torch_cuda):
    # 4 workgroups over 202 windows (some empty): a window owns a workspace
    # slot only when it is some workgroup's last, so most are merged with
    # atomics and reach the reduce kernel only for their flags
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    rec, n_sites = s["rec"], s["reg"].n_sites
    rng = np.random.default_rng(77)
    cuts = np.sort(rng.integers(0, rec.n + 1, size=200))
    off = np.concatenate([[0], cuts, [rec.n, rec.n]]).astype(np.uint64)
    exp = s["orc"].classify_aggregate(rec, window_offsets=off)
    means = mean_rates(exp, n_sites)
    thr = means[len(means) // 2]
    for grid in (4, 0):
        say("case: 202 windows, grid", grid)
        _, got, fl = fused(reg, rec, off, thr, 0, True, grid_blocks=grid)
        assert (got == exp).all(), diff(got, exp)
        assert (fl == oracle.flags(exp, n_sites, thr)).all()
        sg, sf = separate(reg, rec, off, thr, 0, True, grid_blocks=grid)
        assert (sg == got).all() and (sf == fl).all()


def test_fused_flag_accumulate(torch_cuda):
    # two calls into one table: the second call's flags judge the sums of both
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    rec, n_sites = s["rec"], s["reg"].n_sites
    half = rec.n // 2
    a, b = rec.slice(0, half), rec.slice(half, rec.n)
    exp = s["exp"]
    thr = mean_rates(exp, n_sites)[len(mean_rates(exp, n_sites)) // 3]
    for ws in (True, False):
        say("case: accumulate, workspace", ws)
        acc, _, _ = fused(reg, a, None, thr, 0, ws)
        _, got, fl = fused(reg, b, None, thr, 0, ws, accumulate=True, acc=acc)
        assert (got[0] == exp).all(), diff(got[0], exp)
        assert (fl[0] == oracle.flags(exp, n_sites, thr)).all()


def test_fused_flag_empty_run(torch_cuda):
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    empty = s["rec"].slice(0, 0)
    off = np.zeros(4, dtype=np.uint64)
    for ws in (True, False):
        say("case: empty run, 3 windows, workspace", ws)
        _, got, fl = fused(reg, empty, off, 2**64 - 1, 0, ws)
        exp = s["orc"].classify_aggregate(empty, window_offsets=off)
        assert (got == exp).all()
        assert (fl == 0).all()


@pytest.mark.parametrize("seed", range(16))
def test_fused_flag_random_tiny(torch_cuda, seed):
    import torch  # noqa: F401
    from tests.test_oracle_pins import _rate_records
    rng = np.random.default_rng(9100 + seed)
    n_sites, sites, local = random_tiny_registry(rng, n_sites=int(rng.integers(1, 10)), n_local=int(rng.integers(1, 4)))
    recs = _rate_records(rng, int(rng.integers(0, 5000)), sites, local)
    n = len(recs)
    cuts = sorted(int(c) for c in rng.integers(0, n + 1, size=int(rng.integers(0, 5))))
    off = np.array([0] + cuts + [n], dtype=np.uint64)
    nw = len(off) - 1
    grid = int(rng.choice([0, 1, 3, 300]))
    ws = rng.random() < 0.7
    rpt = int(rng.choice([0, 1, 2, 4]))
    mb = int(rng.choice([0, 1, 2, 5]))
    la, ll = [x[0] for x in local], [x[1] for x in local]
    args = ([x[0] for x in sites], [x[1] for x in sites], [x[2] for x in sites], n_sites, la, ll)
    reg, orc = gnm.Registry(*args), oracle.Registry(*args)
    rec = soa(recs)
    exp = orc.classify_aggregate(rec, window_offsets=off)
    means = mean_rates(exp, n_sites)
    thr = int(rng.choice(means)) + int(rng.integers(0, 2)) if means else int(rng.integers(0, 2**40))
    say("case: seed", seed, "sites", n_sites, "rows", reg.rows, "records", n, "windows", nw, "grid", grid,
        "ws", ws, "rpt", rpt, "min_bulk", mb, "threshold", thr)
    _, got, fl = fused(reg, rec, off, thr, mb, ws, grid_blocks=grid, records_per_thread=rpt)
    assert (got == exp).all(), diff(got, exp)
    assert (fl == oracle.flags(exp, n_sites, thr, mb)).all()


def test_fused_flag_plain_large_1m(torch_cuda):
    # the 1,000-site registry: 251 reduce tiles of four sites
    r = flowgen.registry_for(flowgen.PLAIN_LARGE)
    rec = flowgen.records_for(flowgen.PLAIN_LARGE, reg=r, n=1_000_000, stream=31)
    orc = oracle.Registry.from_generated(r)
    exp = orc.classify_aggregate(rec)
    reg = gnm.Registry.from_generated(r)
    means = mean_rates(exp, r.n_sites)
    for thr in (1_000_000, means[len(means) // 2]):
        say("case: plain-large 1M, threshold", thr)
        _, got, fl = fused(reg, rec, None, thr, 0, True)
        assert (got[0] == exp).all(), diff(got[0], exp)
        assert (fl[0] == oracle.flags(exp, r.n_sites, thr)).all()


def test_fused_flag_with_histograms_hosts_and_filters(torch_cuda):
    # every option of the classify call at once, with the flag test fused
    import torch
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    rec, n_sites = s["rec"], s["reg"].n_sites
    f = {"min_avg_packet_bytes": 100, "min_packets": 1000, "min_duration_ms": 5000}
    exp = s["orc"].classify_aggregate(rec, filters=f)
    thr = mean_rates(exp, n_sites)[len(mean_rates(exp, n_sites)) // 2]
    for ws in (True, False):
        say("case: fused flag with histograms, hosts and filters, workspace", ws)
        acc = torch.empty((1, reg.rows, 8), dtype=torch.int64, device=DEV)
        flags = torch.full((n_sites,), 0xA5, dtype=torch.uint8, device=DEV)
        hist = gnm.make_rate_hist(reg, 1)
        hosts = gnm.HostTable(reg, 1 << 16, rec.n, device=DEV)
        gnm.classify_flag(reg, to_device(rec), acc, flags, thr, 0, n=rec.n, rate_hist=hist, hosts=hosts, filters=f,
                          workspace=gnm.make_workspace(reg) if ws else None)
        torch.cuda.synchronize()
        got = gnm.acc_to_numpy(acc)[0]
        assert (got == exp).all(), diff(got, exp)
        assert (flags.cpu().numpy() == oracle.flags(exp, n_sites, thr)).all()
        S2 = 2 * n_sites
        h = hist.cpu().numpy().view(np.uint32).reshape(1, S2, -1)
        assert (h == oracle.rate_histograms(s["orc"], rec, filters=f)[:, :S2]).all()
        keys, st, med, found, _ = hosts.to_numpy()
        ek, es = oracle.host_stats(s["orc"], rec, filters=f)
        _, em = oracle.host_medians(s["orc"], rec, filters=f)
        assert found == keys.size and (keys == ek).all() and (st == es).all() and (med == em).all()
