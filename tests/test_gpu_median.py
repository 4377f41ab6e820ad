"""GPU parity of the median statistic: rate histograms filled by the classify
pass, lower medians and the two-window warning, through the C ABI, against
the CPU oracle.

Integer work: every histogram count, median bucket and flag byte must equal
the oracle's (tolerance 0), on generated windows (full size for the 10 M
window), the batched form with the warning chained across two calls, edge
rates around bucket edges and 1 Mbps, accumulation, the large-table
registry, graph replays, and maximum contention on one bucket.  Both ways of
filling the histograms are checked: the LDS cache with device atomics (no
workspace for the histograms), and staged keys counted by the histogram
kernels (a workspace of gnm_workspace_bytes_hist: workspace="hist"), with
one, two and four rows per partition, rows split over several slices, and
the fallback beyond 65,536 rows.
"""
import sys

import numpy as np
import pytest

import flowgen
import oracle
import paper_1108_1785_amd as gnm
from tests._gpu import DEV, offsets_to_device, to_device
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


def _regs(sites, local, n_sites, **kw):
    a, l, s = [x[0] for x in sites], [x[1] for x in sites], [x[2] for x in sites]
    la, ll = [x[0] for x in local], [x[1] for x in local]
    return gnm.Registry(a, l, s, n_sites, la, ll, **kw), oracle.Registry(a, l, s, n_sites, la, ll)


def gpu_median(reg, rec, off=None, bulk_bytes=1_000_000, threshold_bps=1_000_000, min_bulk_flows=0,
               prev=None, grid_blocks=0, records_per_thread=0, workspace=False, dev_rec=None):
    """One classify pass with histograms, then gnm_median_flags; host arrays
    (hist [nw, 2S, 10001], median [nw, 2S], flags [nw, S])."""
    import torch
    nw = 1 if off is None else len(off) - 1
    hist = gnm.make_rate_hist(reg, nw)
    hist.fill_(-1)  # stale contents: the call must zero them
    acc = torch.empty((nw, reg.rows, 8), dtype=torch.int64, device=DEV)
    d = dev_rec if dev_rec is not None else to_device(rec)
    doff = None if off is None else offsets_to_device(off)
    gnm.classify_aggregate(reg, d, acc, window_offsets=doff, n_windows=nw, bulk_bytes=bulk_bytes,
                           records_per_thread=records_per_thread, grid_blocks=grid_blocks, n=rec.n,
                           workspace=make_ws(reg, workspace, rec.n, nw, grid_blocks), rate_hist=hist)
    med = torch.full((nw * 2 * reg.n_sites,), 7, dtype=torch.int32, device=DEV)
    flg = torch.full((nw * reg.n_sites,), 0xAA, dtype=torch.uint8, device=DEV)
    pt = None if prev is None else torch.from_numpy(np.ascontiguousarray(prev, dtype=np.uint8)).to(DEV)
    gnm.median_flags(reg, hist, nw, flg, threshold_bps, min_bulk_flows, prev_flags=pt, median_bucket=med)
    torch.cuda.synchronize()
    S = reg.n_sites
    return (hist.cpu().numpy().view(np.uint32), med.cpu().numpy().view(np.uint32).reshape(nw, 2 * S),
            flg.cpu().numpy().reshape(nw, S))


def make_ws(reg, kind, n, nw=1, grid_blocks=0):
    """No workspace (False), the tables' workspace (True: histograms through
    the LDS cache and atomics), or one that also holds staged keys ("hist")."""
    if kind == "hist":
        return gnm.make_workspace(reg, grid_blocks, n_records=n, n_windows=nw, hist=True)
    return gnm.make_workspace(reg, grid_blocks) if kind else None


def oracle_median(orc, rec, off=None, bulk_bytes=1_000_000, threshold_bps=1_000_000, min_bulk_flows=0,
                  prev=None):
    S = orc.n_sites
    h = oracle.rate_histograms(orc, rec, window_offsets=off, bulk_bytes=bulk_bytes)[:, :2 * S]
    med, cnt = oracle.rate_medians(orc, rec, window_offsets=off, bulk_bytes=bulk_bytes)
    f = oracle.median_flags(med, cnt, S, threshold_bps, min_bulk_flows, prev)
    return h, med[:, :2 * S], f


def check(got, exp, what=""):
    for name, g, e in zip(("hist", "median", "flags"), got, exp):
        assert g.shape == e.shape, (what, name, g.shape, e.shape)
        bad = np.argwhere(g != e)
        assert bad.size == 0, (what, name, [(tuple(i), int(g[tuple(i)]), int(e[tuple(i)])) for i in bad[:5]])


_SMALL = {}


def _small():
    if not _SMALL:
        r = flowgen.registry_for(flowgen.PLAIN_SMALL)
        _SMALL["reg"] = r
        _SMALL["orc"] = oracle.Registry.from_generated(r)
        _SMALL["rec"] = flowgen.records_for(flowgen.PLAIN_SMALL, reg=r)
    return _SMALL


@pytest.mark.parametrize("rpt,ws", [(0, True), (0, False), (1, True), (2, False), (4, True), (0, "hist"),
                                    (1, "hist"), (2, "hist"), (4, "hist")])
def test_median_plain_small(torch_cuda, rpt, ws):
    say("case: median plain-small 100k, records_per_thread", rpt, "workspace", ws)
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    exp = oracle_median(s["orc"], s["rec"])
    got = gpu_median(reg, s["rec"], records_per_thread=rpt, workspace=ws)
    check(got, exp)
    assert got[0].sum() > 10_000 and (got[2] & 3).any()


def test_median_thresholds_and_min_bulk(torch_cuda):
    say("case: median thresholds and minimum bulk counts")
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    rec = s["rec"].slice(0, 30_000)
    for thr, mb in ((0, 0), (250_000, 0), (260_000, 40), (995_000, 1), (10_000_000, 0), (2**64 - 1, 0)):
        exp = oracle_median(s["orc"], rec, threshold_bps=thr, min_bulk_flows=mb)
        got = gpu_median(reg, rec, threshold_bps=thr, min_bulk_flows=mb)
        check(got, exp, (thr, mb))


def test_median_plain_large_full_size(torch_cuda):
    say("case: median plain-large 10M records (full size, bench launch shape)")
    r = flowgen.registry_for(flowgen.PLAIN_LARGE)
    rec = flowgen.records_for(flowgen.PLAIN_LARGE, reg=r)
    orc = oracle.Registry.from_generated(r)
    reg = gnm.Registry.from_generated(r)
    exp = oracle_median(orc, rec)
    for ws in ("hist", True):
        say("  workspace", ws)
        got = gpu_median(reg, rec, workspace=ws)
        check(got, exp, ws)


def test_median_batched_chained(torch_cuda):
    """256 windows in one launch; the warning evaluated in two calls, the
    second taking the first call's last window as its previous window."""
    import torch
    say("case: median batched 256 windows (scaled to 3M records), chained over two calls")
    r = flowgen.registry_for(flowgen.PLAIN_SMALL)
    rec = flowgen.records_for(flowgen.BATCHED, reg=r, n=3_000_000)
    off = rec.window_offsets.copy()
    nw = len(off) - 1
    orc = oracle.Registry.from_generated(r)
    reg = gnm.Registry.from_generated(r)
    prev = (np.arange(r.n_sites) % 4).astype(np.uint8)
    exp = oracle_median(orc, rec, off, prev=prev)
    # 256 windows x 128 rows: staged with four rows per partition
    for grid, ws in ((0, True), (37, False), (2000, True), (0, "hist"), (37, "hist"), (2000, "hist")):
        say("  grid", grid, "workspace", ws)
        got = gpu_median(reg, rec, off, prev=prev, grid_blocks=grid, workspace=ws)
        check(got, exp, grid)
    # the same warning from two calls over windows [0, 100) and [100, 256)
    S = r.n_sites
    hist = torch.from_numpy(got[0].view(np.int32)).to(DEV)
    f1 = torch.empty(100 * S, dtype=torch.uint8, device=DEV)
    f2 = torch.empty((nw - 100) * S, dtype=torch.uint8, device=DEV)
    gnm.median_flags(reg, hist[:100], 100, f1, prev_flags=torch.from_numpy(prev).to(DEV))
    gnm.median_flags(reg, hist[100:], nw - 100, f2, prev_flags=f1[99 * S:])
    torch.cuda.synchronize()
    both = np.concatenate([f1.cpu().numpy(), f2.cpu().numpy()]).reshape(nw, S)
    assert (both == exp[2]).all()
    assert (exp[2] & 12).any()  # the two-window rule fired somewhere


def _rate_recs(rng, n, sites, local):
    from tests.test_oracle_pins import _rate_records
    return _rate_records(rng, n, sites, local)


@pytest.mark.parametrize("seed", range(6))
def test_median_edge_rates(torch_cuda, seed):
    say("case: median edge rates, seed", seed)
    rng = np.random.default_rng(900 + seed)
    n_sites, sites, local = random_tiny_registry(rng, n_local=int(rng.integers(1, 4)))
    recs = _rate_recs(rng, 5000, sites, local)
    cuts = sorted(int(c) for c in rng.integers(0, len(recs) + 1, size=5))
    off = np.array([0] + cuts + [len(recs)], dtype=np.uint64)
    reg, orc = _regs(sites, local, n_sites)
    bulk = int(rng.choice([0, 1_000_000]))
    prev = rng.integers(0, 4, size=n_sites).astype(np.uint8)
    for thr in (1_000_000, 995_000):
        exp = oracle_median(orc, soa(recs), off, bulk_bytes=bulk, threshold_bps=thr, prev=prev)
        for grid, ws in ((0, False), (1, False), (37, False), (0, "hist"), (1, "hist"), (37, "hist")):
            got = gpu_median(reg, soa(recs), off, bulk_bytes=bulk, threshold_bps=thr, prev=prev, grid_blocks=grid,
                             workspace=ws)
            check(got, exp, (thr, grid, ws))


@pytest.mark.parametrize("ws", [False, "hist"])
def test_median_accumulate(torch_cuda, ws):
    import torch
    say("case: median histograms accumulated over two calls, workspace", ws)
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    a, b = s["rec"].slice(0, 40_000), s["rec"].slice(40_000, 100_000)
    hist = gnm.make_rate_hist(reg)
    hist.fill_(-1)
    acc = torch.empty((1, reg.rows, 8), dtype=torch.int64, device=DEV)
    gnm.classify_aggregate(reg, to_device(a), acc, n=a.n, rate_hist=hist, workspace=make_ws(reg, ws, a.n))
    gnm.classify_aggregate(reg, to_device(b), acc, n=b.n, rate_hist=hist, accumulate=True,
                           workspace=make_ws(reg, ws, b.n))
    torch.cuda.synchronize()
    exp = oracle.rate_histograms(s["orc"], s["rec"])[:, :2 * reg.n_sites]
    assert (hist.cpu().numpy().view(np.uint32) == exp).all()


@pytest.mark.parametrize("ws", [False, "hist"])
def test_median_accumulate_hot_row(torch_cuda, ws):
    """Accumulating into histograms that already hold counts, with one row
    hot enough to be split over several slices of the histogram kernels."""
    import torch
    from tests._helpers import ip
    say("case: accumulate with a row of 100k flows, workspace", ws)
    sites = [(ip("10.0.0.0"), 8, 0), (ip("11.0.0.0"), 8, 1), (ip("12.0.0.0"), 8, 2)]
    local = [(ip("192.168.0.0"), 16)]
    reg, orc = _regs(sites, local, 3)
    rng = np.random.default_rng(77)
    n = 160_000
    hot = rng.random(n) < 0.7
    dst = np.where(hot, ip("10.1.2.3"), np.uint64(ip("11.0.0.0")) + rng.integers(0, 1 << 24, n, dtype=np.uint64))
    dur = rng.integers(1, 5000, n)
    recs = [(ip("192.168.1.1"), int(d), int(b), 10, 1000, 1000 + int(t))
            for d, b, t in zip(dst, rng.integers(1_000_001, 90_000_000, n), dur)]
    rec = soa(recs)
    first, second = rec.slice(0, 70_000), rec.slice(70_000, n)
    hist = gnm.make_rate_hist(reg)
    acc = torch.empty((1, reg.rows, 8), dtype=torch.int64, device=DEV)
    gnm.classify_aggregate(reg, to_device(first), acc, n=first.n, rate_hist=hist, workspace=make_ws(reg, ws, first.n))
    gnm.classify_aggregate(reg, to_device(second), acc, n=second.n, rate_hist=hist, accumulate=True,
                           workspace=make_ws(reg, ws, second.n))
    torch.cuda.synchronize()
    exp = oracle.rate_histograms(orc, rec)[:, :6]
    got = hist.cpu().numpy().view(np.uint32)
    assert exp[0, 1].sum() > 100_000
    assert (got == exp).all(), np.argwhere(got != exp)[:5]


def test_median_large_table(torch_cuda):
    """20,000 sites: accumulator rows behind the LDS cache; every histogram
    count still lands in the record's own row."""
    say("case: median large-table registry, 1M records")
    r = flowgen.registry_for(flowgen.LARGE_TABLE)
    rec = flowgen.records_for(flowgen.LARGE_TABLE, reg=r, n=1_000_000, stream=3)
    orc = oracle.Registry.from_generated(r)
    reg = gnm.Registry.from_generated(r)
    assert not reg.info()["acc_in_lds"]
    exp = oracle_median(orc, rec)
    for ws in (True, "hist"):
        got = gpu_median(reg, rec, workspace=ws)
        check(got, exp, ws)


@pytest.mark.parametrize("ws", [True, "hist"])
def test_median_graph_replays(torch_cuda, ws):
    import torch
    say("case: graph replay with histograms, buffers refilled between replays, workspace", ws)
    s = _small()
    r, orc = s["reg"], s["orc"]
    reg = gnm.Registry.from_generated(r)
    rec_a = s["rec"]
    rec_b = flowgen.permuted(rec_a.slice(0, rec_a.n), np.random.default_rng(9))
    rec_b.bytes[::3] = rec_b.bytes[::3] * np.uint64(5)  # other rates
    d = to_device(rec_a)
    acc = torch.empty((1, reg.rows, 8), dtype=torch.int64, device=DEV)
    hist = gnm.make_rate_hist(reg)
    g = gnm.Graph(reg, d, acc, n=rec_a.n, rate_hist=hist, workspace=make_ws(reg, ws, rec_a.n))
    exp = {0: oracle.rate_histograms(orc, rec_a)[:, :2 * r.n_sites],
           1: oracle.rate_histograms(orc, rec_b)[:, :2 * r.n_sites]}
    db = to_device(rec_b)
    for it in range(4):
        src = db if it % 2 else to_device(rec_a)
        for f in d:
            d[f].copy_(src[f])
        hist.fill_(3)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert (hist.cpu().numpy().view(np.uint32) == exp[it % 2]).all(), it
    g.close()


@pytest.mark.parametrize("ws", [False, "hist"])
def test_median_one_bucket_contention(torch_cuda, ws):
    say("case: every record in one (row, bucket), workspace", ws)
    from tests._helpers import ip
    sites = [(ip("10.0.0.0"), 8, 0), (ip("11.0.0.0"), 8, 1)]
    local = [(ip("192.168.0.0"), 16)]
    reg, orc = _regs(sites, local, 2)
    n = 300_000
    recs = [(ip("192.168.1.1"), ip("10.1.2.3"), 5_000_000, 10, 1000, 1000 + 40_000)] * n
    exp = oracle_median(orc, soa(recs))
    got = gpu_median(reg, soa(recs), workspace=ws)
    check(got, exp)
    assert got[0][0, 1, 100] == n and got[1][0, 1] == 100  # 1 Mbps exactly: bucket 100, OUT row


def test_median_hist_alignment_rejected(torch_cuda):
    import torch
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    rec = s["rec"].slice(0, 1000)
    h = torch.empty(gnm.rate_hist_words(reg) + 4, dtype=torch.int32, device=DEV)
    acc = torch.empty((1, reg.rows, 8), dtype=torch.int64, device=DEV)
    with pytest.raises(gnm.GnmError) as e:
        gnm.classify_aggregate(reg, to_device(rec), acc, n=rec.n, rate_hist=h[1:])
    assert e.value.code == -1


def test_median_empty_windows(torch_cuda):
    """Empty windows have all-zero histograms, no medians and no low bits; the
    warning chain passes through them (an empty window breaks a run)."""
    say("case: median with empty windows")
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    rec = s["rec"]
    off = np.array([0, 0, 0, 30_000, 30_000, 60_000, rec.n, rec.n], dtype=np.uint64)
    prev = np.full(s["reg"].n_sites, 3, dtype=np.uint8)
    exp = oracle_median(s["orc"], rec, off, prev=prev)
    for grid, ws in ((0, False), (7, False), (0, "hist"), (7, "hist")):
        got = gpu_median(reg, rec, off, prev=prev, grid_blocks=grid, workspace=ws)
        check(got, exp, (grid, ws))
    assert (got[0][[0, 1, 3, 6]] == 0).all() and (got[1][[0, 1, 3, 6]] == oracle.NO_MEDIAN).all()
    assert (got[2][[0, 1, 3, 6]] == 0).all()


def test_median_worked_example_on_gpu(torch_cuda):
    """The hand-worked example: histograms, lower medians and flags as derived by hand."""
    from tests._helpers import dense_histograms, median_example
    say("case: median worked example")
    sites, local, S, recs, off, g = median_example()
    reg, _ = _regs(sites, local, S)
    for ws in (False, "hist"):
        got = gpu_median(reg, soa(recs), off, bulk_bytes=g["bulk_bytes"], threshold_bps=g["threshold_bps"],
                         prev=np.array(g["prev_flags"], dtype=np.uint8), workspace=ws)
        assert (got[0] == dense_histograms(g, 2 * S)).all()
        want = [[gnm.NO_MEDIAN if m == "NONE" else m for m in w] for w in g["expected_medians"]]
        assert got[1].tolist() == want
        assert got[2].tolist() == g["expected_flags"]


@pytest.mark.parametrize("nw", [130, 520])
def test_median_staged_many_windows(torch_cuda, nw):
    """130 windows x 128 rows (16,640 rows: two rows per partition) and 520
    windows (66,560 rows: beyond the staged limit, so the cache and atomics
    fill them even with the workspace)."""
    say("case: staged histograms over", nw, "windows")
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    rec = s["rec"]
    rng = np.random.default_rng(nw)
    cuts = np.sort(rng.integers(0, rec.n + 1, size=nw - 1))
    off = np.concatenate([[0], cuts, [rec.n]]).astype(np.uint64)
    exp = oracle_median(s["orc"], rec, off)
    got = gpu_median(reg, rec, off, workspace="hist")
    check(got, exp, nw)
    assert gnm.workspace_bytes_hist(reg, rec.n, nw) > gnm.workspace_bytes_n(reg, rec.n, nw) or nw == 520


def test_median_staged_with_hosts(torch_cuda):
    """Staged histogram keys and per-host entries in the same pass share one
    reservation; both results stay exact."""
    import torch
    say("case: staged histograms with per-host statistics")
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    rec = s["rec"]
    hist = gnm.make_rate_hist(reg)
    hist.fill_(-1)
    acc = torch.empty((1, reg.rows, 8), dtype=torch.int64, device=DEV)
    hosts = gnm.HostTable(reg, 1 << 16, rec.n, device=DEV)
    gnm.classify_aggregate(reg, to_device(rec), acc, n=rec.n, rate_hist=hist, hosts=hosts,
                           workspace=make_ws(reg, "hist", rec.n))
    torch.cuda.synchronize()
    exp = oracle.rate_histograms(s["orc"], rec)[:, :2 * reg.n_sites]
    assert (hist.cpu().numpy().view(np.uint32) == exp).all()
    keys, st, med, found, _ = hosts.to_numpy()
    ek, es = oracle.host_stats(s["orc"], rec)
    _, em = oracle.host_medians(s["orc"], rec)
    assert found == ek.size and (keys == ek).all() and (st == es).all() and (med == em).all()
