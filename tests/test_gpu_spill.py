"""GPU parity of the spilled accumulator table: registries whose table does
not fit LDS, classified with a workspace that holds the spilled rows (the
rows that miss a workgroup's LDS row cache and the cache flushes at window
changes become staged partial rows, merged by one workgroup per (window, 256
rows) without device-scope atomics).  Tables and flags must equal the
oracle's bit for bit in every launch shape, over windows (empty ones too),
with many segments per workgroup, accumulating, with histograms, hosts and
filters in the same pass, through graph replays, and equal the atomic path
that a workspace too small for the spill falls back to."""
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


_T = {}


def _table():
    if not _T:
        r = flowgen.registry_for(flowgen.LARGE_TABLE)
        rec = flowgen.records_for(flowgen.LARGE_TABLE, reg=r, n=2_000_000, stream=31)
        _T.update(reg=r, orc=oracle.Registry.from_generated(r), rec=rec, g=gnm.Registry.from_generated(r))
        assert not _T["g"].info()["acc_in_lds"]
    return _T


def call(reg, rec, off=None, ws=True, flags=True, threshold=1_000_000, grid_blocks=0, records_per_thread=0,
         acc=None, accumulate=False, d=None, **kw):
    import torch
    nw = 1 if off is None else len(off) - 1
    if acc is None:
        acc = torch.full((nw, reg.rows, 8), 0x77, dtype=torch.int64, device=DEV)
    fl = torch.full((nw * reg.n_sites,), 0xA5, dtype=torch.uint8, device=DEV)
    wsp = gnm.make_workspace(reg, grid_blocks, n_records=rec.n, n_windows=nw) if ws is True else ws
    args = dict(window_offsets=None if off is None else offsets_to_device(off), n_windows=nw, n=rec.n,
                grid_blocks=grid_blocks, records_per_thread=records_per_thread, workspace=wsp,
                accumulate=accumulate, **kw)
    d = to_device(rec) if d is None else d
    if flags:
        gnm.classify_flag(reg, d, acc, fl, threshold, 0, **args)
    else:
        gnm.classify_aggregate(reg, d, acc, **args)
    torch.cuda.synchronize()
    return acc, gnm.acc_to_numpy(acc), fl.cpu().numpy().reshape(nw, reg.n_sites)


def expect(orc, rec, off=None, **kw):
    e = orc.classify_aggregate(rec, window_offsets=off, **kw)
    return e if off is not None else e[None]


@pytest.mark.parametrize("rpt,grid", [(0, 0), (1, 0), (2, 0), (4, 64), (0, 700), (0, 1)])
def test_spill_launch_shapes(torch_cuda, rpt, grid):
    say("case: spilled large-table, records_per_thread", rpt, "grid", grid)
    t = _table()
    rec = t["rec"] if grid != 1 else t["rec"].slice(0, 200_000)
    exp = expect(t["orc"], rec)
    _, got, fl = call(t["g"], rec, records_per_thread=rpt, grid_blocks=grid)
    assert (got == exp).all(), diff(got, exp)
    assert (fl == oracle.flags(exp, t["reg"].n_sites)).all()


def test_spill_windows_and_segments(torch_cuda):
    say("case: spilled large-table, 6 windows (two empty), short flush segments")
    t = _table()
    rec = t["rec"]
    off = np.array([0, 1, 500_000, 500_000, 1_300_007, 2_000_000, 2_000_000], dtype=np.uint64)
    exp = expect(t["orc"], rec, off)
    for fr in (0, 5_000, 777):
        _, got, fl = call(t["g"], rec, off, flush_records=fr)
        assert (got == exp).all(), (fr, diff(got, exp))
        assert (fl == oracle.flags(exp, t["reg"].n_sites)).all()


def test_spill_accumulate_and_fallback(torch_cuda):
    say("case: spilled large-table, accumulating over two calls; atomics without the spill workspace")
    t = _table()
    rec, g = t["rec"], t["g"]
    off = np.array([0, 700_000, 2_000_000], dtype=np.uint64)
    exp = expect(t["orc"], rec, off)
    first = np.concatenate([np.arange(0, 350_000), np.arange(700_000, 1_350_000)])
    second = np.concatenate([np.arange(350_000, 700_000), np.arange(1_350_000, 2_000_000)])
    parts = []
    for idx in (first, second):
        p = flowgen.Records(*(getattr(rec, f)[idx] for f in flowgen.Records.FIELDS))
        parts.append(p)
    o1 = np.array([0, 350_000, first.size], dtype=np.uint64)
    o2 = np.array([0, 350_000, second.size], dtype=np.uint64)
    acc, _, _ = call(g, parts[0], o1, flags=False)
    _, got, fl = call(g, parts[1], o2, acc=acc, accumulate=True)
    assert (got == exp).all(), diff(got, exp)
    assert (fl == oracle.flags(exp, t["reg"].n_sites)).all()
    # a workspace too small for the spilled rows: device-scope atomics, same results
    small = gnm.make_workspace(g, 0, n_records=1000)
    _, got2, fl2 = call(g, rec, off, ws=small)
    assert (got2 == exp).all() and (fl2 == fl).all()
    _, got3, _ = call(g, rec, off, ws=None)
    assert (got3 == exp).all()


@pytest.mark.parametrize("staged", [False, True])
def test_spill_with_histograms_hosts_filters(torch_cuda, staged):
    say("case: spilled large-table with histograms, hosts and filters; staged histogram keys", staged)
    t = _table()
    rec = t["rec"].slice(0, 600_000)
    g = t["g"]
    f = {"min_avg_packet_bytes": 100, "min_packets": 500}
    hist = gnm.make_rate_hist(g)
    hist.fill_(-1)
    hosts = gnm.HostTable(g, 1 << 18, rec.n, device=DEV)
    ws = gnm.make_workspace(g, n_records=rec.n, hist=staged)
    _, got, fl = call(g, rec, rate_hist=hist, hosts=hosts, filters=f, ws=ws)
    exp = expect(t["orc"], rec, filters=f)
    assert (got == exp).all(), diff(got, exp)
    assert (fl == oracle.flags(exp, t["reg"].n_sites)).all()
    S2 = 2 * t["reg"].n_sites
    assert (hist.cpu().numpy().view(np.uint32).reshape(1, S2, -1) ==
            oracle.rate_histograms(t["orc"], rec, filters=f)[:, :S2]).all()
    keys, st, med, found, _ = hosts.to_numpy()
    ek, es = oracle.host_stats(t["orc"], rec, filters=f)
    _, em = oracle.host_medians(t["orc"], rec, filters=f)
    assert found == ek.size and (keys == ek).all() and (st == es).all() and (med == em).all()


def test_spill_graph_replays(torch_cuda):
    import torch
    say("case: spilled large-table through graph replays")
    t = _table()
    rec, g = t["rec"].slice(0, 800_000), t["g"]
    off = np.array([0, 300_000, 800_000], dtype=np.uint64)
    exp = expect(t["orc"], rec, off)
    d = to_device(rec)
    acc = torch.empty((2, g.rows, 8), dtype=torch.int64, device=DEV)
    fl = torch.empty(2 * g.n_sites, dtype=torch.uint8, device=DEV)
    ws = gnm.make_workspace(g, n_records=rec.n, n_windows=2)
    gr = gnm.Graph(g, d, acc, window_offsets=offsets_to_device(off), n_windows=2, flags=fl, n=rec.n, workspace=ws)
    for _ in range(3):
        acc.fill_(5)
        fl.fill_(9)
        torch.cuda.synchronize()
        gr.launch()
        torch.cuda.synchronize()
        got = gnm.acc_to_numpy(acc)
        assert (got == exp).all(), diff(got, exp)
        assert (fl.cpu().numpy().reshape(2, g.n_sites) == oracle.flags(exp, t["reg"].n_sites)).all()
    gr.close()


@pytest.mark.parametrize("seed", range(4))
def test_spill_edge_records(torch_cuda, seed):
    say("case: spilled table on edge records of a tiny registry with 3,000 sites, seed", seed)
    from tests.test_oracle_pins import _rate_records
    rng = np.random.default_rng(4400 + seed)
    n_sites, sites, local = random_tiny_registry(rng, n_sites=3000, n_prefixes=3000, n_local=2)
    recs = _rate_records(rng, 4000, sites, local)
    recs += [recs[int(i)] for i in rng.integers(0, len(recs), size=4000)]
    la, ll = [x[0] for x in local], [x[1] for x in local]
    args = ([x[0] for x in sites], [x[1] for x in sites], [x[2] for x in sites], n_sites, la, ll)
    reg, orc = gnm.Registry(*args), oracle.Registry(*args)
    assert not reg.info()["acc_in_lds"]
    cuts = sorted(int(c) for c in rng.integers(0, len(recs) + 1, size=3))
    off = np.array([0] + cuts + [len(recs)], dtype=np.uint64)
    bulk = int(rng.choice([0, 1_000_000]))
    rec = soa(recs)
    exp = orc.classify_aggregate(rec, bulk, window_offsets=off)
    for grid, rpt in ((0, 0), (3, 1), (50, 2)):
        _, got, fl = call(reg, rec, off, grid_blocks=grid, records_per_thread=rpt, bulk_bytes=bulk)
        assert (got == exp).all(), diff(got, exp)
        assert (fl == oracle.flags(exp, n_sites)).all()
