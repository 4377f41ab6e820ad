"""GPU parity of the exclusion filters (reverse-ACK average packet size,
administrative packet count and duration) against the CPU oracle: every field
of every row, and the histograms, medians and flags they feed, bit for bit."""
import sys

import numpy as np
import pytest

import flowgen
import oracle
import paper_1108_1785_amd as gnm
from tests._gpu import DEV, diff, offsets_to_device, to_device
from tests._helpers import random_tiny_registry, soa

pytestmark = pytest.mark.gpu

FILTER_SETS = [
    {"min_avg_packet_bytes": 100},
    {"min_packets": 1000},
    {"min_duration_ms": 5000},
    {"min_avg_packet_bytes": 100, "min_packets": 1000, "min_duration_ms": 5000},
    {"min_avg_packet_bytes": 2**32 - 1},
]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def run(reg, rec, off=None, filters=None, bulk_bytes=1_000_000, grid_blocks=0, records_per_thread=0,
        workspace=True, hist=False):
    import torch
    nw = 1 if off is None else len(off) - 1
    acc = torch.empty((nw, reg.rows, 8), dtype=torch.int64, device=DEV)
    h = gnm.make_rate_hist(reg, nw) if hist else None
    gnm.classify_aggregate(reg, to_device(rec), acc, window_offsets=None if off is None else offsets_to_device(off),
                           n_windows=nw, bulk_bytes=bulk_bytes, grid_blocks=grid_blocks,
                           records_per_thread=records_per_thread, n=rec.n,
                           workspace=gnm.make_workspace(reg, grid_blocks) if workspace else None,
                           rate_hist=h, filters=filters)
    torch.cuda.synchronize()
    out = gnm.acc_to_numpy(acc)
    return (out, h.cpu().numpy().view(np.uint32)) if hist else out


_S = {}


def _small():
    if not _S:
        r = flowgen.registry_for(flowgen.PLAIN_SMALL)
        _S.update(reg=r, orc=oracle.Registry.from_generated(r),
                  rec=flowgen.records_for(flowgen.PLAIN_SMALL, reg=r))
    return _S


@pytest.mark.parametrize("fi", range(len(FILTER_SETS)))
def test_filters_plain_small(torch_cuda, fi):
    f = FILTER_SETS[fi]
    say("case: filters plain-small", f)
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    exp = s["orc"].classify_aggregate(s["rec"], filters=f)
    base = s["orc"].classify_aggregate(s["rec"])
    assert exp[:, 4].sum() < base[:, 4].sum()  # the filter removes flows here
    for rpt, ws in ((0, True), (1, False), (2, True)):
        got = run(reg, s["rec"], filters=f, records_per_thread=rpt, workspace=ws)[0]
        assert (got == exp).all(), (rpt, ws, diff(got, exp))
    got, h = run(reg, s["rec"], filters=f, hist=True)
    assert (got[0] == exp).all()
    S2 = 2 * s["reg"].n_sites
    assert (h == oracle.rate_histograms(s["orc"], s["rec"], filters=f)[:, :S2]).all()


@pytest.mark.parametrize("seed", range(6))
def test_filters_edge_records(torch_cuda, seed):
    say("case: filters on edge records, seed", seed)
    from tests.test_oracle_pins import _edge_records, _random_filters
    rng = np.random.default_rng(1700 + seed)
    n_sites, sites, local = random_tiny_registry(rng, n_local=int(rng.integers(1, 4)))
    recs = _edge_records(rng, 4000, sites, local)
    recs = [(a, d, b, int(rng.choice([0, 1, 2, 10, b // 64 + 1, b // 1500 + 1, 2**32 - 1])) & 0xFFFFFFFF, f, l)
            for a, d, b, _p, f, l in recs]
    la, ll = [x[0] for x in local], [x[1] for x in local]
    args = ([x[0] for x in sites], [x[1] for x in sites], [x[2] for x in sites], n_sites, la, ll)
    reg, orc = gnm.Registry(*args), oracle.Registry(*args)
    cuts = sorted(int(c) for c in rng.integers(0, len(recs) + 1, size=4))
    off = np.array([0] + cuts + [len(recs)], dtype=np.uint64)
    bulk = int(rng.choice([0, 1_000_000]))
    for _ in range(3):
        f = _random_filters(rng)
        exp = orc.classify_aggregate(soa(recs), bulk, window_offsets=off, filters=f)
        for grid in (0, 1, 37):
            got = run(reg, soa(recs), off, filters=f, bulk_bytes=bulk, grid_blocks=grid, workspace=grid != 37)
            assert (got == exp).all(), (f, grid, diff(got, exp))


def test_filters_large_table_batched(torch_cuda):
    say("case: filters on the large-table registry, 1.5M records in 3 windows")
    r = flowgen.registry_for(flowgen.LARGE_TABLE)
    rec = flowgen.records_for(flowgen.LARGE_TABLE, reg=r, n=1_500_000, stream=11)
    orc = oracle.Registry.from_generated(r)
    reg = gnm.Registry.from_generated(r)
    off = np.array([0, 500_000, 500_001, 1_500_000], dtype=np.uint64)
    f = FILTER_SETS[3]
    exp = orc.classify_aggregate(rec, window_offsets=off, filters=f)
    got = run(reg, rec, off, filters=f)
    assert (got == exp).all(), diff(got, exp)


def test_filters_median_and_graph(torch_cuda):
    import torch
    say("case: filters with histograms, medians and a graph replay")
    s = _small()
    r, orc = s["reg"], s["orc"]
    reg = gnm.Registry.from_generated(r)
    f = FILTER_SETS[0]
    d = to_device(s["rec"])
    acc = torch.empty((1, reg.rows, 8), dtype=torch.int64, device=DEV)
    hist = gnm.make_rate_hist(reg)
    g = gnm.Graph(reg, d, acc, n=s["rec"].n, rate_hist=hist, filters=f, workspace=gnm.make_workspace(reg))
    exp = orc.classify_aggregate(s["rec"], filters=f)
    med, cnt = oracle.rate_medians(orc, s["rec"], filters=f)
    fexp = oracle.median_flags(med, cnt, r.n_sites)
    for _ in range(3):
        acc.fill_(5)
        hist.fill_(9)
        torch.cuda.synchronize()
        g.launch()
        flg = torch.empty(r.n_sites, dtype=torch.uint8, device=DEV)
        mb = torch.empty(2 * r.n_sites, dtype=torch.int32, device=DEV)
        gnm.median_flags(reg, hist, 1, flg, median_bucket=mb)
        torch.cuda.synchronize()
        assert (gnm.acc_to_numpy(acc)[0] == exp).all()
        assert (mb.cpu().numpy().view(np.uint32) == med[0, :2 * r.n_sites]).all()
        assert (flg.cpu().numpy() == fexp[0]).all()
    g.close()
