"""GPU parity of the mid-launch table flush.

A classify workgroup aggregates its slice in an LDS table whose count word
packs flows (low 32 bits) and bulk flows (high 32 bits), so it flushes the
table to the window's device table with device-scope atomics at least every
2^31 records, as it does at every window change.  The launch parameter
flush_records lowers that limit so the flush runs on small inputs: every
case is compared bit for bit with the oracle, with one window and many, with
and without a workspace (one window with a workspace then adds its final
tables into an initialised table instead of overwriting it), on the
large-table registry (whose rows sit behind an LDS cache) and when
accumulating over two calls.
"""
import sys

import numpy as np
import pytest

import flowgen
import oracle
import paper_1108_1785_amd as gnm
from tests._gpu import diff, run

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


_CACHE = {}


def _workload(name, n):
    key = (name, n)
    if key not in _CACHE:
        r = flowgen.registry_for(name)
        _CACHE[key] = (r, oracle.Registry.from_generated(r), flowgen.records_for(name, reg=r, n=n))
    return _CACHE[key]


@pytest.mark.parametrize("flush", [1000, 3001, 4096])
@pytest.mark.parametrize("rpt", [0, 1])
@pytest.mark.parametrize("ws", [False, True])
def test_flush_one_window(flush, rpt, ws):
    say("case: plain-small 100k, one window, flush_records", flush, "rpt", rpt, "workspace", ws)
    r, orc, rec = _workload(flowgen.PLAIN_SMALL, None)
    reg = gnm.Registry.from_generated(r)
    exp = orc.classify_aggregate(rec)
    got = run(reg, rec, records_per_thread=rpt, workspace=gnm.make_workspace(reg) if ws else None,
              flush_records=flush)
    assert (got == exp).all(), diff(got, exp)


@pytest.mark.parametrize("grid", [0, 7])
@pytest.mark.parametrize("ws", [False, True])
def test_flush_many_windows(grid, ws):
    say("case: 37 uneven windows, flush_records 2500, grid", grid, "workspace", ws)
    r, orc, rec = _workload(flowgen.PLAIN_SMALL, None)
    rng = np.random.default_rng(31)
    cuts = np.sort(rng.integers(0, rec.n, size=36))
    off = np.concatenate([[0], cuts, [rec.n]]).astype(np.uint64)
    reg = gnm.Registry.from_generated(r)
    got = run(reg, rec, window_offsets=off, grid_blocks=grid,
              workspace=gnm.make_workspace(reg, grid) if ws else None, flush_records=2500)
    for w in range(len(off) - 1):
        exp = orc.classify_aggregate(rec.slice(int(off[w]), int(off[w + 1])))
        assert (got[w] == exp).all(), (w, diff(got[w], exp))


def test_flush_large_table_cache():
    say("case: large-table registry, 3 windows of 100k, flush_records 5000")
    r, orc, rec = _workload(flowgen.LARGE_TABLE, 300_000)
    reg = gnm.Registry.from_generated(r)
    assert reg.info()["acc_in_lds"] == 0
    off = np.array([0, 100_000, 200_000, 300_000], dtype=np.uint64)
    got = run(reg, rec, window_offsets=off, workspace=gnm.make_workspace(reg), flush_records=5000)
    for w in range(3):
        exp = orc.classify_aggregate(rec.slice(int(off[w]), int(off[w + 1])))
        assert (got[w] == exp).all(), (w, diff(got[w], exp))


def test_flush_accumulate_two_calls():
    import torch
    say("case: accumulate over two calls with flush_records 1500")
    r, orc, rec = _workload(flowgen.PLAIN_SMALL, None)
    reg = gnm.Registry.from_generated(r)
    a, b = rec.slice(0, 60_000), rec.slice(60_000, rec.n)
    acc = torch.empty((1, reg.rows, 8), dtype=torch.int64, device="cuda:0")
    ws = gnm.make_workspace(reg)
    run(reg, a, acc=acc, workspace=ws, flush_records=1500)
    got = run(reg, b, acc=acc, accumulate=True, workspace=ws, flush_records=1500)
    exp = orc.classify_aggregate(rec)
    assert (got == exp).all(), diff(got, exp)


def test_flush_records_clamped_and_checked():
    say("case: flush_records above 2^31 is clamped; beyond 32 bits is refused")
    r, orc, rec = _workload(flowgen.PLAIN_SMALL, None)
    reg = gnm.Registry.from_generated(r)
    small = rec.slice(0, 20_000)
    got = run(reg, small, workspace=gnm.make_workspace(reg), flush_records=(1 << 32) - 1)
    exp = orc.classify_aggregate(small)
    assert (got == exp).all(), diff(got, exp)
    with pytest.raises(ValueError):
        gnm.make_params(flush_records=1 << 32)
