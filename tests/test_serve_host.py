"""Scheduler of the served form on the CPU, with an executor that computes
with the oracle.

The fake executor writes a window's records into its arena at the earliest
moment a device copy could (start_copy) and reads the arena only when a launch
is reported finished (the latest moment a device launch could still read).
Any arena region handed out while still in use therefore corrupts a result
and fails the comparison with the oracle of that window alone.
"""
import threading
import time

import numpy as np
import pytest

import flowgen
import oracle
from paper_1108_1785_amd.serve import RECORD_FIELDS, AdmissionError, RingArena, Server


class _Ev:
    def __init__(self, ticks):
        self.ticks = ticks


class FakeExecutor:
    def __init__(self, orc, n_sites, capacity, max_w=64, slots=2, copy_ticks=2, run_ticks=3):
        self.orc, self.n_sites = orc, n_sites
        self.capacity, self.max_w = capacity, max_w
        self.arena = {f: np.zeros(capacity, dtype=np.uint64 if f == "bytes" else np.uint32)
                      for f in RECORD_FIELDS}
        self.slots = [None] * slots
        self.copy_ticks, self.run_ticks = copy_ticks, run_ticks
        self.batches = []
        self.max_inflight_seen = 0
        self.lock = threading.Lock()

    def start_copy(self, req):
        if req.n == 0:
            return None
        assert 0 <= req.offset and req.offset + req.n <= self.capacity
        for f in RECORD_FIELDS:
            self.arena[f][req.offset:req.offset + req.n] = req.records[f]
        return _Ev(self.copy_ticks)

    def done(self, ev):
        if ev is None:
            return True
        if ev.ticks > 0:
            ev.ticks -= 1
        return ev.ticks == 0

    def free_slot(self):
        for i, s in enumerate(self.slots):
            if s is None:
                return i
        return None

    def launch(self, slot, batch):
        assert len(batch) <= self.max_w
        for a, b in zip(batch, batch[1:]):
            assert b.offset == a.offset + a.n, "a launch covers consecutive arena windows"
        self.slots[slot] = [batch, self.run_ticks]
        self.batches.append([r.rid for r in batch])
        self.max_inflight_seen = max(self.max_inflight_seen, sum(s is not None for s in self.slots))

    def poll(self, slot):
        s = self.slots[slot]
        if s[1] > 0:
            s[1] -= 1
            return None
        batch = s[0]
        base = batch[0].offset
        total = batch[-1].offset + batch[-1].n - base
        rec = flowgen.Records(*(self.arena[f][base:base + total] if f in RECORD_FIELDS
                                else np.zeros(total, dtype=np.uint16 if f != "proto" else np.uint8)
                                for f in flowgen.Records.FIELDS))
        off = np.zeros(len(batch) + 1, dtype=np.uint64)
        np.cumsum([r.n for r in batch], out=off[1:])
        acc = self.orc.classify_aggregate(rec, window_offsets=off, threads=1)
        fl = oracle.flags(acc, self.n_sites)
        self.slots[slot] = None
        return acc, fl


@pytest.fixture(scope="module")
def setup():
    reg = flowgen.registry_for(flowgen.PLAIN_SMALL)
    orc = oracle.Registry.from_generated(reg)
    rec = flowgen.records_for(flowgen.PLAIN_SMALL, reg=reg, n=60_000)
    return reg, orc, rec


def _windows(rec, sizes):
    out, lo = [], 0
    for n in sizes:
        out.append(rec.slice(lo, lo + n))
        lo += n
    return out


def _as_dict(w):
    return {f: getattr(w, f) for f in RECORD_FIELDS}


def _alone(orc, n_sites, w):
    acc = orc.classify_aggregate(w, threads=1)
    return acc, oracle.flags(acc, n_sites)


def test_ring_arena_fifo_wrap():
    a = RingArena(10)
    assert a.alloc(4) == 0 and a.alloc(4) == 4
    assert a.alloc(3) is None          # 2 free at the end, 0 at the front
    a.free_oldest()
    assert a.alloc(3) == 0             # wraps to the front
    assert a.alloc(1) == 3 and a.alloc(1) is None
    a.free_oldest()                    # frees [4, 8)
    assert a.alloc(2) == 4 and a.used == 3 + 1 + 2
    with pytest.raises(AdmissionError):
        a.alloc(11)
    with pytest.raises(ValueError):
        a.alloc(0)


def test_ring_arena_random_never_overlaps():
    rng = np.random.default_rng(7)
    cap = 1000
    a = RingArena(cap)
    for _ in range(5000):
        if a.live and rng.random() < 0.45:
            a.free_oldest()
        else:
            n = int(rng.integers(1, 300))
            off = a.alloc(n)
            if off is None:
                continue
        occ = np.zeros(cap, dtype=np.int32)
        for o, n in a.live:
            assert 0 <= o and o + n <= cap
            occ[o:o + n] += 1
        assert occ.max(initial=0) <= 1


@pytest.mark.parametrize("capacity,slots,max_w", [(60_000, 2, 64), (9_000, 2, 3), (5_000, 1, 1)])
def test_served_windows_match_alone(setup, capacity, slots, max_w):
    reg, orc, rec = setup
    rng = np.random.default_rng(capacity)
    sizes = [int(x) for x in rng.integers(0, 4_000, size=14)] + [0, 4_999, 1]
    wins = _windows(rec, sizes)
    ex = FakeExecutor(orc, reg.n_sites, capacity, max_w=max_w, slots=slots)
    srv = Server(ex)
    futs = [srv.submit(_as_dict(w), n=w.n) for w in wins]
    res = [f.result(timeout=60) for f in futs]
    srv.close()
    for w, r in zip(wins, res):
        acc, fl = _alone(orc, reg.n_sites, w)
        assert (r.acc == acc).all()
        assert (r.flags == fl).all()
        assert r.n_records == w.n and r.latency_s >= 0
    # every window launched exactly once, in submission order
    order = [rid for b in ex.batches for rid in b]
    assert order == list(range(len(wins)))
    assert max(len(b) for b in ex.batches) <= max_w
    assert ex.max_inflight_seen <= slots
    if capacity == 60_000 and max_w == 64:
        assert any(len(b) > 1 for b in ex.batches), "continuous batching groups ready windows"
    if capacity < sum(sizes):
        assert srv.stats["admission_waits"] > 0, "a small arena makes windows wait"


def test_oversized_window_rejected_others_served(setup):
    reg, orc, rec = setup
    wins = _windows(rec, [1_000, 3_000, 500])
    ex = FakeExecutor(orc, reg.n_sites, 2_000)
    srv = Server(ex)
    futs = [srv.submit(_as_dict(w), n=w.n) for w in wins]
    with pytest.raises(AdmissionError):
        futs[1].result(timeout=10)
    for i in (0, 2):
        acc, _ = _alone(orc, reg.n_sites, wins[i])
        assert (futs[i].result(timeout=30).acc == acc).all()
    srv.close()


def test_executor_failure_fails_pending(setup):
    reg, orc, rec = setup

    class Broken(FakeExecutor):
        def launch(self, slot, batch):
            raise RuntimeError("launch failed")

    ex = Broken(orc, reg.n_sites, 10_000)
    srv = Server(ex)
    futs = [srv.submit(_as_dict(w), n=w.n) for w in _windows(rec, [100, 200])]
    for f in futs:
        with pytest.raises(RuntimeError, match="launch failed"):
            f.result(timeout=10)
    srv.close()


def test_interleaved_submitters(setup):
    """Windows from several threads: each result equals that window alone."""
    reg, orc, rec = setup
    wins = _windows(rec, [700 + 37 * i for i in range(24)])
    ex = FakeExecutor(orc, reg.n_sites, 6_000, max_w=8)
    srv = Server(ex)
    futs = [None] * len(wins)

    def worker(k):
        for i in range(k, len(wins), 3):
            futs[i] = srv.submit(_as_dict(wins[i]), n=wins[i].n)
            time.sleep(0.001)

    th = [threading.Thread(target=worker, args=(k,)) for k in range(3)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for w, f in zip(wins, futs):
        acc, fl = _alone(orc, reg.n_sites, w)
        r = f.result(timeout=60)
        assert (r.acc == acc).all() and (r.flags == fl).all()
    srv.close()
