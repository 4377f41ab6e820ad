"""Served form on the GPU: every window's tables and flags are the same alone
and in the mix, and equal to the oracle of that window."""
import threading
import time

import numpy as np
import pytest

import flowgen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    import paper_1108_1785_amd as gnm
    reg_h = flowgen.registry_for(flowgen.PLAIN_SMALL)
    reg = gnm.Registry.from_generated(reg_h)
    orc = oracle.Registry.from_generated(reg_h)
    pool = flowgen.records_for(flowgen.PLAIN_SMALL, reg=reg_h, n=400_000, stream=3)
    return reg_h, reg, orc, pool


def _windows(pool, sizes, seed):
    rng = np.random.default_rng(seed)
    out = []
    for n in sizes:
        lo = int(rng.integers(0, pool.n - n + 1))
        out.append(pool.slice(lo, lo + int(n)))
    return out


def _expect(orc, n_sites, w):
    acc = orc.classify_aggregate(w)
    return acc, oracle.flags(acc, n_sites)


def _server(reg, capacity, max_w, inflight=2):
    from paper_1108_1785_amd.serve import GpuExecutor, Server
    ex = GpuExecutor(reg, capacity=capacity, max_batch_windows=max_w, max_inflight=inflight)
    return Server(ex)


def test_served_alone_equals_mix_equals_oracle(small):
    from paper_1108_1785_amd.serve import pin_records
    reg_h, reg, orc, pool = small
    rng = np.random.default_rng(41)
    sizes = list(np.clip(flowgen.served_sizes(rng, 40, median=4_000, sigma=1.0, cap=60_000), 1, 60_000))
    sizes[5] = 0
    sizes[17] = 60_000
    wins = _windows(pool, sizes, 42)
    pinned = [pin_records(w) for w in wins]
    srv = _server(reg, capacity=250_000, max_w=16)
    try:
        # in the mix: submitted from two threads with short gaps, so arrivals
        # overlap copies and launches of earlier windows
        futs = [None] * len(wins)

        def worker(k):
            r = np.random.default_rng(100 + k)
            for i in range(k, len(wins), 2):
                futs[i] = srv.submit(pinned[i], n=wins[i].n)
                time.sleep(float(r.uniform(0, 0.002)))

        th = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        mix = [f.result(timeout=120) for f in futs]
        assert srv.stats["launches"] < len(wins), "continuous batching put several windows in a launch"
        # alone: one window at a time through the same server
        alone = {}
        for i in (0, 5, 17, 23, 39):
            alone[i] = srv.submit(pinned[i], n=wins[i].n).result(timeout=60)
    finally:
        srv.close()
    for i, (w, r) in enumerate(zip(wins, mix)):
        acc, fl = _expect(orc, reg_h.n_sites, w)
        assert (r.acc == acc).all(), "window %d (n=%d) differs from the oracle" % (i, w.n)
        assert (r.flags == fl).all(), "window %d flags differ" % i
        if i in alone:
            assert (alone[i].acc == r.acc).all() and (alone[i].flags == r.flags).all()


def test_served_back_pressure_tiny_arena(small):
    from paper_1108_1785_amd.serve import pin_records
    reg_h, reg, orc, pool = small
    sizes = [9_000, 12_000, 3_000, 15_000, 1, 14_999, 7_000, 8_000, 15_000, 2_500, 11_000, 6_000]
    wins = _windows(pool, sizes, 7)
    srv = _server(reg, capacity=16_000, max_w=4, inflight=2)
    try:
        futs = [srv.submit(pin_records(w), n=w.n) for w in wins]
        res = [f.result(timeout=120) for f in futs]
        assert srv.stats["admission_waits"] > 0
    finally:
        srv.close()
    for w, r in zip(wins, res):
        acc, fl = _expect(orc, reg_h.n_sites, w)
        assert (r.acc == acc).all() and (r.flags == fl).all()


def test_served_rejects_oversized_window(small):
    from paper_1108_1785_amd.serve import AdmissionError, pin_records
    reg_h, reg, orc, pool = small
    big, ok = _windows(pool, [20_001, 500], 9)
    srv = _server(reg, capacity=20_000, max_w=4)
    try:
        f_big = srv.submit(pin_records(big), n=big.n)
        f_ok = srv.submit(pin_records(ok), n=ok.n)
        with pytest.raises(AdmissionError):
            f_big.result(timeout=10)
        r = f_ok.result(timeout=60)
    finally:
        srv.close()
    acc, _ = _expect(orc, reg_h.n_sites, ok)
    assert (r.acc == acc).all()


def test_served_device_resident_records(small):
    """Windows already in device memory are staged device to device."""
    from tests._gpu import to_device
    reg_h, reg, orc, pool = small
    wins = _windows(pool, [30_000, 0, 777, 45_000], 13)
    srv = _server(reg, capacity=100_000, max_w=8)
    try:
        futs = [srv.submit(to_device(w), n=w.n) for w in wins]
        res = [f.result(timeout=60) for f in futs]
    finally:
        srv.close()
    for w, r in zip(wins, res):
        acc, fl = _expect(orc, reg_h.n_sites, w)
        assert (r.acc == acc).all() and (r.flags == fl).all()


def test_served_device_resident_burst_grouped_staging(small):
    """A burst of device-resident windows, empty ones among them, through an
    arena small enough to wrap and push back: windows admitted together are
    staged with one concatenating copy per field; each result still equals the
    oracle of its window."""
    from tests._gpu import to_device
    reg_h, reg, orc, pool = small
    rng = np.random.default_rng(21)
    sizes = [0 if rng.random() < 0.15 else int(rng.integers(1, 20_000)) for _ in range(60)]
    wins = _windows(pool, sizes, 22)
    dev = [to_device(w) for w in wins]
    srv = _server(reg, capacity=64_000, max_w=16, inflight=2)
    try:
        futs = [srv.submit(d, n=w.n) for d, w in zip(dev, wins)]
        res = [f.result(timeout=120) for f in futs]
        stats = dict(srv.stats)
    finally:
        srv.close()
    for w, r in zip(wins, res):
        acc, fl = _expect(orc, reg_h.n_sites, w)
        assert (r.acc == acc).all() and (r.flags == fl).all()
    assert stats["admission_waits"] > 0 and stats["launches"] < 60


def test_served_waits_for_the_producer_stream(small):
    """A window written on the caller's stream by queued device work and
    submitted without a synchronisation: the staging copy waits for that
    work (an event recorded at submit), so the result is the oracle's, not
    the buffers' stale contents."""
    import torch

    from tests._gpu import to_device
    reg_h, reg, orc, pool = small
    wins = _windows(pool, [40_000, 25_000, 0, 33_333], 17)
    src = [to_device(w) for w in wins]
    # the buffers the caller will submit start as garbage (another window)
    stale = _windows(pool, [w.n for w in wins], 18)
    bufs = [to_device(s) for s in stale]
    torch.cuda.synchronize()
    srv = _server(reg, capacity=150_000, max_w=8)
    side = torch.cuda.Stream()  # default priority
    try:
        futs = []
        with torch.cuda.stream(side):
            for b, s_, w in zip(bufs, src, wins):
                # a bounded spin, then the real records: both queued, nothing waited on
                torch.cuda._sleep(20_000_000)
                for f in b:
                    b[f].copy_(s_[f], non_blocking=True)
                futs.append(srv.submit(b, n=w.n))
        res = [f.result(timeout=60) for f in futs]
    finally:
        srv.close()
    for w, r in zip(wins, res):
        acc, fl = _expect(orc, reg_h.n_sites, w)
        assert (r.acc == acc).all() and (r.flags == fl).all()
