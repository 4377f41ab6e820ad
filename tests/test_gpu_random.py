"""Seeded random sweep of the classify pass with its options combined: random
tiny registries (nesting, /0 and /32), edge-case records, random window cuts
and launch shapes, with histograms, a host table and the exclusion filters
switched on at random, sometimes over two accumulating calls.  Every table,
histogram and host entry is compared with the oracle bit for bit."""
import sys

import numpy as np
import pytest

import oracle
import paper_1108_1785_amd as gnm
from tests._gpu import DEV, diff, offsets_to_device, to_device
from tests._helpers import random_tiny_registry, soa

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("seed", range(24))
def test_random_option_combinations(seed):
    import torch
    from tests.test_oracle_pins import _random_filters, _rate_records
    rng = np.random.default_rng(5000 + seed)
    n_sites, sites, local = random_tiny_registry(rng, n_local=int(rng.integers(0, 4)))
    recs = _rate_records(rng, int(rng.integers(0, 6000)), sites, local)
    if recs and rng.random() < 0.5:
        recs += [recs[int(i)] for i in rng.integers(0, len(recs), size=len(recs))]
    recs = [(a, d, b, int(rng.choice([p, 0, 1, b // 1500 + 1])) & 0xFFFFFFFF, f, l) for a, d, b, p, f, l in recs]
    n = len(recs)
    cuts = sorted(int(c) for c in rng.integers(0, n + 1, size=int(rng.integers(0, 6))))
    off = np.array([0] + cuts + [n], dtype=np.uint64)
    nw = len(off) - 1
    bulk = int(rng.choice([0, 1_000_000, 5_000_000]))
    filters = _random_filters(rng) if rng.random() < 0.4 else None
    use_hist, use_hosts = rng.random() < 0.6, rng.random() < 0.5
    accumulate = n > 1 and rng.random() < 0.3 and not use_hosts  # a host table covers one call
    rpt = int(rng.choice([0, 1, 2, 4]))
    grid = int(rng.choice([0, 1, 7, 300]))
    ws = rng.random() < 0.6
    layout = str(rng.choice(["auto", "wide", "lines"]))
    say("case: seed", seed, "records", n, "windows", nw, "bulk", bulk, "filters", filters, "hist", use_hist,
        "hosts", use_hosts, "accumulate", accumulate, "rpt", rpt, "grid", grid, "ws", ws, "layout", layout)
    la, ll = [x[0] for x in local], [x[1] for x in local]
    args = ([x[0] for x in sites], [x[1] for x in sites], [x[2] for x in sites], n_sites, la, ll)
    kw = {} if layout == "auto" else {"layout": layout}
    reg, orc = gnm.Registry(*args, **kw), oracle.Registry(*args)
    rec = soa(recs)
    acc = torch.empty((nw, reg.rows, 8), dtype=torch.int64, device=DEV)
    hist = gnm.make_rate_hist(reg, nw) if use_hist else None
    hosts = gnm.HostTable(reg, 1 << 14, n, grid, device=DEV) if use_hosts else None
    call = dict(window_offsets=offsets_to_device(off), n_windows=nw, bulk_bytes=bulk, records_per_thread=rpt,
                grid_blocks=grid, workspace=gnm.make_workspace(reg, grid) if ws else None, rate_hist=hist,
                hosts=hosts, filters=filters)
    if accumulate:
        # first call over the records of the first half of each window, then the rest
        mid = np.array([(int(off[w]) + int(off[w + 1])) // 2 for w in range(nw)], dtype=np.uint64)
        first = np.concatenate([np.arange(int(off[w]), int(mid[w])) for w in range(nw)]).astype(np.int64)
        second = np.concatenate([np.arange(int(mid[w]), int(off[w + 1])) for w in range(nw)]).astype(np.int64)
        off1 = np.concatenate([[0], np.cumsum(mid - off[:-1])]).astype(np.uint64)
        off2 = np.concatenate([[0], np.cumsum(off[1:] - mid)]).astype(np.uint64)
        for idx, o, accum in ((first, off1, False), (second, off2, True)):
            part = soa([recs[i] for i in idx])
            c = dict(call, window_offsets=offsets_to_device(o), accumulate=accum)
            gnm.classify_aggregate(reg, to_device(part), acc, n=part.n, **c)
    else:
        gnm.classify_aggregate(reg, to_device(rec), acc, n=n, **call)
    torch.cuda.synchronize()
    exp = orc.classify_aggregate(rec, bulk, window_offsets=off, filters=filters)
    got = gnm.acc_to_numpy(acc)
    assert (got == exp).all(), diff(got, exp)
    if use_hist:
        eh = oracle.rate_histograms(orc, rec, window_offsets=off, bulk_bytes=bulk, filters=filters)
        assert (hist.cpu().numpy().view(np.uint32) == eh[:, :2 * n_sites]).all()
    if use_hosts:
        keys, st, med, found, _ = hosts.to_numpy()
        ek, es = oracle.host_stats(orc, rec, bulk, filters)
        _, em = oracle.host_medians(orc, rec, bulk, filters)
        assert found == keys.size == ek.size
        assert (keys == ek).all() and (st == es).all() and (med == em).all()
