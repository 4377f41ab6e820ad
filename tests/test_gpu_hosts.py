"""GPU parity of the per-host statistics against the CPU oracle.  Slot
positions in the hash table depend on timing; the set of (key, statistics)
pairs does not, so the used slots are compared, sorted by key, bit for bit,
together with the slot count and the left-out flows."""
import ctypes
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


def run(reg, rec, capacity, off=None, table=None, accumulate=False, **kw):
    import torch
    nw = 1 if off is None else len(off) - 1
    t = table if table is not None else gnm.HostTable(capacity, device=DEV)
    if table is None:
        t.keys.fill_(123)
        t.stats.fill_(456)
        t.counters.fill_(789)
    acc = torch.empty((nw, reg.rows, 8), dtype=torch.int64, device=DEV)
    gnm.classify_aggregate(reg, to_device(rec), acc, window_offsets=None if off is None else offsets_to_device(off),
                           n_windows=nw, n=rec.n, hosts=t, accumulate=accumulate, **kw)
    torch.cuda.synchronize()
    return t, gnm.acc_to_numpy(acc)


def check(t, orc, rec, **kw):
    keys, st, used, dropped = t.to_numpy()
    ek, es = oracle.host_stats(orc, rec, **kw)
    assert dropped == 0 and used == keys.size
    assert keys.size == ek.size and (keys == ek).all()
    bad = np.argwhere(st != es)
    assert bad.size == 0, [(int(keys[i]), int(j), int(st[i, j]), int(es[i, j])) for i, j in bad[:5]]
    return keys.size


_S = {}


def _small():
    if not _S:
        r = flowgen.registry_for(flowgen.PLAIN_SMALL)
        _S.update(reg=r, orc=oracle.Registry.from_generated(r),
                  rec=flowgen.records_for(flowgen.PLAIN_SMALL, reg=r))
    return _S


@pytest.mark.parametrize("rpt,ws", [(0, True), (0, False), (1, True), (2, False)])
def test_hosts_plain_small(torch_cuda, rpt, ws):
    say("case: hosts plain-small, records_per_thread", rpt, "workspace", ws)
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    t, acc = run(reg, s["rec"], 1 << 16, records_per_thread=rpt, workspace=gnm.make_workspace(reg) if ws else None)
    assert (acc[0] == s["orc"].classify_aggregate(s["rec"])).all()
    assert check(t, s["orc"], s["rec"]) > 5_000


def test_hosts_with_histograms_and_filters(torch_cuda):
    say("case: hosts + histograms + filters")
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    f = {"min_avg_packet_bytes": 100, "min_packets": 1000}
    h = gnm.make_rate_hist(reg)
    t, acc = run(reg, s["rec"], 1 << 16, rate_hist=h, filters=f, workspace=gnm.make_workspace(reg))
    assert (acc[0] == s["orc"].classify_aggregate(s["rec"], filters=f)).all()
    assert (h.cpu().numpy().view(np.uint32) ==
            oracle.rate_histograms(s["orc"], s["rec"], filters=f)[:, :2 * reg.n_sites]).all()
    check(t, s["orc"], s["rec"], filters=f)


@pytest.mark.parametrize("seed", range(5))
def test_hosts_edge_records_windows_and_accumulate(torch_cuda, seed):
    say("case: hosts on edge records, seed", seed)
    from tests.test_oracle_pins import _rate_records
    rng = np.random.default_rng(2500 + seed)
    n_sites, sites, local = random_tiny_registry(rng, n_local=int(rng.integers(1, 4)))
    recs = _rate_records(rng, 3000, sites, local)
    recs += [recs[int(i)] for i in rng.integers(0, len(recs), size=3000)]
    la, ll = [x[0] for x in local], [x[1] for x in local]
    args = ([x[0] for x in sites], [x[1] for x in sites], [x[2] for x in sites], n_sites, la, ll)
    reg, orc = gnm.Registry(*args), oracle.Registry(*args)
    cuts = sorted(int(c) for c in rng.integers(0, len(recs) + 1, size=3))
    off = np.array([0] + cuts + [len(recs)], dtype=np.uint64)
    bulk = int(rng.choice([0, 1_000_000]))
    for grid in (0, 1, 37):
        t, _ = run(reg, soa(recs), 1 << 13, off=off, bulk_bytes=bulk, grid_blocks=grid)
        check(t, orc, soa(recs), bulk_bytes=bulk)  # the table covers every window
    # two calls accumulating into one table
    half = len(recs) // 2
    t, _ = run(reg, soa(recs[:half]), 1 << 13, bulk_bytes=bulk)
    run(reg, soa(recs[half:]), 1 << 13, table=t, accumulate=True, bulk_bytes=bulk)
    check(t, orc, soa(recs), bulk_bytes=bulk)


def test_hosts_table_overflow(torch_cuda):
    say("case: hosts table smaller than the hosts")
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    t, _ = run(reg, s["rec"], 1024)
    keys, st, used, dropped = t.to_numpy()
    ek, es = oracle.host_stats(s["orc"], s["rec"])
    assert used == keys.size and 900 < used <= 1024  # probing stops 256 slots from a key's hash position
    pos = np.searchsorted(ek, keys)
    assert (ek[pos] == keys).all() and (es[pos] == st).all()  # every recorded host is exact
    missing = np.setdiff1d(np.arange(ek.size), pos)
    assert dropped == int(es[missing, 0].sum())               # and the rest is counted as left out


def test_hosts_large_table(torch_cuda):
    say("case: hosts on the large-table registry, 1M records")
    r = flowgen.registry_for(flowgen.LARGE_TABLE)
    rec = flowgen.records_for(flowgen.LARGE_TABLE, reg=r, n=1_000_000, stream=21)
    orc = oracle.Registry.from_generated(r)
    reg = gnm.Registry.from_generated(r)
    t, acc = run(reg, rec, 1 << 20, workspace=gnm.make_workspace(reg))
    assert (acc[0] == orc.classify_aggregate(rec)).all()
    check(t, orc, rec)


def test_hosts_full_size(torch_cuda):
    say("case: hosts on the plain-large 10M window")
    r = flowgen.registry_for(flowgen.PLAIN_LARGE)
    rec = flowgen.records_for(flowgen.PLAIN_LARGE, reg=r)
    orc = oracle.Registry.from_generated(r)
    reg = gnm.Registry.from_generated(r)
    t, _ = run(reg, rec, 1 << 22, workspace=gnm.make_workspace(reg))
    assert check(t, orc, rec) > 400_000


def test_hosts_graph_replay(torch_cuda):
    import torch
    say("case: hosts through graph replays")
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    d = to_device(s["rec"])
    acc = torch.empty((1, reg.rows, 8), dtype=torch.int64, device=DEV)
    t = gnm.HostTable(1 << 16, device=DEV)
    g = gnm.Graph(reg, d, acc, n=s["rec"].n, hosts=t, workspace=gnm.make_workspace(reg))
    for _ in range(3):
        t.keys.fill_(7)
        t.counters.fill_(9)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        check(t, s["orc"], s["rec"])
    g.close()


def test_hosts_bad_capacity_rejected(torch_cuda):
    import torch
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    t = gnm.HostTable(1024, device=DEV)
    t.c.capacity = 1000  # not a power of two
    acc = torch.empty((1, reg.rows, 8), dtype=torch.int64, device=DEV)
    with pytest.raises(gnm.GnmError) as e:
        gnm.classify_aggregate(reg, to_device(s["rec"].slice(0, 100)), acc, n=100, hosts=t)
    assert e.value.code == -1
    with pytest.raises(ValueError):
        gnm.HostTable(1000, device=DEV)


def test_hosts_no_records(torch_cuda):
    import torch
    say("case: hosts with no records")
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    t = gnm.HostTable(256, device=DEV)
    t.keys.fill_(5)
    t.counters.fill_(9)
    acc = torch.empty((1, reg.rows, 8), dtype=torch.int64, device=DEV)
    empty = to_device(s["rec"].slice(0, 0))
    gnm.classify_aggregate(reg, empty, acc, n=0, hosts=t)
    torch.cuda.synchronize()
    keys, st, used, dropped = t.to_numpy()
    assert keys.size == 0 and used == 0 and dropped == 0
