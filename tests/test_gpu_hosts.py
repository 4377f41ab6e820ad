"""GPU parity of the per-host statistics and medians against the CPU oracle.
The order of hosts in the table depends on timing; the set of (key,
statistics, median) does not, so the hosts are compared sorted by key, bit
for bit, together with the host count and the number of bulk flows of
registered sites.  Cases cover the launch shapes, several windows in one
call, histograms and filters in the same pass, a table too small for the
hosts, hot hosts (one partition holding most entries), partitions with more
hosts than one reduce batch holds, the large-table and full-size windows,
graph replays and the rejected arguments."""
import ctypes
import sys

import numpy as np
import pytest

import flowgen
import oracle
import paper_1108_1785_amd as gnm
from tests._gpu import DEV, offsets_to_device, to_device
from tests._helpers import ip, load_golden, random_tiny_registry, soa

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def run(reg, rec, capacity, off=None, table=None, grid_blocks=0, **kw):
    import torch
    nw = 1 if off is None else len(off) - 1
    t = table if table is not None else gnm.HostTable(reg, capacity, rec.n, grid_blocks, device=DEV)
    t.keys.fill_(123)
    t.stats.fill_(456)
    t.median.fill_(77)
    t.counters.fill_(789)
    acc = torch.empty((nw, reg.rows, 8), dtype=torch.int64, device=DEV)
    gnm.classify_aggregate(reg, to_device(rec), acc, window_offsets=None if off is None else offsets_to_device(off),
                           n_windows=nw, n=rec.n, hosts=t, grid_blocks=grid_blocks, **kw)
    torch.cuda.synchronize()
    return t, gnm.acc_to_numpy(acc)


def expected(orc, rec, **kw):
    ek, es = oracle.host_stats(orc, rec, **kw)
    mk, em = oracle.host_medians(orc, rec, **kw)
    assert (mk == ek).all()
    return ek, es, em


def check(t, orc, rec, **kw):
    keys, st, med, found, flows = t.to_numpy()
    ek, es, em = expected(orc, rec, **kw)
    assert found == ek.size == keys.size
    assert flows == int(es[:, 0].sum()) if ek.size else flows == 0
    assert (keys == ek).all()
    bad = np.argwhere(st != es)
    assert bad.size == 0, [(int(keys[i]), int(j), int(st[i, j]), int(es[i, j])) for i, j in bad[:5]]
    badm = np.flatnonzero(med != em)
    assert badm.size == 0, [(int(keys[i]), int(med[i]), int(em[i]), int(st[i, 0])) for i in badm[:5]]
    return keys.size


_S = {}


def _small():
    if not _S:
        r = flowgen.registry_for(flowgen.PLAIN_SMALL)
        _S.update(reg=r, orc=oracle.Registry.from_generated(r),
                  rec=flowgen.records_for(flowgen.PLAIN_SMALL, reg=r))
    return _S


def test_hosts_golden(torch_cuda):
    say("case: hosts on the hand-worked golden")
    g = load_golden("host_median_example.json")
    sites = [(ip(a), l, s) for a, l, s in g["sites"]]
    local = [(ip(a), l) for a, l in g["local"]]
    recs = soa([(ip(r[0]), ip(r[1]), r[2], r[3], r[4], r[5]) for r in g["records"]])
    reg = gnm.Registry([x[0] for x in sites], [x[1] for x in sites], [x[2] for x in sites], g["n_sites"],
                       [x[0] for x in local], [x[1] for x in local])
    t, _ = run(reg, recs, 16, bulk_bytes=g["bulk_bytes"])
    keys, st, med, found, flows = t.to_numpy()
    exp = sorted(((ip(a) << 32) | row, s, m) for a, row, s, m in g["expected_hosts"])
    assert found == len(exp) and flows == sum(e[1][0] for e in exp)
    assert keys.tolist() == [e[0] for e in exp]
    assert st.tolist() == [e[1] for e in exp]
    assert med.tolist() == [e[2] for e in exp]


@pytest.mark.parametrize("rpt,ws,grid", [(0, True, 0), (0, False, 0), (1, True, 0), (2, False, 0), (4, True, 3)])
def test_hosts_plain_small(torch_cuda, rpt, ws, grid):
    say("case: hosts plain-small, records_per_thread", rpt, "workspace", ws, "grid", grid)
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    t, acc = run(reg, s["rec"], 1 << 16, records_per_thread=rpt, grid_blocks=grid,
                 workspace=gnm.make_workspace(reg, grid) if ws else None)
    assert (acc[0] == s["orc"].classify_aggregate(s["rec"])).all()
    assert check(t, s["orc"], s["rec"]) > 5_000


def test_hosts_without_medians(torch_cuda):
    import torch
    say("case: hosts without the median array")
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    t = gnm.HostTable(reg, 1 << 16, s["rec"].n, device=DEV, medians=False)
    acc = torch.empty((1, reg.rows, 8), dtype=torch.int64, device=DEV)
    gnm.classify_aggregate(reg, to_device(s["rec"]), acc, n=s["rec"].n, hosts=t)
    torch.cuda.synchronize()
    keys, st, med, found, _ = t.to_numpy()
    ek, es, _ = expected(s["orc"], s["rec"])
    assert med is None and (keys == ek).all() and (st == es).all()


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
def test_hosts_edge_records_and_windows(torch_cuda, seed):
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


def test_hosts_table_too_small(torch_cuda):
    say("case: hosts table smaller than the hosts")
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    t, _ = run(reg, s["rec"], 1000)
    keys, st, med, found, flows = t.to_numpy()
    ek, es, em = expected(s["orc"], s["rec"])
    assert found == ek.size > 1000 and keys.size == 1000 and np.unique(keys).size == 1000
    pos = np.searchsorted(ek, keys)
    assert (ek[pos] == keys).all() and (es[pos] == st).all() and (em[pos] == med).all()  # each written host exact
    assert flows == int(es[:, 0].sum())


def _host_records(n, remote, rng, local=0x0A000000, rates="spread"):
    """n inbound bulk flows from the given remote addresses to a local /16."""
    dst = (local | rng.integers(0, 1 << 16, size=n)).astype(np.uint32)
    src = np.asarray(remote, dtype=np.uint32)
    b = rng.integers(1_000_001, 2_000_000_000, size=n).astype(np.uint64)
    dur = rng.integers(1, 300_000, size=n).astype(np.uint32)
    first = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    return flowgen.Records(src_ip=src, dst_ip=dst, src_port=np.zeros(n, np.uint16), dst_port=np.zeros(n, np.uint16),
                           proto=np.zeros(n, np.uint8), bytes=b, packets=np.full(n, 1000, np.uint32),
                           first_ms=first, last_ms=(first + dur).astype(np.uint32))


def test_hosts_hot_host_and_full_partitions(torch_cuda):
    say("case: one host with most flows; partitions with more hosts than a reduce batch")
    rng = np.random.default_rng(77)
    reg_args = ([0x0B000000, 0x0C000000], [8, 8], [0, 1], 2, [0x0A000000], [16])
    reg, orc = gnm.Registry(*reg_args), oracle.Registry(*reg_args)
    # 150,000 flows of one host in 11.0.0.0/8, 50,000 of a few others
    remote = np.where(rng.random(200_000) < 0.75, 0x0B000001, 0x0B000000 | rng.integers(2, 40, size=200_000))
    rec = _host_records(200_000, remote, rng)
    t, _ = run(reg, rec, 64)
    keys, st, med, found, flows = t.to_numpy()
    assert st[keys == ((0x0B000001 << 32) | 0)][0, 0] > 140_000
    check(t, orc, rec)
    # 120,000 distinct hosts in 64 partitions: about 1,900 hosts per partition, several batches each
    remote = (0x0C000000 | rng.permutation(1 << 20)[:120_000]).astype(np.uint32)
    rec = _host_records(120_000, remote, rng)
    t, _ = run(reg, rec, 1 << 17)
    assert check(t, orc, rec) == 120_000


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
    t, _ = run(reg, rec, 1 << 20, workspace=gnm.make_workspace(reg))
    assert check(t, orc, rec) > 400_000


def test_hosts_graph_replay(torch_cuda):
    import torch
    say("case: hosts through graph replays")
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    d = to_device(s["rec"])
    acc = torch.empty((1, reg.rows, 8), dtype=torch.int64, device=DEV)
    t = gnm.HostTable(reg, 1 << 16, s["rec"].n, device=DEV)
    g = gnm.Graph(reg, d, acc, n=s["rec"].n, hosts=t, workspace=gnm.make_workspace(reg))
    for _ in range(3):
        t.keys.fill_(7)
        t.median.fill_(3)
        t.counters.fill_(9)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        check(t, s["orc"], s["rec"])
    g.close()


def test_hosts_bad_arguments_rejected(torch_cuda):
    import torch
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    acc = torch.empty((1, reg.rows, 8), dtype=torch.int64, device=DEV)
    d = to_device(s["rec"].slice(0, 1000))
    t = gnm.HostTable(reg, 1024, 1000, 4, device=DEV)
    for change in ("work_bytes", "work_align", "accumulate", "counters"):
        saved = (t.c.work_bytes, t.c.work, t.c.counters)
        if change == "work_bytes":
            t.c.work_bytes = gnm.host_work_bytes(reg, 1000, 4) - 1
        elif change == "work_align":
            t.c.work = t.c.work + 8
        elif change == "counters":
            t.c.counters = 0
        with pytest.raises(gnm.GnmError) as e:
            gnm.classify_aggregate(reg, d, acc, n=1000, hosts=t, grid_blocks=4, accumulate=change == "accumulate")
        assert e.value.code == gnm.GNM_E_INVAL
        t.c.work_bytes, t.c.work, t.c.counters = saved
    # a table sized for fewer records is refused for more
    with pytest.raises(gnm.GnmError):
        gnm.classify_aggregate(reg, to_device(s["rec"].slice(0, 100_000)), acc, n=100_000, hosts=t)


def test_hosts_no_records(torch_cuda):
    import torch
    say("case: hosts with no records")
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    t = gnm.HostTable(reg, 256, 0, device=DEV)
    t.keys.fill_(5)
    t.counters.fill_(9)
    acc = torch.empty((1, reg.rows, 8), dtype=torch.int64, device=DEV)
    empty = to_device(s["rec"].slice(0, 0))
    gnm.classify_aggregate(reg, empty, acc, n=0, hosts=t)
    torch.cuda.synchronize()
    keys, st, med, found, flows = t.to_numpy()
    assert keys.size == 0 and found == 0 and flows == 0
