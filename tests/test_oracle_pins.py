"""Pins of the CPU oracle against facts independent of it (CPU only).

The oracle is trusted only after these pass: the hand-derived worked example,
the paper's decimal-unit arithmetic, closed forms of the integer rate,
brute-force longest-prefix match at every interval boundary, brute-force
aggregation of random small windows full of edge cases, and conservation /
permutation / split-merge invariants on generated windows.
"""
import statistics

import numpy as np
import pytest

import flowgen
import oracle
from oracle import brute
from tests._helpers import (M64, boundary_points, ip, load_golden, random_tiny_registry, soa,
                            tuples, worked_example)


def _oracle_reg(sites, local, n_sites):
    a = np.array([s[0] for s in sites], dtype=np.uint32)
    l = np.array([s[1] for s in sites], dtype=np.uint32)
    s = np.array([s[2] for s in sites], dtype=np.uint32)
    la = np.array([x[0] for x in local], dtype=np.uint32)
    ll = np.array([x[1] for x in local], dtype=np.uint32)
    return oracle.Registry(a, l, s, n_sites, la, ll)


# ---------------------------------------------------------------- worked example

def test_worked_example_brute():
    sites, local, S, recs, exp, g = worked_example()
    rows = brute.classify_aggregate(sites, local, S, recs, g["bulk_bytes"])
    assert rows == exp
    assert [sum(r[k] for r in rows) for k in range(6)] == g["expected_column_totals"]
    assert brute.flags(rows, S, g["threshold_bps"], 0) == g["expected_flags"]


def test_worked_example_c_oracle():
    sites, local, S, recs, exp, g = worked_example()
    reg = _oracle_reg(sites, local, S)
    rows = reg.classify_aggregate(soa(recs), g["bulk_bytes"])
    assert rows.tolist() == exp
    assert oracle.flags(rows, S, g["threshold_bps"]).tolist() == g["expected_flags"]
    for a, site in g["lpm_spot_checks"]:
        assert int(reg.lookup([ip(a)])[0]) == site


def test_worked_example_strict_threshold():
    # Dropping r8 leaves site 1 outbound with mean exactly 1,000,000: not flagged.
    sites, local, S, recs, exp, g = worked_example()
    reg = _oracle_reg(sites, local, S)
    rows = reg.classify_aggregate(soa(recs[:8] + recs[9:]), g["bulk_bytes"])
    assert int(rows[3, 5]) // int(rows[3, 4]) == 1_000_000
    assert oracle.flags(rows, S, g["threshold_bps"]).tolist() == [0, 0, 0]
    # a minimum bulk-flow count above what the row holds suppresses the flag
    rows = reg.classify_aggregate(soa(recs), g["bulk_bytes"])
    assert oracle.flags(rows, S, g["threshold_bps"], min_bulk_flows=3).tolist() == [0, 0, 0]
    assert oracle.flags(rows, S, g["threshold_bps"], min_bulk_flows=2).tolist() == [0, 2, 0]


def test_worked_example_threads_and_order():
    sites, local, S, recs, exp, g = worked_example()
    reg = _oracle_reg(sites, local, S)
    for threads in (1, 3, 8):
        assert reg.classify_aggregate(soa(recs[::-1]), g["bulk_bytes"], threads=threads).tolist() == exp


# ---------------------------------------------------------------- units and rate

def test_paper_decimal_units():
    u = load_golden("paper_units.json")
    dgrams = u["records_per_hour"] / 3600 / u["records_per_datagram"]
    assert round(dgrams) == u["printed_datagrams_per_s"]
    bps = u["printed_datagrams_per_s"] * u["datagram_bytes"] * 8
    assert round(bps / 1e6, 2) == u["printed_mbps"]
    c = u["rate_case"]
    assert int(oracle.rate_bps([c["bytes"]], [c["duration_ms"]])[0]) == c["rate_bps"] == bps
    assert brute.rate_bps(c["bytes"], c["duration_ms"]) == c["rate_bps"]


RATE_TABLE = [
    # (bytes, dur_ms, expected) — closed forms worked by hand
    (1 << 40, 1, 8_796_093_022_208_000),          # 2^40 * 8000
    (1_000_003, 3, 2_666_674_666),                 # 8,000,024,000 / 3 = ...666.67
    (1_000_000, 8000, 1_000_000),                  # exact 1 Mbps
    (1, 8000, 1),                                  # one byte over 8 s = 1 bit/s
    (1, 8001, 0),                                  # just under 1 bit/s
    (1 << 63, 1, M64),                             # 2^63 * 8000 > 2^64: saturates
    (M64, 0xFFFFFFFF, 34_359_738_376_000),         # (2^64-1)/(2^32-1) = 2^32+1, times 8000
    (0xFFFFFFFF, 0xFFFFFFFF, 8000),
]


@pytest.mark.parametrize("b,d,exp", RATE_TABLE)
def test_rate_closed_forms(b, d, exp):
    assert int(oracle.rate_bps([b], [d])[0]) == exp
    assert brute.rate_bps(b, d) == exp


def test_rate_floor_characterisation():
    # rate is the unique integer q with q*d <= 8000*b < (q+1)*d (unless saturated)
    rng = np.random.default_rng(7)
    b = rng.integers(0, 1 << 63, size=4000, dtype=np.uint64) >> rng.integers(0, 63, size=4000).astype(np.uint64)
    d = rng.integers(1, 1 << 32, size=4000, dtype=np.uint64).astype(np.uint32)
    d[::7] = 1
    d[1::7] = 3
    r = oracle.rate_bps(b, d)
    for bi, di, ri in zip(b.tolist(), d.tolist(), r.tolist()):
        if ri == M64:
            assert 8000 * bi >= M64 * di
        else:
            assert ri * di <= 8000 * bi < (ri + 1) * di


def test_rate_near_integer_quotients():
    # 8000*b = k*d - 1 just below an integer: a floating-point floor of the
    # rounded quotient would return k; the exact answer is k-1.
    rng = np.random.default_rng(11)
    cases = []
    while len(cases) < 2000:
        d = int(rng.integers(2, 1 << 32))
        if d % 2 == 0 or d % 5 == 0:
            continue  # 8000 must be invertible mod d
        b = (-pow(8000, -1, d)) % d
        # lift b towards 2^40 (largest bytes of the synthetic workloads)
        b += d * int(rng.integers(0, max(1, ((1 << 40) - b) // d)))
        cases.append((b, d))
    assert len(cases) > 50
    b = np.array([c[0] for c in cases], dtype=np.uint64)
    d = np.array([c[1] for c in cases], dtype=np.uint32)
    r = oracle.rate_bps(b, d).tolist()
    for (bi, di), ri in zip(cases, r):
        assert ri == (8000 * bi + 1) // di - 1


# ---------------------------------------------------------------- prefix matching

@pytest.mark.parametrize("seed", range(40))
def test_lpm_matches_brute_force_at_every_boundary(seed):
    rng = np.random.default_rng(seed)
    n_sites, sites, local = random_tiny_registry(rng)
    reg = _oracle_reg(sites, local, n_sites)
    norm = brute.normalise(sites)
    pts = boundary_points(sites)
    got = reg.lookup(np.array(pts, dtype=np.uint32)).tolist()
    exp = [brute.lpm(norm, p, n_sites) for p in pts]
    assert got == exp


def test_lpm_slash0_and_slash32():
    sites = [(0, 0, 0), (ip("9.9.9.9"), 32, 1), (ip("9.9.9.0"), 24, 2)]
    reg = _oracle_reg(sites, [], 3)
    q = [ip("9.9.9.9"), ip("9.9.9.8"), ip("9.9.9.10"), ip("9.9.8.255"), 0, 0xFFFFFFFF]
    assert reg.lookup(np.array(q, dtype=np.uint32)).tolist() == [1, 2, 2, 0, 0, 0]


def test_registry_normalises_host_bits_and_duplicates():
    # 10.1.2.3/8 is 10.0.0.0/8; the same prefix twice for one site is fine
    sites = [(ip("10.1.2.3"), 8, 1), (ip("10.0.0.0"), 8, 1), (ip("10.200.0.0"), 16, 0)]
    reg = _oracle_reg(sites, [], 2)
    assert reg.lookup(np.array([ip("10.0.0.1"), ip("10.200.3.4"), ip("11.0.0.0")], dtype=np.uint32)).tolist() == [1, 0, 2]


@pytest.mark.parametrize("sites,n_sites,code", [
    ([(ip("10.0.0.0"), 8, 0), (ip("10.9.9.9"), 8, 1)], 2, oracle.E_CONFLICT),
    ([(ip("10.0.0.0"), 33, 0)], 1, oracle.E_INVAL),
    ([(ip("10.0.0.0"), 8, 2)], 2, oracle.E_INVAL),
])
def test_registry_errors(sites, n_sites, code):
    with pytest.raises(oracle.OracleError) as e:
        _oracle_reg(sites, [], n_sites)
    assert e.value.code == code
    if code == oracle.E_CONFLICT or sites[0][1] > 32:
        with pytest.raises(ValueError):
            brute.normalise(sites)


# ---------------------------------------------------------------- aggregation

def _edge_records(rng, n, sites, local):
    """Random records biased towards every edge the definition has."""
    pool = [a for a, _, _ in sites] + [a for a, _ in local] + [0, 0xFFFFFFFF]
    out = []
    for _ in range(n):
        def addr():
            if pool and rng.random() < 0.7:
                return (pool[int(rng.integers(0, len(pool)))] + int(rng.integers(-2, 300))) & 0xFFFFFFFF
            return int(rng.integers(0, 1 << 32))
        src, dst = addr(), addr()
        kind = rng.random()
        if kind < 0.1:
            b = 1_000_000 + int(rng.integers(-1, 2))           # around the bulk threshold
        elif kind < 0.15:
            b = int(rng.integers(1 << 62, 1 << 63)) * 2 + 1    # huge: rate saturates, sums wrap
        else:
            b = int(rng.integers(0, 1 << 41))
        p = int(rng.integers(0, 1 << 32))
        f = int(rng.integers(0, 1 << 32))
        dk = rng.random()
        dur = 0 if dk < 0.1 else (1 if dk < 0.2 else int(rng.integers(0, 1 << 32)))
        out.append((src, dst, b, p, f, (f + dur) & 0xFFFFFFFF))
    return out


@pytest.mark.parametrize("seed", range(25))
def test_c_oracle_matches_brute_on_edge_windows(seed):
    rng = np.random.default_rng(100 + seed)
    n_sites, sites, local = random_tiny_registry(rng, n_local=int(rng.integers(0, 4)))
    recs = _edge_records(rng, int(rng.integers(0, 120)), sites, local)
    bulk = int(rng.choice([0, 1_000_000, 1 << 40]))
    exp = brute.classify_aggregate(sites, local, n_sites, recs, bulk)
    reg = _oracle_reg(sites, local, n_sites)
    got = reg.classify_aggregate(soa(recs), bulk, threads=int(rng.integers(1, 5)))
    assert got.tolist() == exp


def test_generated_window_matches_brute_force():
    reg = flowgen.registry_for(flowgen.PLAIN_SMALL)
    rec = flowgen.records_for(flowgen.PLAIN_SMALL, n=3000)
    sites = list(zip(reg.addr.tolist(), reg.length.tolist(), reg.site.tolist()))
    local = list(zip(reg.local_addr.tolist(), reg.local_len.tolist()))
    exp = brute.classify_aggregate(sites, local, reg.n_sites, tuples(rec), 1_000_000)
    got = oracle.Registry.from_generated(reg).classify_aggregate(rec)
    assert got.tolist() == exp


def _combine(a, b):
    out = a.copy()
    out[:, :6] = a[:, :6] + b[:, :6]  # uint64 wraps mod 2^64
    out[:, 6] = np.minimum(a[:, 6], b[:, 6])
    out[:, 7] = np.maximum(a[:, 7], b[:, 7])
    return out


@pytest.mark.parametrize("workload", [flowgen.PLAIN_SMALL, flowgen.PLAIN_LARGE])
def test_invariants_on_generated_windows(workload):
    reg = flowgen.registry_for(workload)
    rec = flowgen.records_for(workload, reg=reg, n=200_000)
    o = oracle.Registry.from_generated(reg)
    rows = o.classify_aggregate(rec)
    # conservation: every record lands in exactly one row
    assert int(rows[:, 0].sum()) == rec.n
    assert int(rows[:, 1].sum(dtype=np.uint64)) == int(rec.bytes.sum(dtype=np.uint64))
    assert int(rows[:, 2].sum(dtype=np.uint64)) == int(rec.packets.astype(np.uint64).sum())
    dur = (rec.last_ms.astype(np.int64) - rec.first_ms.astype(np.int64)) % (1 << 32)
    assert int(rows[:, 3].sum()) == int(dur.sum())
    bulk = (rec.bytes > 1_000_000) & (dur > 0)
    assert int(rows[:, 4].sum()) == int(bulk.sum())
    rates = oracle.rate_bps(rec.bytes[bulk], dur[bulk].astype(np.uint32))
    assert int(rows[:, 5].sum(dtype=np.uint64)) == int(rates.sum(dtype=np.uint64))
    assert int(rows[:, 6].min()) == int(rates.min()) and int(rows[:, 7].max()) == int(rates.max())
    # rows without bulk flows keep the min sentinel and a zero max
    nb = rows[:, 4] == 0
    assert (rows[nb, 6] == np.uint64(M64)).all() and (rows[nb, 7] == 0).all()
    # permutation invariance
    perm = flowgen.permuted(rec, np.random.default_rng(5))
    assert (o.classify_aggregate(perm) == rows).all()
    # split / merge
    k = 77_777
    a = o.classify_aggregate(rec.slice(0, k))
    b = o.classify_aggregate(rec.slice(k, rec.n))
    assert (_combine(a, b) == rows).all()
    # direction: the NODIR row holds exactly the both-or-neither-local records
    def is_local(x):
        m = np.zeros(x.shape[0], bool)
        for la, ll in zip(reg.local_addr.tolist(), reg.local_len.tolist()):
            mask = (0xFFFFFFFF << (32 - ll)) & 0xFFFFFFFF
            m |= (x & np.uint32(mask)) == np.uint32(la & mask)
        return m
    ls, ld = is_local(rec.src_ip), is_local(rec.dst_ip)
    assert int(rows[-1, 0]) == int((ls == ld).sum())
    assert int(rows[0:-1:2, 0].sum()) == int((~ls & ld).sum())   # inbound rows
    assert int(rows[1:-1:2, 0].sum()) == int((ls & ~ld).sum())   # outbound rows


def test_windows_equal_window_by_window():
    reg = flowgen.registry_for(flowgen.PLAIN_SMALL)
    rec = flowgen.records_for(flowgen.BATCHED, reg=reg, n=400_000)
    o = oracle.Registry.from_generated(reg)
    allw = o.classify_aggregate(rec)
    assert allw.shape[0] == rec.n_windows == 256
    for w in (0, 1, 100, 255):
        assert (o.classify_aggregate(rec.window(w)) == allw[w]).all()


def test_generator_is_deterministic():
    a = flowgen.records_for(flowgen.PLAIN_SMALL, n=5000)
    b = flowgen.records_for(flowgen.PLAIN_SMALL, n=5000)
    for f in flowgen.Records.FIELDS:
        assert (getattr(a, f) == getattr(b, f)).all()
    c = flowgen.records_for(flowgen.PLAIN_SMALL, n=5000, stream=1)
    assert not (a.src_ip == c.src_ip).all()


# ---------------------------------------------------------------- median statistic (§III.B.2, §IV.B)

@pytest.mark.parametrize("rate,bucket", [
    (0, 0), (9_999, 0), (10_000, 1), (999_999, 99), (1_000_000, 100), (99_999_999, 9_999),
    (100_000_000, 10_000), (100_009_999, 10_000), (100_010_000, 10_000), (M64, 10_000)])
def test_rate_bucket_closed_forms(rate, bucket):
    # 10 kbps per bucket; everything past 100 Mbps shares the last of 10,001 buckets
    assert int(oracle.rate_bucket(np.array([rate], dtype=np.uint64))[0]) == bucket


def _brute_buckets(sites, local, n_sites, recs, bulk_bytes, filters=None):
    """{row: [bucket of each bulk flow]} by brute force: one record at a time."""
    out = {}
    for src, dst, b, p, f, l in recs:
        dur = (l - f) & 0xFFFFFFFF
        if brute.is_bulk(b, p, dur, bulk_bytes, filters):
            row = brute.row_of(sites, local, n_sites, src, dst)
            out.setdefault(row, []).append(min(brute.rate_bps(b, dur) // 10_000, 10_000))
    return out


def _rate_records(rng, n, sites, local):
    """Bulk-heavy records whose rates cluster near bucket edges and near 1 Mbps."""
    recs = _edge_records(rng, n, sites, local)
    out = []
    for src, dst, b, p, f, l in recs:
        if rng.random() < 0.5:
            dur = int(rng.integers(1, 100_000))
            target = int(rng.choice([999_999, 1_000_000, 10_000 * int(rng.integers(0, 10_002)),
                                     int(rng.integers(0, 1 << 30))]))
            b = max(1_000_001, -(-target * dur // 8000) + int(rng.integers(-2, 3)))
            l = (f + dur) & 0xFFFFFFFF
        out.append((src, dst, b, p, f, l))
    return out


@pytest.mark.parametrize("seed", range(20))
def test_medians_match_brute_force(seed):
    rng = np.random.default_rng(700 + seed)
    n_sites, sites, local = random_tiny_registry(rng, n_local=int(rng.integers(1, 4)))
    recs = _rate_records(rng, int(rng.integers(0, 200)), sites, local)
    bulk = int(rng.choice([0, 1_000_000]))
    cuts = sorted(int(c) for c in rng.integers(0, len(recs) + 1, size=int(rng.integers(0, 4))))
    off = np.array([0] + cuts + [len(recs)], dtype=np.uint64)
    reg = _oracle_reg(sites, local, n_sites)
    med, cnt = oracle.rate_medians(reg, soa(recs), window_offsets=off, bulk_bytes=bulk)
    hist = oracle.rate_histograms(reg, soa(recs), window_offsets=off, bulk_bytes=bulk)
    rows = 2 * n_sites + 3
    assert med.shape == cnt.shape == (len(off) - 1, rows) and hist.shape == (len(off) - 1, rows, 10001)
    for w in range(len(off) - 1):
        exp = _brute_buckets(sites, local, n_sites, recs[int(off[w]):int(off[w + 1])], bulk)
        for r in range(rows):
            b = exp.get(r, [])
            assert int(cnt[w, r]) == len(b)
            assert int(med[w, r]) == (statistics.median_low(b) if b else oracle.NO_MEDIAN)
            assert np.array_equal(hist[w, r], np.bincount(np.array(b, dtype=np.int64), minlength=10001))


def test_median_is_bucket_of_median_rate_on_generated_window():
    reg = flowgen.registry_for(flowgen.PLAIN_SMALL)
    rec = flowgen.records_for(flowgen.PLAIN_SMALL, reg=reg, n=20_000)
    o = oracle.Registry.from_generated(reg)
    med, cnt = oracle.rate_medians(o, rec)
    rows = o.classify_aggregate(rec)
    sites = list(zip(reg.addr.tolist(), reg.length.tolist(), reg.site.tolist()))
    local = list(zip(reg.local_addr.tolist(), reg.local_len.tolist()))
    rates = {}
    for src, dst, b, _p, f, l in tuples(rec):
        dur = (l - f) & 0xFFFFFFFF
        if b > 1_000_000 and dur > 0:
            rates.setdefault(brute.row_of(sites, local, reg.n_sites, src, dst), []).append(brute.rate_bps(b, dur))
    assert cnt[0].tolist() == rows[:, 4].tolist()  # bulk flows, as the aggregate counts them
    for r in range(o.rows):
        if r in rates:
            assert int(med[0, r]) == min(statistics.median_low(rates[r]) // 10_000, 10_000)
            assert int(oracle.rate_bucket(rows[r, 6:7])[0]) <= med[0, r] <= int(oracle.rate_bucket(rows[r, 7:8])[0])
        else:
            assert med[0, r] == oracle.NO_MEDIAN
    assert len(rates) > 20


def _mf(meds, cnts, **kw):
    med = np.array(meds, dtype=np.uint32)
    cnt = np.array(cnts, dtype=np.uint64)
    return oracle.median_flags(med, cnt, med.shape[1] // 2, **kw).tolist()


def test_median_flag_threshold_boundary():
    # bucket 99 covers [990,000, 1,000,000): its flows are all below 1 Mbps; bucket 100 starts at 1 Mbps
    assert _mf([[99, 100]], [[1, 1]]) == [[1]]
    assert _mf([[100, 99]], [[1, 1]]) == [[2]]
    assert _mf([[0, 10_000]], [[5, 5]], threshold_bps=100_000_000) == [[1]]
    assert _mf([[0, 0]], [[1, 1]], threshold_bps=0) == [[0]]
    # no bulk flow, or fewer than the minimum: no median to judge
    assert _mf([[oracle.NO_MEDIAN, 0]], [[0, 1]]) == [[2]]
    assert _mf([[0, 0]], [[2, 3]], min_bulk_flows=3) == [[2]]
    assert _mf([[0, 0]], [[1, 1]], min_bulk_flows=0) == [[3]]


def test_median_flag_two_consecutive_windows():
    # one site; windows: low IN, low IN+OUT, low OUT, nothing, low IN
    meds = [[0, 500], [0, 0], [500, 0], [500, 500], [0, 500]]
    cnts = [[1, 1]] * 5
    assert [f[0] for f in _mf(meds, cnts)] == [1, 3 | 4, 2 | 8, 0, 1]
    # the window before the first comes from the caller
    assert [f[0] for f in _mf(meds, cnts, prev=np.array([1], dtype=np.uint8))] == [1 | 4, 3 | 4, 2 | 8, 0, 1]
    assert [f[0] for f in _mf(meds, cnts, prev=np.array([2 | 8], dtype=np.uint8))] == [1, 3 | 4, 2 | 8, 0, 1]
    # sites are judged independently
    two = _mf([[0, 500, 500, 0], [0, 500, 500, 0]], [[1, 1, 1, 1]] * 2)
    assert two == [[1, 2], [1 | 4, 2 | 8]]


# ---------------------------------------------------------------- exclusion filters (§III.B.2)

@pytest.mark.parametrize("b,p,d,filters,exp", [
    (2_000_000, 10, 5, {}, True),
    (2_000_000, 10, 5, {"min_avg_packet_bytes": 200_000}, True),      # average exactly the minimum
    (2_000_000, 11, 5, {"min_avg_packet_bytes": 200_000}, False),     # 181,818.18... B per packet
    (1_999_999, 10, 5, {"min_avg_packet_bytes": 200_000}, False),
    (2_000_000, 0, 5, {"min_avg_packet_bytes": 4_000_000_000}, True),  # no packets: no average to judge
    (M64, 2**32 - 1, 5, {"min_avg_packet_bytes": 2**32 - 1}, True),   # product near 2^64
    (2_000_000, 4, 5, {"min_packets": 5}, False),
    (2_000_000, 5, 5, {"min_packets": 5}, True),
    (2_000_000, 5, 99, {"min_duration_ms": 100}, False),
    (2_000_000, 5, 100, {"min_duration_ms": 100}, True),
    (2_000_000, 5, 0, {"min_duration_ms": 0}, False),                 # a zero duration never has a rate
    (1_000_000, 5, 100, {}, False),                                   # bulk threshold is strict
])
def test_bulk_rule_closed_forms(b, p, d, filters, exp):
    assert brute.is_bulk(b, p, d, 1_000_000, filters) is exp
    assert oracle.is_bulk(b, p, d, 1_000_000, filters) is exp


def _random_filters(rng):
    f = {}
    if rng.random() < 0.7:
        f["min_avg_packet_bytes"] = int(rng.choice([1, 64, 100, 1000, 2**31, 2**32 - 1]))
    if rng.random() < 0.5:
        f["min_packets"] = int(rng.choice([1, 2, 10, 2**31]))
    if rng.random() < 0.5:
        f["min_duration_ms"] = int(rng.choice([1, 2, 1000, 2**31]))
    return f


@pytest.mark.parametrize("seed", range(15))
def test_filters_match_brute_on_edge_windows(seed):
    rng = np.random.default_rng(1300 + seed)
    n_sites, sites, local = random_tiny_registry(rng, n_local=int(rng.integers(1, 4)))
    recs = _edge_records(rng, int(rng.integers(0, 150)), sites, local)
    # packet counts spread around typical ACK and data sizes
    recs = [(s, d, b, int(rng.choice([0, 1, 2, 10, b // 64 + 1, b // 1500 + 1, 2**32 - 1])) & 0xFFFFFFFF, f, l)
            for s, d, b, _p, f, l in recs]
    bulk = int(rng.choice([0, 1_000_000]))
    filters = _random_filters(rng)
    exp = brute.classify_aggregate(sites, local, n_sites, recs, bulk, filters)
    reg = _oracle_reg(sites, local, n_sites)
    got = reg.classify_aggregate(soa(recs), bulk, threads=int(rng.integers(1, 4)), filters=filters)
    assert got.tolist() == exp
    med, cnt = oracle.rate_medians(reg, soa(recs), bulk_bytes=bulk, filters=filters)
    buckets = _brute_buckets(sites, local, n_sites, recs, bulk, filters)
    for r in range(2 * n_sites + 3):
        b = buckets.get(r, [])
        assert int(cnt[0, r]) == len(b) == exp[r][4]
        assert int(med[0, r]) == (statistics.median_low(b) if b else oracle.NO_MEDIAN)


def test_filters_only_remove_rate_eligible_flows():
    reg = flowgen.registry_for(flowgen.PLAIN_SMALL)
    rec = flowgen.records_for(flowgen.PLAIN_SMALL, reg=reg, n=100_000)
    o = oracle.Registry.from_generated(reg)
    base = o.classify_aggregate(rec)
    assert (o.classify_aggregate(rec, filters={"min_avg_packet_bytes": 0, "min_packets": 0,
                                               "min_duration_ms": 0}) == base).all()
    prev = base
    for f in ({"min_avg_packet_bytes": 100}, {"min_avg_packet_bytes": 100, "min_packets": 1000},
              {"min_avg_packet_bytes": 100, "min_packets": 1000, "min_duration_ms": 5000}):
        got = o.classify_aggregate(rec, filters=f)
        assert (got[:, :4] == base[:, :4]).all()      # flows, bytes, packets, duration: every record
        assert (got[:, 4] <= prev[:, 4]).all()        # each added filter keeps a subset
        assert (got[:, 6] >= prev[:, 6]).all() and (got[:, 7] <= prev[:, 7]).all()
        assert got[:, 4].sum() < prev[:, 4].sum()     # and removes some on this workload
        prev = got


# ---------------------------------------------------------------- per-host statistics (§III.B.2)

def _brute_hosts(sites, local, n_sites, recs, bulk_bytes, filters=None):
    out = {}
    for src, dst, b, p, f, l in recs:
        dur = (l - f) & 0xFFFFFFFF
        if not brute.is_bulk(b, p, dur, bulk_bytes, filters):
            continue
        row = brute.row_of(sites, local, n_sites, src, dst)
        if row >= 2 * n_sites:
            continue
        remote = src if row % 2 == 0 else dst
        rate = brute.rate_bps(b, dur)
        e = out.setdefault((remote << 32) | row, [0, 0, 0, M64, 0])
        e[0] += 1
        e[1] = (e[1] + b) & M64
        e[2] = (e[2] + rate) & M64
        e[3] = min(e[3], rate)
        e[4] = max(e[4], rate)
    return out


@pytest.mark.parametrize("seed", range(15))
def test_host_stats_match_brute(seed):
    rng = np.random.default_rng(2100 + seed)
    n_sites, sites, local = random_tiny_registry(rng, n_local=int(rng.integers(1, 4)))
    recs = _rate_records(rng, int(rng.integers(0, 300)), sites, local)
    # repeat some remote hosts so hosts hold several flows
    recs += [recs[int(i)] for i in rng.integers(0, len(recs), size=len(recs) // 2)] if recs else []
    bulk = int(rng.choice([0, 1_000_000]))
    filters = _random_filters(rng) if rng.random() < 0.3 else None
    exp = _brute_hosts(sites, local, n_sites, recs, bulk, filters)
    reg = _oracle_reg(sites, local, n_sites)
    keys, st = oracle.host_stats(reg, soa(recs), bulk, filters)
    assert sorted(exp) == keys.tolist()
    assert [exp[k] for k in sorted(exp)] == st.tolist()


def test_host_stats_add_up_to_the_site_rows():
    reg = flowgen.registry_for(flowgen.PLAIN_LARGE)
    rec = flowgen.records_for(flowgen.PLAIN_LARGE, reg=reg, n=300_000)
    o = oracle.Registry.from_generated(reg)
    rows = o.classify_aggregate(rec)
    keys, st = oracle.host_stats(o, rec)
    row_of_key = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
    S2 = 2 * reg.n_sites
    for field, col in ((4, 0), (5, 2)):   # bulk flows, rate sum
        agg = np.zeros(S2, dtype=np.uint64)
        np.add.at(agg, row_of_key, st[:, col])
        assert (agg == rows[:S2, field]).all()
    mn = np.full(S2, M64, dtype=np.uint64)
    mx = np.zeros(S2, dtype=np.uint64)
    np.minimum.at(mn, row_of_key, st[:, 3])
    np.maximum.at(mx, row_of_key, st[:, 4])
    assert (mn == rows[:S2, 6]).all() and (mx == rows[:S2, 7]).all()
    # the remote address of a key lies in its site (the LPM answer for it is the key's site)
    ips = (keys >> np.uint64(32)).astype(np.uint32)
    assert (o.lookup(ips) == (row_of_key // 2).astype(np.uint32)).all()
    assert keys.size > 10_000 and (st[:, 0] > 1).any()


def test_median_worked_example():
    from tests._helpers import dense_histograms, median_example
    sites, local, S, recs, off, g = median_example()
    reg = _oracle_reg(sites, local, S)
    h = oracle.rate_histograms(reg, soa(recs), window_offsets=off, bulk_bytes=g["bulk_bytes"])
    assert (h[:, :2 * S] == dense_histograms(g, 2 * S)).all()
    # the oracle also counts the rows the library keeps no histogram for: the
    # inbound flow from 203.0.113.9 (no registered site) and the both-local one
    assert h[0, 2 * S].sum() == 1 and h[0, 2 * S + 2].sum() == 1 and h[:, 2 * S:].sum() == 2
    med, cnt = oracle.rate_medians(reg, soa(recs), window_offsets=off, bulk_bytes=g["bulk_bytes"])
    want = [[oracle.NO_MEDIAN if m == "NONE" else m for m in w] for w in g["expected_medians"]]
    assert med[:, :2 * S].tolist() == want
    assert cnt[:, :2 * S].tolist() == g["expected_counts"]
    f = oracle.median_flags(med, cnt, S, g["threshold_bps"], 0, np.array(g["prev_flags"], dtype=np.uint8))
    assert f.tolist() == g["expected_flags"]


# ---------------------------------------------------------------- per-host medians (§III.B.2)

def _brute_bucket(rate: int) -> int:
    # 10 kbps buckets, everything from 100 Mbps up in the last (bucket 10,000)
    return min(rate // 10_000, 10_000)


def _brute_host_rates(sites, local, n_sites, recs, bulk_bytes, filters=None):
    out = {}
    for src, dst, b, p, f, l in recs:
        dur = (l - f) & 0xFFFFFFFF
        if not brute.is_bulk(b, p, dur, bulk_bytes, filters):
            continue
        row = brute.row_of(sites, local, n_sites, src, dst)
        if row >= 2 * n_sites:
            continue
        remote = src if row % 2 == 0 else dst
        out.setdefault((remote << 32) | row, []).append(brute.rate_bps(b, dur))
    return out


@pytest.mark.parametrize("seed", range(15))
def test_host_medians_match_brute(seed):
    rng = np.random.default_rng(2600 + seed)
    n_sites, sites, local = random_tiny_registry(rng, n_local=int(rng.integers(1, 4)))
    recs = _rate_records(rng, int(rng.integers(0, 300)), sites, local)
    recs += [recs[int(i)] for i in rng.integers(0, len(recs), size=len(recs))] if recs else []
    bulk = int(rng.choice([0, 1_000_000]))
    filters = _random_filters(rng) if rng.random() < 0.3 else None
    rates = _brute_host_rates(sites, local, n_sites, recs, bulk, filters)
    reg = _oracle_reg(sites, local, n_sites)
    keys, med = oracle.host_medians(reg, soa(recs), bulk, filters)
    assert sorted(rates) == keys.tolist()
    # the lower median of the rates, then its bucket (buckets are monotone in the rate)
    assert [_brute_bucket(statistics.median_low(rates[k])) for k in sorted(rates)] == med.tolist()


def test_host_medians_bucket_array_definition():
    """On a generated window: each host's median is where its bucket array's
    cumulative count first reaches ceil(N/2) (the paper's bucket arrays, built
    here per host with bincount), lies between the buckets of its minimum and
    maximum rates, and the keys are host_stats'."""
    reg = flowgen.registry_for(flowgen.PLAIN_LARGE)
    rec = flowgen.records_for(flowgen.PLAIN_LARGE, reg=reg, n=300_000, stream=3)
    o = oracle.Registry.from_generated(reg)
    keys, med = oracle.host_medians(o, rec)
    k2, st = oracle.host_stats(o, rec)
    assert (keys == k2).all() and keys.size > 10_000
    lo, hi = oracle.rate_bucket(st[:, 3]), oracle.rate_bucket(st[:, 4])
    assert ((lo <= med) & (med <= hi)).all()
    # per-host bucket arrays for the hosts with the most flows, and a sample of the rest
    row, is_bulk, rate = oracle._classify_rows(o, rec, 1_000_000)
    sel = is_bulk & (row < 2 * reg.n_sites)
    remote = np.where(row % 2 == 0, rec.src_ip, rec.dst_ip)[sel]
    key = (remote.astype(np.uint64) << np.uint64(32)) | row[sel].astype(np.uint64)
    bucket = oracle.rate_bucket(rate[sel])
    pick = list(np.argsort(-st[:, 0].astype(np.int64))[:20]) + \
        list(np.random.default_rng(4).choice(keys.size, 200, replace=False))
    for i in pick:
        arr = np.bincount(bucket[key == keys[i]], minlength=10_001)
        n = int(arr.sum())
        assert n == int(st[i, 0])
        assert int(np.argmax(np.cumsum(arr) >= (n + 1) // 2)) == int(med[i])
    assert st[pick[0], 0] >= 10  # the busiest hosts hold many flows


def test_host_worked_example():
    g = load_golden("host_median_example.json")
    sites = [(ip(a), l, s) for a, l, s in g["sites"]]
    local = [(ip(a), l) for a, l in g["local"]]
    recs = [(ip(r[0]), ip(r[1]), r[2], r[3], r[4], r[5]) for r in g["records"]]
    reg = _oracle_reg(sites, local, g["n_sites"])
    want_keys = [(ip(a) << 32) | row for a, row, _, _ in g["expected_hosts"]]
    keys, st = oracle.host_stats(reg, soa(recs), g["bulk_bytes"])
    assert keys.tolist() == want_keys
    assert st.tolist() == [s for _, _, s, _ in g["expected_hosts"]]
    keys, med = oracle.host_medians(reg, soa(recs), g["bulk_bytes"])
    assert keys.tolist() == want_keys
    assert med.tolist() == [m for _, _, _, m in g["expected_hosts"]]
    # and the brute force agrees with the hand derivation
    assert sorted(_brute_hosts(sites, local, g["n_sites"], recs, g["bulk_bytes"])) == want_keys
