"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Integer work, so the bar is bit-exact equality of every field of every row
(tolerance 0) on the same seeded inputs: the worked example, generated
windows of each workload (full size for the 100 k and 10 M windows), the
batched form window by window, launch-shape and registry-layout variants, and
edge cases (empty and ragged runs, tile boundaries, maximum contention,
wrap-around and saturation).
"""
import sys

import numpy as np
import pytest

import flowgen
import oracle
import paper_1108_1785_amd as gnm
from oracle import brute
from tests._gpu import diff, flags, run, to_device
from tests._helpers import M64, random_tiny_registry, soa, worked_example

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
    a = [s[0] for s in sites]
    l = [s[1] for s in sites]
    s = [s[2] for s in sites]
    la = [x[0] for x in local]
    ll = [x[1] for x in local]
    return gnm.Registry(a, l, s, n_sites, la, ll, **kw), oracle.Registry(a, l, s, n_sites, la, ll)


def test_worked_example(torch_cuda):
    say("case: worked example")
    sites, local, S, recs, exp, g = worked_example()
    reg, _ = _regs(sites, local, S)
    got = run(reg, soa(recs), bulk_bytes=g["bulk_bytes"])
    assert got.tolist() == exp
    assert flags(reg, got, g["threshold_bps"]).tolist() == g["expected_flags"]


_SMALL = {}


def _small():
    if not _SMALL:
        r = flowgen.registry_for(flowgen.PLAIN_SMALL)
        _SMALL["reg"] = r
        _SMALL["orc"] = oracle.Registry.from_generated(r)
        _SMALL["rec"] = flowgen.records_for(flowgen.PLAIN_SMALL, reg=r)
    return _SMALL


@pytest.mark.parametrize("rpt", [0, 1, 2, 4])
@pytest.mark.parametrize("ws", [False, True])
def test_plain_small_full(torch_cuda, rpt, ws):
    say("case: plain-small 100k records, records_per_thread", rpt, "workspace", ws)
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    exp = s["orc"].classify_aggregate(s["rec"])
    got = run(reg, s["rec"], records_per_thread=rpt, workspace=gnm.make_workspace(reg) if ws else None)
    assert (got == exp).all(), diff(got, exp)
    assert (flags(reg, got) == oracle.flags(exp, s["reg"].n_sites)).all()


def test_records_per_thread_8_rejected(torch_cuda):
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    with pytest.raises(gnm.GnmError) as e:
        run(reg, s["rec"].slice(0, 100), records_per_thread=8)
    assert e.value.code == gnm.GNM_E_INVAL


@pytest.mark.parametrize("shift", [1, 2, 3, 5])
@pytest.mark.parametrize("rpt", [0, 2])
def test_misaligned_record_views(torch_cuda, shift, rpt):
    say("case: record pointers offset by", shift, "records, rpt", rpt)
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    rec = s["rec"].slice(0, 54_321)
    exp = s["orc"].classify_aggregate(rec)
    got = run(reg, rec, shift=shift, records_per_thread=rpt, workspace=gnm.make_workspace(reg))
    assert (got == exp).all(), diff(got, exp)


@pytest.mark.parametrize("grid", [1, 3, 64, 256, 1000])
@pytest.mark.parametrize("ws", [False, True])
def test_plain_small_grid_shapes(torch_cuda, grid, ws):
    say("case: plain-small grid_blocks", grid, "workspace", ws)
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    exp = s["orc"].classify_aggregate(s["rec"])
    got = run(reg, s["rec"], grid_blocks=grid, workspace=gnm.make_workspace(reg, grid) if ws else None)
    assert (got == exp).all(), diff(got, exp)


def test_workspace_too_small_falls_back(torch_cuda):
    import torch
    say("case: undersized workspace -> atomic merge")
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    exp = s["orc"].classify_aggregate(s["rec"])
    small = torch.empty(64, dtype=torch.uint8, device="cuda:0")
    got = run(reg, s["rec"], workspace=small)
    assert (got == exp).all(), diff(got, exp)


@pytest.mark.parametrize("kw", [dict(layout="wide"), dict(layout="wide", root_bits=8), dict(layout="lines"),
                                dict(root_bits=8, list_max=2), dict(root_bits=14, list_max=8),
                                dict(root_bits=10, list_max=3), dict(lds_bytes=8192 + 256, root_bits=10),
                                dict(lds_bytes=2048, root_bits=8), dict(layout="shallow"),
                                dict(layout="wide-shallow"), dict(layout="wide-shallow", lds_bytes=2048, root_bits=8),
                                dict(layout="wide-shallow", root_bits=14), dict(node_bits=8),
                                dict(node_bits=4, root_bits=8), dict(node_bits=16, root_bits=14, layout="wide")])
def test_registry_layout_variants(torch_cuda, kw):
    say("case: layout", kw)
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"], **kw)
    info = reg.info()
    say("  info", info)
    exp = s["orc"].classify_aggregate(s["rec"])
    got = run(reg, s["rec"])
    assert (got == exp).all(), diff(got, exp)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 63, 64, 65, 1023, 1024, 1025, 4095, 4096, 4097, 8191, 8193, 70001])
def test_ragged_sizes(torch_cuda, n):
    say("case: ragged n", n)
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    rec = s["rec"].slice(0, n)
    exp = s["orc"].classify_aggregate(rec)
    for ws in (None, gnm.make_workspace(reg)):
        got = run(reg, rec, workspace=ws)
        assert (got == exp).all(), diff(got, exp)


def test_edge_registries_and_records(torch_cuda):
    from tests.test_oracle_pins import _edge_records
    for seed in range(30):
        say("case: edge registry seed", seed)
        rng = np.random.default_rng(500 + seed)
        n_sites, sites, local = random_tiny_registry(rng, n_prefixes=int(rng.integers(0, 60)),
                                                     n_local=int(rng.integers(0, 4)))
        recs = _edge_records(rng, int(rng.integers(0, 3000)), sites, local)
        bulk = int(rng.choice([0, 1_000_000, 1 << 40]))
        kw = dict(root_bits=int(rng.integers(8, 15)), list_max=int(rng.integers(2, 9)),
                  layout=str(rng.choice(["auto", "wide", "lines", "shallow", "wide-shallow"])))
        reg, orc = _regs(sites, local, n_sites, **kw)
        rec = soa(recs)
        exp = orc.classify_aggregate(rec, bulk)
        got = run(reg, rec, bulk_bytes=bulk, records_per_thread=int(rng.choice([0, 1, 2, 4])),
                  workspace=gnm.make_workspace(reg) if seed % 2 else None)
        assert (got == exp).all(), (seed, diff(got, exp))
        if seed < 5:
            assert got.tolist() == brute.classify_aggregate(sites, local, n_sites, recs, bulk)


def test_max_contention_one_row(torch_cuda):
    say("case: all records in one row")
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    rec = s["rec"].slice(0, 50_000).copy()
    rec.src_ip[:] = rec.src_ip[0]
    rec.dst_ip[:] = rec.dst_ip[0]
    exp = s["orc"].classify_aggregate(rec)
    assert int((exp[:, 0] > 0).sum()) == 1
    got = run(reg, rec)
    assert (got == exp).all(), diff(got, exp)


def test_all_nodir_and_all_unmatched(torch_cuda):
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    rec = s["rec"].slice(0, 30_000)
    a = rec.copy()
    a.src_ip[:] = 0xF0000001  # neither endpoint local: NODIR
    a.dst_ip[:] = 0xF0000002
    b = rec.copy()
    b.src_ip[:] = s["reg"].local_addr[0] | 5
    b.dst_ip[:] = 0xF0000000 | (np.arange(b.n, dtype=np.uint32) & 0xFFFF)  # remote in no site
    for name, r in (("nodir", a), ("unmatched", b)):
        say("case:", name)
        exp = s["orc"].classify_aggregate(r)
        got = run(reg, r)
        assert (got == exp).all(), diff(got, exp)


def test_wrap_and_saturation(torch_cuda):
    say("case: 2^63-byte records (sums wrap, rates saturate)")
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    r = s["rec"].slice(0, 20_000).copy()
    r.bytes[::3] = np.uint64(1 << 63) + np.uint64(12345)
    r.bytes[1::7] = np.uint64(M64)
    r.packets[::5] = np.uint32(0xFFFFFFFF)
    exp = s["orc"].classify_aggregate(r)
    assert int(exp[:, 7].max()) == M64
    got = run(reg, r)
    assert (got == exp).all(), diff(got, exp)


def test_near_integer_rates(torch_cuda):
    say("case: near-integer quotients")
    rng = np.random.default_rng(3)
    cases = []
    while len(cases) < 20000:
        d = int(rng.integers(2, 1 << 32))
        if d % 2 == 0 or d % 5 == 0:
            continue
        b = (-pow(8000, -1, d)) % d
        b += d * int(rng.integers(0, max(1, ((1 << 40) - b) // d)))
        if b > 1_000_000:
            cases.append((b, d))
    sites = [(0, 0, 0)]
    local = [(0x0A000000, 8)]
    recs = [(0x0A000001, 0x0B000000 + i, b, 1, 7, (7 + d) & 0xFFFFFFFF) for i, (b, d) in enumerate(cases)]
    reg, orc = _regs(sites, local, 1)
    rec = soa(recs)
    exp = orc.classify_aggregate(rec)
    got = run(reg, rec)
    assert (got == exp).all(), diff(got, exp)
    # one record per run pins each rate individually (min = max = rate)
    for b, d in cases[:200]:
        one = soa([(0x0A000001, 0x0B000000, b, 1, 0, d)])
        g1 = run(reg, one)
        assert int(g1[1, 6]) == (8000 * b) // d == int(g1[1, 7])


def test_accumulate_flag(torch_cuda):
    import torch
    say("case: GNM_ACCUMULATE over two halves")
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    rec = s["rec"]
    exp = s["orc"].classify_aggregate(rec)
    for ws in (None, gnm.make_workspace(reg)):
        acc = torch.empty((1, reg.rows, 8), dtype=torch.int64, device="cuda:0")
        run(reg, rec.slice(0, 40_000), acc=acc, workspace=ws)
        got = run(reg, rec.slice(40_000, rec.n), acc=acc, accumulate=True, workspace=ws)
        assert (got == exp).all(), diff(got, exp)


def test_deterministic_repeats(torch_cuda):
    say("case: repeat runs identical")
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    d = to_device(s["rec"])
    a = run(reg, s["rec"], dev_rec=d)
    for _ in range(3):
        assert (run(reg, s["rec"], dev_rec=d) == a).all()
    perm = flowgen.permuted(s["rec"], np.random.default_rng(9))
    assert (run(reg, perm) == a).all()


def test_batched_windows(torch_cuda):
    say("case: batched 256 windows (scaled to 6M records)")
    r = flowgen.registry_for(flowgen.PLAIN_SMALL)
    rec = flowgen.records_for(flowgen.BATCHED, reg=r, n=6_000_000)
    off = rec.window_offsets.copy()
    assert len(off) == 257
    orc = oracle.Registry.from_generated(r)
    exp = orc.classify_aggregate(rec)
    reg = gnm.Registry.from_generated(r)
    for rpt, grid, ws in ((0, 0, False), (0, 0, True), (2, 0, True), (1, 37, True), (4, 2000, True), (4, 2000, False)):
        say("  rpt", rpt, "grid", grid, "workspace", ws)
        got = run(reg, rec, records_per_thread=rpt, grid_blocks=grid,
                  workspace=gnm.make_workspace(reg, grid) if ws else None)
        assert (got == exp).all(), diff(got, exp)
    fexp = oracle.flags(exp, r.n_sites)
    assert (flags(reg, got) == fexp).all()


def test_batched_with_empty_windows(torch_cuda):
    say("case: batched with empty and tiny windows")
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    rec = s["rec"]
    cuts = [0, 0, 0, 1, 1, 64, 65, 5000, 5000, 70000, 99999, rec.n, rec.n]
    off = np.array(cuts, dtype=np.uint64)
    exp = s["orc"].classify_aggregate(rec, window_offsets=off)
    for grid in (0, 1, 7, 300):
        for ws in (None, gnm.make_workspace(reg, grid)):
            got = run(reg, rec, window_offsets=off, grid_blocks=grid, workspace=ws)
            assert (got == exp).all(), diff(got, exp)
    assert (got[0, :, 6] == np.uint64(M64)).all() and (got[0, :, 0] == 0).all()


def test_many_tiny_windows(torch_cuda):
    """20,000 windows of 0..8 records (every workgroup slice crosses hundreds
    of window boundaries), and offsets past the end, which clamp to n."""
    say("case: 20000 tiny windows")
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    rng = np.random.default_rng(2024)
    sizes = rng.integers(0, 9, size=20_000)
    off = np.zeros(sizes.size + 1, dtype=np.uint64)
    np.cumsum(sizes, out=off[1:])
    rec = s["rec"].slice(0, int(off[-1]))
    exp = s["orc"].classify_aggregate(rec, window_offsets=off)
    for grid, ws in ((0, True), (37, False), (1024, True)):
        got = run(reg, rec, window_offsets=off, grid_blocks=grid,
                  workspace=gnm.make_workspace(reg, grid) if ws else None)
        assert (got == exp).all(), diff(got, exp)
    # offsets beyond the records clamp to n: the last windows are empty
    off2 = off.copy()
    off2[-3:] = np.uint64(rec.n + 1000)
    exp2 = s["orc"].classify_aggregate(rec, window_offsets=np.minimum(off2, np.uint64(rec.n)))
    got2 = run(reg, rec, window_offsets=off2)
    assert (got2 == exp2).all(), diff(got2, exp2)


def test_sites_beyond_16_bits(torch_cuda):
    say("case: 70000 sites (no 16-bit site codes)")
    rng = np.random.default_rng(77)
    from tests.test_oracle_pins import _edge_records
    _, sites, local = random_tiny_registry(rng, n_prefixes=50, n_local=2)
    sites = [(a, l, (s * 13331) % 70000) for a, l, s in sites]
    recs = _edge_records(rng, 3000, sites, local)
    for layout in ("wide", "lines"):
        reg, orc = _regs(sites, local, 70000, layout=layout)
        exp = orc.classify_aggregate(soa(recs))
        got = run(reg, soa(recs))
        assert (got == exp).all(), diff(got, exp)


def test_large_table_batched(torch_cuda):
    """1,000,000 prefixes / 20,000 sites: lookup structure and accumulator
    table both beyond LDS (device-memory lines and tables)."""
    say("case: large-table registry, 3M records in 4 windows (one empty) + one plain window")
    r = flowgen.registry_for(flowgen.LARGE_TABLE)
    rec = flowgen.records_for(flowgen.LARGE_TABLE, reg=r, n=3_000_000, stream=7)
    orc = oracle.Registry.from_generated(r)
    off = np.array([0, 1_200_000, 1_200_000, 2_999_999, 3_000_000], dtype=np.uint64)
    exp = orc.classify_aggregate(rec, window_offsets=off)
    w = rec.slice(0, 1_000_003)
    exp_w = orc.classify_aggregate(w)
    # automatic layout (12-bit first level), and 8-bit first level with leaf
    # lines below it in device memory
    for kw in (dict(), dict(layout="shallow", node_bits=8)):
        reg = gnm.Registry.from_generated(r, **kw)
        info = reg.info()
        say("  layout", kw, info)
        assert not info["acc_in_lds"] and info["cache_slots"] > 0
        for rpt in (0, 1):
            got = run(reg, rec, window_offsets=off, records_per_thread=rpt, workspace=gnm.make_workspace(reg))
            assert (got == exp).all(), diff(got, exp)
        got = run(reg, w)
        assert (got == exp_w).all()
        assert (flags(reg, got) == oracle.flags(got, r.n_sites)).all()
        del reg


def test_plain_large_full_size(torch_cuda):
    say("case: plain-large 10M records (full size, bench launch shape)")
    r = flowgen.registry_for(flowgen.PLAIN_LARGE)
    rec = flowgen.records_for(flowgen.PLAIN_LARGE, reg=r)
    orc = oracle.Registry.from_generated(r)
    exp = orc.classify_aggregate(rec)
    reg = gnm.Registry.from_generated(r)
    say("  info", reg.info())
    d = to_device(rec)
    for ws in (gnm.make_workspace(reg), None):
        got = run(reg, rec, dev_rec=d, workspace=ws)
        assert (got == exp).all(), diff(got, exp)
    assert (flags(reg, got) == oracle.flags(exp, r.n_sites)).all()


def test_graph_replays_match_oracle(torch_cuda):
    import torch
    say("case: hipGraph replay of a batched step, buffers refilled between replays")
    r = flowgen.registry_for(flowgen.PLAIN_SMALL)
    orc = oracle.Registry.from_generated(r)
    reg = gnm.Registry.from_generated(r)
    recs = [flowgen.records_for(flowgen.BATCHED, reg=r, n=1_500_000) for _ in range(1)]
    rec_a = recs[0]
    # a second batch with the same window sizes but other records
    rng = np.random.default_rng(5)
    rec_b = flowgen.permuted(rec_a, rng)
    rec_b.window_offsets = rec_a.window_offsets
    nw = rec_a.n_windows
    d = to_device(rec_a)
    off = torch.from_numpy(rec_a.window_offsets.view(np.int64)).to("cuda:0")
    acc = torch.empty((nw, reg.rows, 8), dtype=torch.int64, device="cuda:0")
    flg = torch.empty(nw * r.n_sites, dtype=torch.uint8, device="cuda:0")
    ws = gnm.make_workspace(reg)
    g = gnm.Graph(reg, d, acc, window_offsets=off, n_windows=nw, flags=flg, n=rec_a.n, workspace=ws)
    exp_a = orc.classify_aggregate(rec_a)
    exp_b = orc.classify_aggregate(rec_b)
    db = to_device(rec_b)
    for it in range(4):
        use_b = it % 2 == 1
        src = db if use_b else to_device(rec_a)
        for f in d:
            d[f].copy_(src[f])  # refill the captured buffers (eager work between replays)
        acc.fill_(7)
        flg.fill_(0xA5)  # every replay must write every flag
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        exp = exp_b if use_b else exp_a
        got = gnm.acc_to_numpy(acc)
        assert (got == exp).all(), (it, diff(got, exp))
        assert (flg.cpu().numpy().reshape(nw, r.n_sites) == oracle.flags(exp, r.n_sites)).all()
    g.close()


def test_graph_accumulates_once_per_replay(torch_cuda):
    """A captured step with GNM_ACCUMULATE: creating the graph runs nothing,
    and each replay adds the records once, so after one plain call and two
    replays the table is that of the records three times over."""
    import torch
    say("case: graph with GNM_ACCUMULATE, one eager call then two replays")
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    rec = s["rec"].slice(0, 70_001)
    d = to_device(rec)
    acc = torch.empty((1, reg.rows, 8), dtype=torch.int64, device="cuda:0")
    ws = gnm.make_workspace(reg)
    gnm.classify_aggregate(reg, d, acc, n=rec.n, workspace=ws)
    g = gnm.Graph(reg, d, acc, n=rec.n, workspace=ws, accumulate=True)
    torch.cuda.synchronize()
    exp1 = s["orc"].classify_aggregate(rec)
    got = gnm.acc_to_numpy(acc)[0]
    assert (got == exp1).all(), diff(got, exp1)
    g.launch()
    g.launch()
    torch.cuda.synchronize()
    three = flowgen.concat([rec, rec, rec])
    three.window_offsets = None
    exp3 = s["orc"].classify_aggregate(three)
    got = gnm.acc_to_numpy(acc)[0]
    assert (got == exp3).all(), diff(got, exp3)
    g.close()


def test_autotune_choice_is_exact(torch_cuda, tmp_path):
    import torch
    from paper_1108_1785_amd import tune
    say("case: autotune then run with the tuned shape")
    s = _small()
    reg = gnm.Registry.from_generated(s["reg"])
    rec = flowgen.records_for(flowgen.BATCHED, reg=s["reg"], n=2_000_000)
    d = to_device(rec)
    off = torch.from_numpy(rec.window_offsets.view(np.int64)).to("cuda:0")
    nw = rec.n_windows
    acc = torch.empty((nw, reg.rows, 8), dtype=torch.int64, device="cuda:0")
    ws = gnm.make_workspace(reg)
    cache = str(tmp_path / "tune.json")
    t = tune.tuned_params(reg, d, acc, window_offsets=off, n_windows=nw, n=rec.n, workspace=ws, cache_path=cache)
    say("  tuned", t)
    assert not t["cached"] and t["records_per_thread"] in (1, 2, 4) and len(t["tried"]) >= 6
    t2 = tune.tuned_params(reg, d, acc, window_offsets=off, n_windows=nw, n=rec.n, workspace=ws, cache_path=cache)
    assert t2["cached"] and t2["records_per_thread"] == t["records_per_thread"]
    exp = oracle.Registry.from_generated(s["reg"]).classify_aggregate(rec)
    got = run(reg, rec, records_per_thread=t["records_per_thread"], grid_blocks=t["grid_blocks"],
              workspace=gnm.make_workspace(reg, t["grid_blocks"]))
    assert (got == exp).all(), diff(got, exp)
