"""C-ABI surface and host-side logic of libgnm (CPU only: no device calls).

The library must load without a GPU, export every function include/gnm.h
declares, and build registries host-only; the host walk of the built trie is
checked against the oracle at every interval boundary (so the layout builder
is pinned before any kernel runs).
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import paper_1108_1785_amd as gnm
from oracle import brute
from tests._helpers import boundary_points, ip, random_tiny_registry, worked_example

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "gnm.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gnm_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert sorted(gnm.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    L = gnm.lib()
    for name in _declared():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", gnm.LIB_PATH], capture_output=True, text=True).stdout
    for name in _declared():
        assert re.search(r"\bT %s\b" % name, out), name


def test_strings_and_defaults():
    assert gnm.version().startswith("gnm")
    L = gnm.lib()
    for code in (0, -1, -2, -3, -4, -5):
        assert L.gnm_strerror(code)
    p = L.gnm_params_default()
    assert p.bulk_bytes == 1_000_000 and p.flags == 0 and p.records_per_thread == 0


def _host_reg(sites, local, n_sites, **kw):
    a = [s[0] for s in sites]
    l = [s[1] for s in sites]
    s = [s[2] for s in sites]
    return gnm.Registry(a, l, s, n_sites, [x[0] for x in local], [x[1] for x in local], host_only=True, **kw)


def test_worked_example_host_lookup():
    sites, local, S, recs, exp, g = worked_example()
    reg = _host_reg(sites, local, S)
    assert reg.rows == 2 * S + 3
    q = np.array([ip(a) for a, _ in g["lpm_spot_checks"]], dtype=np.uint32)
    site, loc = reg.lookup_host(q)
    assert site.tolist() == [s for _, s in g["lpm_spot_checks"]]
    site, loc = reg.lookup_host(np.array([ip("198.18.5.1"), ip("198.19.0.0"), ip("198.17.255.255")], np.uint32))
    assert loc.tolist() == [True, False, False]


@pytest.mark.parametrize("layout", ["lines", "wide", "shallow", "wide-shallow"])
@pytest.mark.parametrize("root_bits,list_max", [(8, 2), (8, 8), (12, 4), (14, 2), (14, 8), (10, 3)])
@pytest.mark.parametrize("seed", range(12))
def test_host_trie_matches_oracle_at_every_boundary(seed, root_bits, list_max, layout):
    rng = np.random.default_rng(1000 + seed)
    n_sites, sites, local = random_tiny_registry(rng, n_prefixes=int(rng.integers(0, 60)))
    if layout == "wide" and seed % 3 == 0:
        n_sites = 70000  # site codes beyond 16 bits: no QUAD entries
    node_bits = [0, 4, 6, 8, 12][seed % 5]
    reg = _host_reg(sites, local, n_sites, root_bits=root_bits, list_max=list_max, layout=layout,
                    node_bits=node_bits)
    orc = oracle.Registry([s[0] for s in sites], [s[1] for s in sites], [s[2] for s in sites], n_sites,
                          [x[0] for x in local], [x[1] for x in local])
    pts = np.array(boundary_points(sites + [(a, l, 0) for a, l in local]), dtype=np.uint32)
    site, loc = reg.lookup_host(pts)
    assert site.tolist() == orc.lookup(pts).tolist()
    assert loc.tolist() == [brute.is_local(local, int(p)) for p in pts.tolist()]


@pytest.mark.parametrize("layout", ["auto", "lines", "wide", "shallow", "wide-shallow"])
def test_host_trie_generated_registries(layout):
    import flowgen
    for wl in (flowgen.PLAIN_SMALL, flowgen.PLAIN_LARGE):
        r = flowgen.registry_for(wl)
        reg = gnm.Registry.from_generated(r, host_only=True, layout=layout)
        orc = oracle.Registry.from_generated(r)
        pts = boundary_points(list(zip(r.addr.tolist(), r.length.tolist(), r.site.tolist())))
        pts = np.array(pts, dtype=np.uint32)
        assert (reg.lookup_host(pts)[0] == orc.lookup(pts)).all()
        info = reg.info()
        assert info["n_prefixes"] == r.n_prefixes and info["n_sites"] == r.n_sites
        assert info["n_local_ranges"] == r.n_local


def test_registry_info_counts_normalisation():
    sites = [(ip("10.1.2.3"), 8, 1), (ip("10.0.0.0"), 8, 1), (ip("10.200.0.0"), 16, 0)]
    reg = _host_reg(sites, [(ip("192.168.1.0"), 24), (ip("192.168.0.0"), 16)], 2)
    info = reg.info()
    assert info["n_prefixes_in"] == 3 and info["n_prefixes"] == 2
    assert info["n_host_bits"] == 1 and info["n_duplicates"] == 1
    assert info["n_local_ranges"] == 1  # nested local prefixes merge
    assert info["n_intervals"] == 5     # none | 10/8 | 10.200/16 | 10/8 | none


@pytest.mark.parametrize("sites,n_sites,local,code", [
    ([(ip("10.0.0.0"), 8, 0), (ip("10.9.9.9"), 8, 1)], 2, [], gnm.GNM_E_CONFLICT),
    ([(ip("10.0.0.0"), 33, 0)], 1, [], gnm.GNM_E_INVAL),
    ([(ip("10.0.0.0"), 8, 2)], 2, [], gnm.GNM_E_INVAL),
    ([], 0, [], gnm.GNM_E_INVAL),
    ([], 1, [(ip("10.0.0.0"), 40)], gnm.GNM_E_INVAL),
    ([], 1, [(i << 20, 12) for i in range(0, 66, 2)], gnm.GNM_E_UNSUPPORTED),
])
def test_registry_errors(sites, n_sites, local, code):
    with pytest.raises(gnm.GnmError) as e:
        _host_reg(sites, local, n_sites)
    assert e.value.code == code


def test_build_option_errors():
    for kw in (dict(root_bits=7), dict(root_bits=15), dict(list_max=1), dict(list_max=9), dict(node_bits=3),
               dict(node_bits=17), dict(lds_bytes=163840 + 16)):
        with pytest.raises(gnm.GnmError) as e:
            _host_reg([], [], 1, **kw)
        assert e.value.code == gnm.GNM_E_INVAL


def test_workspace_size_formula():
    reg = _host_reg([(ip("10.0.0.0"), 8, 0)], [], 5)
    rows = reg.rows
    assert rows == 2 * 6 + 1
    for grid in (1, 7, 256):
        need = grid * 7 * rows * 8 + ((grid * 4 + 255) // 256) * 256
        assert gnm.workspace_bytes(reg, grid) == need
    assert gnm.workspace_bytes(reg) >= gnm.workspace_bytes(reg, 1)
    assert gnm.lib().gnm_workspace_bytes(None, 3) == 0


def test_device_calls_reject_host_only_registry_and_nulls():
    L = gnm.lib()
    reg = _host_reg([(ip("10.0.0.0"), 8, 0)], [], 1)
    rec = gnm.RecordsC()
    p = L.gnm_params_default()
    rc = L.gnm_classify_aggregate(reg.handle, ctypes.byref(rec), None, 1, ctypes.byref(p), ctypes.c_void_p(8), None)
    assert rc == gnm.GNM_E_UNSUPPORTED
    rc = L.gnm_flag_suboptimal(reg.handle, ctypes.c_void_p(8), 1, 10, 0, ctypes.c_void_p(8), None)
    assert rc == gnm.GNM_E_UNSUPPORTED
    assert L.gnm_classify_aggregate(None, ctypes.byref(rec), None, 1, None, ctypes.c_void_p(8), None) == gnm.GNM_E_INVAL
    assert L.gnm_flag_suboptimal(None, None, 1, 1, 0, None, None) == gnm.GNM_E_INVAL
    rc = L.gnm_classify_flag(reg.handle, ctypes.byref(rec), None, 1, ctypes.byref(p), ctypes.c_void_p(8), 10, 0,
                             ctypes.c_void_p(8), None)
    assert rc == gnm.GNM_E_UNSUPPORTED
    rc = L.gnm_classify_flag(reg.handle, ctypes.byref(rec), None, 1, ctypes.byref(p), ctypes.c_void_p(8), 10, 0,
                             None, None)
    assert rc == gnm.GNM_E_INVAL
    assert L.gnm_classify_flag(None, ctypes.byref(rec), None, 1, None, ctypes.c_void_p(8), 10, 0,
                               ctypes.c_void_p(8), None) == gnm.GNM_E_INVAL
    assert L.gnm_acc_rows(None) == 0
    assert L.gnm_registry_free(None) == 0
    reg.close()


def test_host_trie_large_table():
    """1,000,000 BGP-like prefixes over 20,000 sites, in the automatic layout
    (12-bit first-level nodes) and in the 8-bit shallow one (leaf lines below
    the first level); every boundary agrees with the oracle."""
    import flowgen
    r = flowgen.registry_for(flowgen.LARGE_TABLE)
    reg = gnm.Registry.from_generated(r, host_only=True)
    orc = oracle.Registry.from_generated(r)
    info = reg.info()
    assert info["n_prefixes"] == 1_000_000 and info["n_sites"] == 20_000
    assert info["acc_in_lds"] == 0  # 40,003 rows do not fit
    assert info["node_bits"] == 12 and info["cache_slots"] > 1000
    pts = np.array(boundary_points(list(zip(r.addr.tolist(), r.length.tolist(), r.site.tolist()))), dtype=np.uint32)
    assert (reg.lookup_host(pts)[0] == orc.lookup(pts)).all()
    loc = reg.lookup_host(pts)[1]
    from tests._helpers import is_local_np
    assert (loc == is_local_np(r, pts)).all()
    shallow = gnm.Registry.from_generated(r, host_only=True, layout="shallow", node_bits=8)
    assert shallow.info()["n_leaf_lines"] > 0
    assert (shallow.lookup_host(pts)[0] == orc.lookup(pts)).all()


@pytest.mark.parametrize("root_bits,node_bits", [(8, 16), (14, 16), (8, 4), (12, 5)])
def test_host_trie_node_bits_extremes(root_bits, node_bits):
    rng = np.random.default_rng(4242 + node_bits + root_bits)
    n_sites, sites, local = random_tiny_registry(rng, n_prefixes=40)
    reg = _host_reg(sites, local, n_sites, root_bits=root_bits, node_bits=node_bits, layout="wide")
    assert reg.info()["node_bits"] == min(node_bits, 32 - root_bits)
    orc = oracle.Registry([s[0] for s in sites], [s[1] for s in sites], [s[2] for s in sites], n_sites,
                          [x[0] for x in local], [x[1] for x in local])
    pts = np.array(boundary_points(sites + [(a, l, 0) for a, l in local]), dtype=np.uint32)
    assert reg.lookup_host(pts)[0].tolist() == orc.lookup(pts).tolist()


def test_automatic_first_level_width():
    import flowgen
    for wl in (flowgen.PLAIN_LARGE, flowgen.LARGE_TABLE):
        info = gnm.Registry.from_generated(flowgen.registry_for(wl), host_only=True).info()
        assert info["node_bits"] == 12


def test_filter_params_checked():
    p = gnm.make_params(filters={"min_avg_packet_bytes": 100, "min_packets": 2, "min_duration_ms": 3})
    assert (p.min_avg_packet_bytes, p.min_packets, p.min_duration_ms) == (100, 2, 3)
    assert gnm.make_params().min_packets == 0
    with pytest.raises(ValueError):
        gnm.make_params(filters={"min_packets": 2**32})
    with pytest.raises(ValueError):
        gnm.make_params(filters={"max_packets": 1})
    assert set(gnm.FILTER_KEYS) == set(oracle.FILTER_KEYS)


def test_new_binding_arguments_checked_on_the_host():
    with pytest.raises(ValueError):
        gnm.HostTable(None, -1, 1000)  # a negative capacity, rejected before any allocation
    with pytest.raises(ValueError):
        gnm.make_params(hosts=object())
    with pytest.raises(ValueError):
        gnm.make_params(filters={"min_packets": -1})
    assert gnm.RATE_BUCKETS == 10001 and gnm.RATE_BUCKET_BPS == 10_000
    assert gnm.RATE_BUCKETS == oracle.RATE_BUCKETS and gnm.NO_MEDIAN == oracle.NO_MEDIAN
    # the workspace of the v5 decode grows with the datagram count, from a fixed floor
    w0, w1 = gnm.netflow_v5_workspace_bytes(0), gnm.netflow_v5_workspace_bytes(1000)
    assert w0 > 0 and w1 >= w0 + 1000 * 12


def test_gnm_params_layout_matches_header():
    # the binding's structure must match the C one field for field: the library
    # fills the defaults through it
    p = gnm.lib().gnm_params_default()
    assert p.bulk_bytes == 1_000_000 and p.flags == 0 and not p.rate_hist and not p.hosts
    assert (p.min_avg_packet_bytes, p.min_packets, p.min_duration_ms) == (0, 0, 0)
    assert ctypes.sizeof(gnm.Params) == 8 + 4 * 4 + 8 + 8 + 8 + 4 * 4 + 8


def test_host_work_bytes():
    # two staged copies of a 32-byte entry per record, plus per-workgroup partition counts
    reg = gnm.Registry([0x0B000000], [8], [0], 1, [0x0A000000], [16], host_only=True)
    assert gnm.host_work_bytes(reg, 0, 256) > 0
    for n in (1, 1000, 10_000_000):
        w1, w2 = gnm.host_work_bytes(reg, n, 256), gnm.host_work_bytes(reg, n, 512)
        assert 64 * n <= w1 < w2 <= 64 * n + 512 * 4 * 16384 + 8 * 16384 + 4096
    assert gnm.lib().gnm_host_work_bytes(None, 100, 1) == 0


def test_workspace_bytes_hist():
    # the tables' part rounded up to 256 bytes, then about 8 bytes per record
    # (keys staged, then in partition order) plus the count matrix; the tables'
    # part alone beyond 65,536 rows over all windows
    reg = gnm.Registry([0x0B000000, 0x0C000000], [8, 8], [0, 1], 2, [0x0A000000], [16], host_only=True)
    rows = 2 * reg.n_sites
    for n, nw, grid in ((1, 1, 1), (1000, 3, 7), (10_000_000, 8, 256), (10_000_000, 1, 512)):
        base = (gnm.workspace_bytes_n(reg, n, nw, grid) + 255) // 256 * 256
        w = gnm.workspace_bytes_hist(reg, n, nw, grid)
        parts = (nw * rows + 63) // 64 * 64
        assert base + 8 * n <= w <= base + 8 * n + 4 * grid * parts + 4 * (n // 16384 + 1) + 16 * 256, (n, nw, grid)
    big = 65536 // rows + 1  # windows past the staged limit
    assert gnm.workspace_bytes_hist(reg, 1000, big, 4) == (gnm.workspace_bytes_n(reg, 1000, big, 4) + 255) // 256 * 256
    assert gnm.lib().gnm_workspace_bytes_hist(None, 100, 1, 1) == 0
    assert gnm.workspace_bytes_hist(reg, 100, 0, 1) == 0
