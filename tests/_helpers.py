"""Small helpers shared by tests (no method arithmetic)."""
import ipaddress
import json
import os

import numpy as np

M64 = (1 << 64) - 1
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def ip(s: str) -> int:
    return int(ipaddress.IPv4Address(s))


def load_golden(name: str):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def worked_example():
    """(sites, local, n_sites, records-as-tuples, expected rows, golden dict)."""
    g = load_golden("worked_example.json")
    sites = [(ip(a), l, s) for a, l, s in g["sites"]]
    local = [(ip(a), l) for a, l in g["local"]]
    recs = [(ip(r[0]), ip(r[1]), r[2], r[3], r[4], r[5]) for r in g["records"]]
    exp = [[M64 if v == "MAX" else v for v in r] for r in g["expected_rows"]]
    return sites, local, g["n_sites"], recs, exp, g


def soa(records):
    """Tuples (src, dst, bytes, packets, first, last) -> flowgen.Records."""
    import flowgen
    a = np.array(records, dtype=object).reshape(-1, 6) if records else np.zeros((0, 6), dtype=object)
    n = a.shape[0]
    return flowgen.Records(
        src_ip=a[:, 0].astype(np.uint32), dst_ip=a[:, 1].astype(np.uint32),
        src_port=np.zeros(n, np.uint16), dst_port=np.zeros(n, np.uint16), proto=np.zeros(n, np.uint8),
        bytes=np.array([int(x) for x in a[:, 2]], dtype=np.uint64),
        packets=a[:, 3].astype(np.uint32), first_ms=a[:, 4].astype(np.uint32),
        last_ms=a[:, 5].astype(np.uint32))


def tuples(rec, lo=0, hi=None):
    hi = rec.n if hi is None else hi
    return list(zip(rec.src_ip[lo:hi].tolist(), rec.dst_ip[lo:hi].tolist(), rec.bytes[lo:hi].tolist(),
                    rec.packets[lo:hi].tolist(), rec.first_ms[lo:hi].tolist(), rec.last_ms[lo:hi].tolist()))


def random_tiny_registry(rng, n_sites=None, n_prefixes=None, n_local=None):
    """Tiny random registry with nesting, duplicates of the same site and /0../32."""
    n_sites = n_sites or int(rng.integers(1, 6))
    n_prefixes = n_prefixes if n_prefixes is not None else int(rng.integers(0, 33))
    out = []
    for _ in range(n_prefixes):
        L = int(rng.integers(0, 33)) if rng.random() < 0.3 else int(rng.integers(8, 33))
        if out and rng.random() < 0.5:  # nest inside an existing prefix
            pa, pl, _ = out[int(rng.integers(0, len(out)))]
            L = max(L, pl)
            a = pa | (int(rng.integers(0, 1 << 32)) & ~(0 if pl == 0 else (0xFFFFFFFF << (32 - pl))) & 0xFFFFFFFF)
        else:
            a = int(rng.integers(0, 1 << 32))
        out.append((a & 0xFFFFFFFF, L, int(rng.integers(0, n_sites))))
    # resolve conflicts: a (net, len) keeps its first site
    seen = {}
    clean = []
    for a, L, s in out:
        m = 0 if L == 0 else (0xFFFFFFFF << (32 - L)) & 0xFFFFFFFF
        k = (a & m, L)
        if k in seen:
            s = seen[k]
        seen[k] = s
        clean.append((a, L, s))
    nl = n_local if n_local is not None else int(rng.integers(0, 4))
    local = [(int(rng.integers(0, 1 << 32)), int(rng.integers(0, 33))) for _ in range(nl)]
    return n_sites, clean, local


def boundary_points(prefixes):
    """Every point where a longest-prefix-match answer can change, and its neighbours."""
    pts = {0, 0xFFFFFFFF}
    for a, L, _ in prefixes:
        m = 0 if L == 0 else (0xFFFFFFFF << (32 - L)) & 0xFFFFFFFF
        lo = a & m
        hi = lo | (~m & 0xFFFFFFFF)
        for p in (lo - 1, lo, lo + 1, hi - 1, hi, hi + 1):
            if 0 <= p <= 0xFFFFFFFF:
                pts.add(p)
    return sorted(pts)


def is_local_np(reg, ips):
    """Locality of addresses against a generated registry's local prefixes (vectorised)."""
    ips = np.asarray(ips, dtype=np.uint64)
    out = np.zeros(ips.shape[0], dtype=bool)
    for a, L in zip(reg.local_addr.tolist(), reg.local_len.tolist()):
        m = 0 if L == 0 else (0xFFFFFFFF << (32 - L)) & 0xFFFFFFFF
        out |= (ips & np.uint64(m)) == np.uint64(a & m)
    return out


def median_example():
    """The hand-worked median example: (sites, local, n_sites, records, offsets, golden dict)."""
    g = load_golden("median_example.json")
    sites = [(ip(a), l, s) for a, l, s in g["sites"]]
    local = [(ip(a), l) for a, l in g["local"]]
    recs = [(ip(r[0]), ip(r[1]), r[2], r[3], r[4], r[5]) for r in g["records"]]
    off = np.array(g["window_offsets"], dtype=np.uint64)
    return sites, local, g["n_sites"], recs, off, g


def dense_histograms(g, rows: int) -> np.ndarray:
    """The golden's sparse (row, bucket, count) lists as uint32[n_windows, rows, 10001]."""
    out = np.zeros((len(g["expected_histograms"]), rows, 10001), dtype=np.uint32)
    for w, entries in enumerate(g["expected_histograms"]):
        for r, b, c in entries:
            out[w, r, b] = c
    return out
