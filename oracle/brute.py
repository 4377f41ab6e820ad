"""Pure-Python brute-force oracle for tiny inputs.

TEST INFRASTRUCTURE ONLY: imported by the test suite, never by the product
library.  Every quantity is a Python integer, so nothing can overflow or
round; sums are reduced modulo 2**64 at the end, as the row format stores them.

Prefix matching is the sequential search the paper describes for its
non-hash variants (§IV.A.1: registered subnets kept in a list and scanned one
by one), except that the whole list is scanned and the longest containing
prefix wins (reading: full CIDR longest-prefix match over /0../32).
"""
from __future__ import annotations

from fractions import Fraction

M64 = (1 << 64) - 1
IN, OUT = 0, 1


def mask(length: int) -> int:
    """Network mask of a prefix length (length 0 matches every address)."""
    return 0 if length == 0 else (0xFFFFFFFF << (32 - length)) & 0xFFFFFFFF


def contains(addr: int, length: int, ip: int) -> bool:
    return (ip & mask(length)) == (addr & mask(length))


def normalise(prefixes):
    """Clear host bits; drop exact duplicates; raise on a (net, len) claimed by two sites."""
    seen = {}
    for addr, length, site in prefixes:
        if not 0 <= length <= 32:
            raise ValueError("prefix length out of range")
        key = (addr & mask(length), length)
        if key in seen and seen[key] != site:
            raise ValueError("conflict")
        seen[key] = site
    return [(a, l, s) for (a, l), s in seen.items()]


def lpm(prefixes, ip: int, n_sites: int) -> int:
    """Site of the longest registered prefix containing ip, else n_sites."""
    best_len, best_site = -1, n_sites
    for addr, length, site in prefixes:
        if contains(addr, length, ip) and length > best_len:
            best_len, best_site = length, site
    return best_site


def is_local(local, ip: int) -> bool:
    return any(contains(a, l, ip) for a, l in local)


def rate_bps(nbytes: int, dur_ms: int) -> int:
    """floor(bytes * 8 bits * 1000 ms/s / duration_ms), saturated to 2**64-1."""
    return min(nbytes * 8 * 1000 // dur_ms, M64)


def row_of(prefixes, local, n_sites: int, src: int, dst: int) -> int:
    """Row index: 2*site+dir, or NODIR = 2*n_sites+2 unless exactly one endpoint is local."""
    ls, ld = is_local(local, src), is_local(local, dst)
    if ls == ld:
        return 2 * n_sites + 2
    if ld:
        return 2 * lpm(prefixes, src, n_sites) + IN
    return 2 * lpm(prefixes, dst, n_sites) + OUT


def empty_rows(n_sites: int):
    return [[0, 0, 0, 0, 0, 0, M64, 0] for _ in range(2 * n_sites + 3)]


def is_bulk(nbytes: int, packets: int, dur: int, bulk_bytes: int, filters=None) -> bool:
    """Rate eligibility: more than bulk_bytes bytes over a non-zero duration,
    and, when given, the exclusion filters of §III.B.2 taken literally: an
    average packet size nbytes / packets of at least min_avg_packet_bytes
    (reverse-direction pure-ACK flows have small packets; a flow without
    packets has no average and is kept), at least min_packets packets and a
    duration of at least min_duration_ms (administrative exchanges)."""
    f = filters or {}
    if not (nbytes > bulk_bytes and dur > 0):
        return False
    k = f.get("min_avg_packet_bytes", 0)
    if packets > 0 and Fraction(nbytes, packets) < k:
        return False
    return packets >= f.get("min_packets", 0) and dur >= f.get("min_duration_ms", 0)


def classify_aggregate(prefixes, local, n_sites: int, records, bulk_bytes: int, filters=None):
    """records: iterable of (src, dst, bytes, packets, first_ms, last_ms)."""
    prefixes = normalise(prefixes)
    rows = empty_rows(n_sites)
    for src, dst, nbytes, packets, first, last in records:
        r = rows[row_of(prefixes, local, n_sites, src, dst)]
        dur = (last - first) % (1 << 32)
        r[0] += 1
        r[1] += nbytes
        r[2] += packets
        r[3] += dur
        if is_bulk(nbytes, packets, dur, bulk_bytes, filters):
            rate = rate_bps(nbytes, dur)
            r[4] += 1
            r[5] += rate
            r[6] = min(r[6], rate)
            r[7] = max(r[7], rate)
    for r in rows:
        for k in (0, 1, 2, 3, 4, 5):
            r[k] &= M64
    return rows


def flags(rows, n_sites: int, threshold_bps: int, min_bulk_flows: int):
    """Per site: bit d set iff enough bulk flows and mean rate < threshold (strict)."""
    out = []
    need = max(1, min_bulk_flows)
    for s in range(n_sites):
        f = 0
        for d in (IN, OUT):
            r = rows[2 * s + d]
            if r[4] >= need and r[5] // r[4] < threshold_bps:
                f |= 1 << d
        out.append(f)
    return out
