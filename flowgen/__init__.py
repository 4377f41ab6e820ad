"""Seeded synthetic inputs for the flow classify/aggregate path.

This module only draws random inputs: site registries (CIDR prefixes mapped
to collaboration sites), local-site prefix sets, and windows of NetFlow-style
flow records in structure-of-arrays form.  It holds none of the method's
arithmetic (no prefix matching, no rates, no aggregation), so both the CPU
oracle and the GPU library can be fed from it without sharing any of the
computation.

The workloads stand in for the paper's measurement data, which is not
available: real border-router NetFlow v5 records (§IV.A: 50 million records,
100 registered /24 subnets).  Distributions follow one fixed recipe:
heavy-tailed (lognormal) byte counts, uniform durations up to five minutes, Zipf-distributed site popularity, 90 % of records with one
local endpoint and 10 % of remote endpoints outside every registered site.

All arrays are little-endian numpy arrays.  IPv4 addresses are host-order
uint32 with the first octet in the most significant byte.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Optional

import numpy as np

SEED_BASE = 1108_1785

# Named workloads (record counts and registry shapes); see WORKLOADS below.
PLAIN_SMALL = "plain-small"       # 100 k records, 64 sites / 512 prefixes
PLAIN_LARGE = "plain-large"       # 10 M records, 1,000 sites / 20,000 prefixes
BATCHED = "batched-256"           # 256 windows of 10 k - 2 M records, small registry
SERVED = "served-stream"          # Poisson window arrivals, small registry
LARGE_TABLE = "large-table"       # 100 M records, 20,000 sites / 1,000,000 prefixes

_SEED_INDEX = {PLAIN_SMALL: 1, PLAIN_LARGE: 2, BATCHED: 3, SERVED: 4, LARGE_TABLE: 5}

U32 = np.uint32
NO_SITE_BASE = 0xF0000000          # remote addresses outside every site: 240.0.0.0/4
SITE_OCTET_LO, SITE_OCTET_HI = 11, 223  # first octet of generated site prefixes
LOCAL_OCTET = 10                   # local prefixes are 10.x.0.0/16


@dataclasses.dataclass
class Registry:
    """Site registry plus local-prefix set (host arrays)."""
    addr: np.ndarray        # uint32[n_prefixes]  network address (host bits clear)
    length: np.ndarray      # uint32[n_prefixes]  prefix length 0..32
    site: np.ndarray        # uint32[n_prefixes]  site id < n_sites
    n_sites: int
    local_addr: np.ndarray  # uint32[n_local]
    local_len: np.ndarray   # uint32[n_local]
    # generator bookkeeping (not part of the method's input)
    site_prefix_start: np.ndarray = None   # int64[n_sites+1] CSR over prefixes sorted by site
    site_prefix_order: np.ndarray = None   # int64[n_prefixes] prefix indices grouped by site
    rank_to_site: np.ndarray = None        # int64[n_sites] popularity rank -> site id

    @property
    def n_prefixes(self) -> int:
        return int(self.addr.shape[0])

    @property
    def n_local(self) -> int:
        return int(self.local_addr.shape[0])


@dataclasses.dataclass
class Records:
    """A run of flow records in SoA form; windows are contiguous slices."""
    src_ip: np.ndarray     # uint32
    dst_ip: np.ndarray     # uint32
    src_port: np.ndarray   # uint16 (not read by the path)
    dst_port: np.ndarray   # uint16 (not read by the path)
    proto: np.ndarray      # uint8  (not read by the path)
    bytes: np.ndarray      # uint64
    packets: np.ndarray    # uint32
    first_ms: np.ndarray   # uint32
    last_ms: np.ndarray    # uint32
    window_offsets: Optional[np.ndarray] = None  # uint64[n_windows+1], None = one window

    FIELDS = ("src_ip", "dst_ip", "src_port", "dst_port", "proto",
              "bytes", "packets", "first_ms", "last_ms")

    @property
    def n(self) -> int:
        return int(self.src_ip.shape[0])

    def slice(self, lo: int, hi: int) -> "Records":
        return Records(*(getattr(self, f)[lo:hi] for f in self.FIELDS))

    def copy(self) -> "Records":
        r = Records(*(np.array(getattr(self, f)) for f in self.FIELDS))
        r.window_offsets = None if self.window_offsets is None else np.array(self.window_offsets)
        return r

    def window(self, w: int) -> "Records":
        off = self.window_offsets
        return self.slice(int(off[w]), int(off[w + 1]))

    @property
    def n_windows(self) -> int:
        return 1 if self.window_offsets is None else int(self.window_offsets.shape[0] - 1)


def _mask(length: np.ndarray) -> np.ndarray:
    """Network mask per prefix length, vectorised (length 0 -> 0)."""
    length = np.asarray(length, dtype=np.uint64)
    m = (np.uint64(0xFFFFFFFF) << (np.uint64(32) - length)) & np.uint64(0xFFFFFFFF)
    return np.where(length == 0, np.uint64(0), m).astype(U32)


def zipf_probs(n: int, s: float = 1.2) -> np.ndarray:
    """Truncated Zipf(s) over ranks 1..n."""
    p = np.arange(1, n + 1, dtype=np.float64) ** (-s)
    return p / p.sum()


def _random_prefixes(rng, lengths: np.ndarray) -> np.ndarray:
    """Random network addresses for the given lengths, first octet in 11..223."""
    n = lengths.shape[0]
    octet = rng.integers(SITE_OCTET_LO, SITE_OCTET_HI + 1, size=n, dtype=np.uint64)
    low = rng.integers(0, 1 << 24, size=n, dtype=np.uint64)
    a = ((octet << np.uint64(24)) | low).astype(U32)
    return a & _mask(lengths)


def _nested_prefixes(rng, lengths, parent_addr, parent_len) -> np.ndarray:
    """Addresses for prefixes placed inside a random strictly shorter parent."""
    out = np.empty(lengths.shape[0], dtype=U32)
    order = np.argsort(parent_len, kind="stable")
    plen_sorted = parent_len[order]
    for L in np.unique(lengths):
        sel = np.nonzero(lengths == L)[0]
        k = int(np.searchsorted(plen_sorted, L, side="left"))  # parents with len < L
        if k == 0:
            out[sel] = _random_prefixes(rng, lengths[sel])
            continue
        pick = order[rng.integers(0, k, size=sel.shape[0])]
        pa = parent_addr[pick]
        pl = parent_len[pick]
        host = rng.integers(0, 1 << 32, size=sel.shape[0], dtype=np.uint64).astype(U32)
        a = pa | (host & ~_mask(pl))
        out[sel] = a & _mask(np.full(sel.shape[0], L))
    return out


def _distinct(addr: np.ndarray, length: np.ndarray) -> np.ndarray:
    """Index of first occurrence of each distinct (addr, len) pair, in order."""
    key = (addr.astype(np.uint64) << np.uint64(6)) | length.astype(np.uint64)
    _, first = np.unique(key, return_index=True)
    return np.sort(first)


def _make_prefix_set(rng, n: int, length_sampler, nested_frac: float):
    """n distinct (addr, len) prefixes; a fraction nested inside shorter ones."""
    addr = np.empty(0, dtype=U32)
    length = np.empty(0, dtype=U32)
    n_top = n - int(round(nested_frac * n))
    while addr.shape[0] < n_top:
        need = n_top - addr.shape[0]
        L = length_sampler(rng, need + need // 8 + 16)
        a = _random_prefixes(rng, L)
        addr = np.concatenate([addr, a])
        length = np.concatenate([length, L])
        keep = _distinct(addr, length)[:n_top]
        addr, length = addr[keep], length[keep]
    while addr.shape[0] < n:
        need = n - addr.shape[0]
        L = length_sampler(rng, need + need // 8 + 16)
        a = _nested_prefixes(rng, L, addr, length)
        addr2 = np.concatenate([addr, a])
        len2 = np.concatenate([length, L])
        keep = _distinct(addr2, len2)
        keep = keep[:n]
        addr, length = addr2[keep], len2[keep]
    perm = rng.permutation(n)
    return addr[perm], length[perm]


def _uniform_lengths(lo: int, hi: int):
    def f(rng, k):
        return rng.integers(lo, hi + 1, size=k).astype(U32)
    return f


def _plain_large_lengths(rng, k):
    # /24 at 50 %; /16-/23 and /25-/28 at 48 % spread evenly over 12 lengths;
    # /8-/15 at 2 %.
    u = rng.random(k)
    mid = np.concatenate([np.arange(16, 24), np.arange(25, 29)])
    out = np.full(k, 24, dtype=U32)
    m = (u >= 0.50) & (u < 0.98)
    out[m] = mid[rng.integers(0, mid.shape[0], size=int(m.sum()))]
    s = u >= 0.98
    out[s] = rng.integers(8, 16, size=int(s.sum()))
    return out


def _bgp_lengths(rng, k):
    # /24 at 60 %; /16-/23 at 35 % uniform; /25-/32 at 4 % uniform;
    # /8-/15 at 1 % weighted by 2**(len-8) (long ones are more common).
    u = rng.random(k)
    out = np.full(k, 24, dtype=U32)
    m = (u >= 0.60) & (u < 0.95)
    out[m] = rng.integers(16, 24, size=int(m.sum()))
    m = (u >= 0.95) & (u < 0.99)
    out[m] = rng.integers(25, 33, size=int(m.sum()))
    m = u >= 0.99
    w = 2.0 ** np.arange(0, 8)
    out[m] = 8 + rng.choice(8, size=int(m.sum()), p=w / w.sum())
    return out


def _local_set(rng, n_local: int):
    x = rng.choice(256, size=n_local, replace=False).astype(np.uint64)
    addr = ((np.uint64(LOCAL_OCTET) << np.uint64(24)) | (x << np.uint64(16))).astype(U32)
    return addr, np.full(n_local, 16, dtype=U32)


def _finish_registry(rng, addr, length, n_sites, local_addr, local_len) -> Registry:
    n = addr.shape[0]
    # prefix i belongs to site perm[i mod n_sites]: every site gets n/n_sites prefixes
    site_of_slot = rng.permutation(n_sites)
    site = site_of_slot[np.arange(n) % n_sites].astype(U32)
    order = np.argsort(site, kind="stable")
    counts = np.bincount(site, minlength=n_sites)
    start = np.zeros(n_sites + 1, dtype=np.int64)
    np.cumsum(counts, out=start[1:])
    rank_to_site = rng.permutation(n_sites)
    return Registry(addr=addr, length=length, site=site, n_sites=n_sites,
                    local_addr=local_addr, local_len=local_len,
                    site_prefix_start=start, site_prefix_order=order.astype(np.int64),
                    rank_to_site=rank_to_site.astype(np.int64))


def make_registry(n_sites: int, n_prefixes: int, length_sampler, n_local: int,
                  rng, nested_frac: float = 0.25) -> Registry:
    local_addr, local_len = _local_set(rng, n_local)
    addr, length = _make_prefix_set(rng, n_prefixes, length_sampler, nested_frac)
    return _finish_registry(rng, addr, length, n_sites, local_addr, local_len)


def _seeds(workload: str):
    ss = np.random.SeedSequence(SEED_BASE + _SEED_INDEX[workload])
    reg_ss, rec_ss = ss.spawn(2)
    return reg_ss, rec_ss


def registry_for(workload: str) -> Registry:
    """The registry a named workload uses (batched/served share plain-small's)."""
    if workload in (BATCHED, SERVED):
        workload = PLAIN_SMALL
    reg_ss, _ = _seeds(workload)
    rng = np.random.Generator(np.random.PCG64(reg_ss))
    if workload == PLAIN_SMALL:
        return make_registry(64, 512, _uniform_lengths(12, 24), 4, rng)
    if workload == PLAIN_LARGE:
        return make_registry(1000, 20000, _plain_large_lengths, 8, rng)
    if workload == LARGE_TABLE:
        return make_registry(20000, 1_000_000, _bgp_lengths, 8, rng)
    raise ValueError(workload)


class SiteSampler:
    """Draws site popularity ranks (then ids) for remote endpoints."""

    def __init__(self, n_sites: int, kind: str = "zipf", s: float = 1.2,
                 top: int = 10, top_share: float = 0.7):
        self.n_sites, self.kind = n_sites, kind
        if kind == "zipf":
            self.cdf = np.cumsum(zipf_probs(n_sites, s))
        elif kind == "top-heavy":
            # with prob top_share a Zipf rank within the first `top`, else within the rest
            self.top, self.top_share = top, top_share
            self.cdf_top = np.cumsum(zipf_probs(top, s))
            self.cdf_rest = np.cumsum(zipf_probs(n_sites - top, s))
        else:
            raise ValueError(kind)

    def ranks(self, rng, k: int) -> np.ndarray:
        if self.kind == "zipf":
            r = np.searchsorted(self.cdf, rng.random(k) * self.cdf[-1], side="right")
            return np.minimum(r, self.n_sites - 1)
        top = rng.random(k) < self.top_share
        r_top = np.minimum(np.searchsorted(self.cdf_top, rng.random(k) * self.cdf_top[-1], side="right"), self.top - 1)
        r_rest = self.top + np.minimum(np.searchsorted(self.cdf_rest, rng.random(k) * self.cdf_rest[-1], side="right"),
                                       self.n_sites - self.top - 1)
        return np.where(top, r_top, r_rest)


def sampler_for(workload: str, reg: Registry) -> SiteSampler:
    if workload == PLAIN_LARGE:
        return SiteSampler(reg.n_sites, "top-heavy")
    return SiteSampler(reg.n_sites, "zipf")


def _remote_addresses(rng, reg: Registry, sampler: SiteSampler, k: int,
                      p_site: float = 0.9) -> np.ndarray:
    out = np.empty(k, dtype=U32)
    hit = rng.random(k) < p_site
    nh = int(hit.sum())
    site = reg.rank_to_site[sampler.ranks(rng, nh)]
    cnt = reg.site_prefix_start[site + 1] - reg.site_prefix_start[site]
    j = reg.site_prefix_start[site] + (rng.random(nh) * cnt).astype(np.int64)
    j = np.minimum(j, reg.site_prefix_start[site + 1] - 1)
    p = reg.site_prefix_order[j]
    pa, pl = reg.addr[p], reg.length[p]
    host = rng.integers(0, 1 << 32, size=nh, dtype=np.uint64).astype(U32)
    out[hit] = pa | (host & ~_mask(pl))
    nm = k - nh
    out[~hit] = (NO_SITE_BASE | rng.integers(0, 1 << 28, size=nm, dtype=np.uint64)).astype(U32)
    return out


def make_records(rng, reg: Registry, sampler: SiteSampler, n: int,
                 p_local: float = 0.9, bytes_cap: int = 1 << 40,
                 max_dur_ms: int = 300_000) -> Records:
    """n flow records drawn from the recipe (one window)."""
    one_local = rng.random(n) < p_local
    src_is_local = rng.random(n) < 0.5
    li = rng.integers(0, reg.n_local, size=n)
    local = (reg.local_addr[li] | (rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(U32)
                                   & ~_mask(reg.local_len[li]))).astype(U32)
    rem_a = _remote_addresses(rng, reg, sampler, n)
    rem_b = _remote_addresses(rng, reg, sampler, n)
    src = np.where(one_local & src_is_local, local, rem_a)
    dst = np.where(one_local & ~src_is_local, local, np.where(one_local, rem_a, rem_b))
    b = np.floor(rng.lognormal(11.0, 3.0, size=n))
    b = np.clip(b, 1, float(bytes_cap)).astype(np.uint64)
    dur = rng.integers(0, max_dur_ms + 1, size=n, dtype=np.uint64)
    first = rng.integers(0, 1 << 32, size=n, dtype=np.uint64)
    last = ((first + dur) & np.uint64(0xFFFFFFFF)).astype(U32)
    size = rng.uniform(40.0, 1500.0, size=n)
    pk = np.ceil(b.astype(np.float64) / size)
    pk = np.clip(pk, 1, 0xFFFFFFFF).astype(U32)
    sport = rng.integers(0, 1 << 16, size=n, dtype=np.uint32).astype(np.uint16)
    dport = rng.integers(0, 1 << 16, size=n, dtype=np.uint32).astype(np.uint16)
    proto = np.where(rng.random(n) < 0.9, 6, 17).astype(np.uint8)
    return Records(src_ip=src.astype(U32), dst_ip=dst.astype(U32), src_port=sport, dst_port=dport,
                   proto=proto, bytes=b, packets=pk, first_ms=first.astype(U32), last_ms=last)


def records_for(workload: str, reg: Optional[Registry] = None, n: Optional[int] = None,
                stream: int = 0) -> Records:
    """Records of a named workload.

    n overrides the record count (parity tests use smaller runs of the same
    distributions); `stream` selects an independent seeded copy (used to rotate
    distinct windows through a timed loop).
    """
    if reg is None:
        reg = registry_for(workload)
    _, rec_ss = _seeds(workload)
    ss = rec_ss.spawn(stream + 1)[stream]
    rng = np.random.Generator(np.random.PCG64(ss))
    sampler = sampler_for(workload, reg)
    if workload == PLAIN_SMALL:
        return make_records(rng, reg, sampler, 100_000 if n is None else n)
    if workload == PLAIN_LARGE:
        return make_records(rng, reg, sampler, 10_000_000 if n is None else n)
    if workload == LARGE_TABLE:
        return make_records(rng, reg, sampler, 100_000_000 if n is None else n)
    if workload == BATCHED:
        return batched_records(rng, reg, sampler, 256, 10_000, 2_000_000, total_cap=n)
    raise ValueError(workload)


def window_sizes(rng, n_windows: int, lo: int, hi: int) -> np.ndarray:
    return rng.integers(lo, hi + 1, size=n_windows).astype(np.int64)


def batched_records(rng, reg: Registry, sampler: SiteSampler, n_windows: int,
                    lo: int, hi: int, total_cap: Optional[int] = None) -> Records:
    """Concatenated windows of uneven size; total_cap scales sizes down for tests."""
    sizes = window_sizes(rng, n_windows, lo, hi)
    if total_cap is not None and sizes.sum() > total_cap:
        sizes = np.maximum(sizes * total_cap // max(int(sizes.sum()), 1), 0)
    off = np.zeros(n_windows + 1, dtype=np.uint64)
    np.cumsum(sizes, out=off[1:])
    rec = make_records(rng, reg, sampler, int(off[-1]))
    rec.window_offsets = off
    return rec


def served_sizes(rng, n: int, median: float = 300_000.0, sigma: float = 1.0,
                 cap: int = 5_000_000) -> np.ndarray:
    """Window sizes for the served stream: lognormal around the median, clamped."""
    s = np.floor(rng.lognormal(np.log(median), sigma, size=n))
    return np.clip(s, 1, cap).astype(np.int64)


def poisson_arrivals(rng, rate_hz: float, duration_s: float) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process."""
    n_est = int(rate_hz * duration_s * 1.5) + 16
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=n_est))
    return t[t < duration_s]


def concat(parts) -> Records:
    """Concatenate record runs into one batch with window offsets."""
    parts = list(parts)
    off = np.zeros(len(parts) + 1, dtype=np.uint64)
    np.cumsum([p.n for p in parts], out=off[1:])
    rec = Records(*(np.concatenate([getattr(p, f) for p in parts]) for f in Records.FIELDS))
    rec.window_offsets = off
    return rec


def permuted(rec: Records, rng) -> Records:
    """Same records in a random order (single window)."""
    perm = rng.permutation(rec.n)
    return Records(*(getattr(rec, f)[perm] for f in Records.FIELDS))


# ---------------------------------------------------------------- NetFlow v5 datagrams
#
# Export datagrams in the public NetFlow version 5 format, which the paper's
# routers send (§III.B.1, FlowData Receiver Thread; §IV.A.3: 48-byte records,
# at most 30 per 1500-byte datagram).  All fields big-endian.  Header, 24 B:
# version u16 (= 5), count u16 (records that follow, 1..30), sys_uptime u32
# (ms), unix_secs u32, unix_nsecs u32, flow_sequence u32, engine_type u8,
# engine_id u8, sampling_interval u16.  Record, 48 B: srcaddr u32, dstaddr
# u32, nexthop u32, input u16, output u16, dPkts u32, dOctets u32, First u32,
# Last u32 (sys_uptime at the first and last packet), srcport u16, dstport
# u16, pad1 u8, tcp_flags u8, prot u8, tos u8, src_as u16, dst_as u16,
# src_mask u8, dst_mask u8, pad2 u16.
V5_HEADER = np.dtype([("version", ">u2"), ("count", ">u2"), ("sys_uptime", ">u4"), ("unix_secs", ">u4"),
                      ("unix_nsecs", ">u4"), ("flow_sequence", ">u4"), ("engine_type", "u1"),
                      ("engine_id", "u1"), ("sampling_interval", ">u2")])
V5_RECORD = np.dtype([("srcaddr", ">u4"), ("dstaddr", ">u4"), ("nexthop", ">u4"), ("input", ">u2"),
                      ("output", ">u2"), ("dPkts", ">u4"), ("dOctets", ">u4"), ("First", ">u4"),
                      ("Last", ">u4"), ("srcport", ">u2"), ("dstport", ">u2"), ("pad1", "u1"),
                      ("tcp_flags", "u1"), ("prot", "u1"), ("tos", "u1"), ("src_as", ">u2"),
                      ("dst_as", ">u2"), ("src_mask", "u1"), ("dst_mask", "u1"), ("pad2", ">u2")])
assert V5_HEADER.itemsize == 24 and V5_RECORD.itemsize == 48
V5_MAX_RECORDS = 30
MALFORMED_KINDS = ("version", "count0", "count31", "truncated", "short", "misaligned")


def v5_records(workload: str, n: int, stream: int = 0) -> Records:
    """Records of a workload's recipe as a router exports them: byte counts fit
    the 32-bit dOctets field (cap 2^32 - 1)."""
    reg = registry_for(workload)
    rng = np.random.Generator(np.random.PCG64([SEED_BASE, _SEED_INDEX[workload], 7, stream]))
    return make_records(rng, reg, sampler_for(workload, reg), n, bytes_cap=0xFFFFFFFF)


def encode_netflow_v5(rec: Records, rng, partial_frac: float = 0.1, malformed: int = 0):
    """Pack records into back-to-back v5 datagrams (uint8 buffer, uint64 offsets[n+1]).

    Most datagrams carry 30 records, a partial_frac share fewer (routers also
    flush partly filled datagrams); `malformed` extra datagrams of the
    MALFORMED_KINDS, which carry none of the records, are mixed in.  Datagram
    starts are multiples of 4 (a misaligned one is preceded by 2 bytes of
    padding in its predecessor's span).
    """
    if int(rec.bytes.max(initial=0)) > 0xFFFFFFFF:
        raise ValueError("NetFlow v5 carries 32-bit byte counts")
    n = rec.n
    counts = []
    left = n
    while left > 0:
        c = V5_MAX_RECORDS if rng.random() >= partial_frac else int(rng.integers(1, V5_MAX_RECORDS))
        c = min(c, left)
        counts.append(c)
        left -= c
    bad_kinds = [MALFORMED_KINDS[int(k)] for k in rng.integers(0, len(MALFORMED_KINDS), size=malformed)]
    bad_at = sorted(int(x) for x in rng.integers(0, len(counts) + 1, size=malformed))
    items = []  # ("ok", first record, count) or ("bad", kind)
    first = 0
    bi = 0
    for d, c in enumerate(counts + [0]):
        while bi < len(bad_at) and bad_at[bi] == d:
            items.append(("bad", bad_kinds[bi]))
            bi += 1
        if d < len(counts):
            items.append(("ok", first, c))
            first += c
    # every well-formed datagram's header and all records, serialised once
    ok = [it for it in items if it[0] == "ok"]
    hdr = np.zeros(len(ok), dtype=V5_HEADER)
    cnt = np.array([it[2] for it in ok], dtype=np.int64)
    seq0 = np.concatenate([[0], np.cumsum(cnt)[:-1]]).astype(np.int64)
    hdr["version"], hdr["count"] = 5, cnt
    hdr["sys_uptime"] = int(rng.integers(0, 1 << 32))
    hdr["unix_secs"], hdr["unix_nsecs"], hdr["flow_sequence"] = 1_300_000_000 + seq0 // 1000, seq0 % 10**9, seq0
    hdr["engine_type"], hdr["engine_id"] = 1, 2
    r = np.zeros(n, dtype=V5_RECORD)
    r["srcaddr"], r["dstaddr"] = rec.src_ip, rec.dst_ip
    r["nexthop"] = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    r["input"], r["output"] = rng.integers(0, 64, size=n), rng.integers(0, 64, size=n)
    r["dPkts"], r["dOctets"] = rec.packets, rec.bytes.astype(np.uint32)
    r["First"], r["Last"] = rec.first_ms, rec.last_ms
    r["srcport"], r["dstport"] = rec.src_port, rec.dst_port
    r["tcp_flags"], r["prot"] = rng.integers(0, 256, size=n), rec.proto
    r["src_as"], r["dst_as"] = rng.integers(0, 1 << 16, size=n), rng.integers(0, 1 << 16, size=n)
    r["src_mask"], r["dst_mask"] = rng.integers(0, 33, size=n), rng.integers(0, 33, size=n)
    hb, rb = memoryview(hdr.tobytes()), memoryview(r.tobytes())
    parts, offsets, pos, k = [], [], 0, 0
    for it in items:
        if it[0] == "ok":
            _, lo, c = it
            offsets.append(pos)
            parts.append(hb[24 * k: 24 * (k + 1)])
            parts.append(rb[48 * lo: 48 * (lo + c)])
            pos += 24 + 48 * c  # a multiple of 8: the next start stays aligned
            k += 1
            continue
        kind = it[1]
        c = int(rng.integers(1, V5_MAX_RECORDS + 1))
        h = np.zeros(1, dtype=V5_HEADER)
        h["version"], h["count"] = 5, c
        body = rng.integers(0, 256, size=48 * c, dtype=np.uint8).tobytes()
        if kind == "version":
            h["version"] = int(rng.choice([1, 7, 9, 0x0500]))
            blob = h.tobytes() + body
        elif kind == "count0":
            h["count"] = 0
            blob = h.tobytes()
        elif kind == "count31":
            h["count"] = int(rng.choice([31, 0xFFFF]))
            blob = h.tobytes() + body
        elif kind == "truncated":
            # cut by a multiple of 4, so that alignment padding cannot restore it
            blob = (h.tobytes() + body)[:24 + 48 * c - 4 * int(rng.integers(1, 12))]
        elif kind == "short":
            blob = h.tobytes()[:4 * int(rng.integers(0, 6))]
        else:  # misaligned: a valid datagram starting 2 bytes past a multiple of 4
            parts.append(b"\0\0")
            pos += 2
            blob = h.tobytes() + body + b"\0\0"
        offsets.append(pos)
        pad = (-(pos + len(blob))) % 4
        parts.append(blob + b"\0" * pad)
        pos += len(blob) + pad
    offsets.append(pos)
    buf = np.frombuffer(b"".join(parts), dtype=np.uint8).copy()
    return buf, np.array(offsets, dtype=np.uint64)
