"""Seeded synthetic inputs for the flow classify/aggregate path.

This module only draws random inputs: site registries (CIDR prefixes mapped
to collaboration sites), local-site prefix sets, and windows of NetFlow-style
flow records in structure-of-arrays form.  It holds none of the method's
arithmetic (no prefix matching, no rates, no aggregation), so both the CPU
oracle and the GPU library can be fed from it without sharing any of the
computation.

The workloads stand in for the paper's measurement data, which is not
available: real border-router NetFlow v5 records (§IV.A: 50 million records,
100 registered /24 subnets).  Distributions follow the recipe written down in
the design notes: heavy-tailed (lognormal) byte counts, uniform durations up
to five minutes, Zipf-distributed site popularity, 90 % of records with one
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
