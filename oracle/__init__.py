"""CPU oracle for the flow classify/aggregate path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg import this package; the product library never
does, and shares no code with it.

Two implementations of one definition:
  * `brute`  — pure Python, big integers, linear prefix scan (tiny inputs);
  * `gnm_oracle.c` — plain C with OpenMP over records, exact 128-bit rate,
    per-length sorted tables probed from the longest length down (full sizes).
The second is pinned against the first, against a worked example, closed-form
rate cases and conservation/permutation invariants in the CPU test suite.

Row layout of every result (one row = 8 unsigned 64-bit fields):
  flows, bytes, packets, duration_ms, bulk_flows, rate_sum_bps,
  rate_min_bps (2**64-1 when no bulk flow), rate_max_bps.
Rows are 2*site+dir (dir 0 inbound, 1 outbound) for site 0..S, where S is the
"no registered site" row, then NODIR = 2*S+2.

Median statistic: `rate_histograms` counts each row's bulk-flow rates in
10,001 buckets of 10 kbps; `rate_medians` sorts each row's buckets and takes
the lower median; `median_flags` applies the two-window warning.  They are
pinned against a per-record brute force and `statistics.median_low`, bucket
closed forms and hand-worked flag sequences.

Per-host statistics (`host_stats`): bulk-flow rate statistics per remote
host and direction of the registered sites, pinned against a per-record brute
force and against the site rows they add up to.

NetFlow v5 decode (`oracle.netflow`): the step before the path, datagrams to
SoA records, parsed with `struct`; pinned by a hand-built datagram, the
paper's sizes, a round trip through the generator's numpy encoder and every
kind of malformed datagram.

Exclusion filters (`filters=`, see `BulkRule`): the paper's reverse-ACK and
administrative-flow exclusions as optional thresholds on rate eligibility,
pinned against the brute force (which compares the exact rational average
packet size) and boundary closed forms.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

from . import brute  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gnm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, E_INVAL, E_CONFLICT, E_NOMEM = 0, -1, -2, -3
M64 = (1 << 64) - 1
FIELDS = ("flows", "bytes", "packets", "duration_ms", "bulk_flows",
          "rate_sum_bps", "rate_min_bps", "rate_max_bps")


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _LIB if os.path.exists(_LIB) else build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        L.orc_registry_build.argtypes = [P, P, P, ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(P)]
        L.orc_registry_build.restype = ctypes.c_int
        L.orc_registry_free.argtypes = [P]
        L.orc_lookup.argtypes = [P, ctypes.c_uint32]
        L.orc_lookup.restype = ctypes.c_uint32
        L.orc_lookup_many.argtypes = [P, P, ctypes.c_uint64, P]
        L.orc_rate_bps.argtypes = [ctypes.c_uint64, ctypes.c_uint32]
        L.orc_rate_bps.restype = ctypes.c_uint64
        L.orc_rate_many.argtypes = [P, P, ctypes.c_uint64, P]
        R = ctypes.POINTER(BulkRule)
        L.orc_is_bulk.argtypes = [R, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]
        L.orc_is_bulk.restype = ctypes.c_int
        L.orc_classify_aggregate.argtypes = [P, P, P, ctypes.c_uint32, P, P, P, P, P, P,
                                             ctypes.c_uint64, R, ctypes.c_int, P]
        L.orc_classify_aggregate.restype = ctypes.c_int
        L.orc_classify_aggregate_windows.argtypes = [P, P, P, ctypes.c_uint32, P, P, P, P, P, P, P,
                                                     ctypes.c_uint32, R, ctypes.c_int, P]
        L.orc_classify_aggregate_windows.restype = ctypes.c_int
        L.orc_classify_rows.argtypes = [P, P, P, ctypes.c_uint32, P, P, P, P, P, P, ctypes.c_uint64, R,
                                        P, P, P]
        L.orc_classify_rows.restype = ctypes.c_int
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


class BulkRule(ctypes.Structure):
    """Rate eligibility: bytes > bulk_bytes, dur > 0, and the two optional
    exclusion filters of §III.B.2 (0 = off): bytes >= min_avg_packet_bytes *
    packets (reverse-direction ACK flows), packets >= min_packets and dur >=
    min_duration_ms (administrative exchanges)."""
    _fields_ = [("bulk_bytes", ctypes.c_uint64), ("min_avg_packet_bytes", ctypes.c_uint32),
                ("min_packets", ctypes.c_uint32), ("min_duration_ms", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


FILTER_KEYS = ("min_avg_packet_bytes", "min_packets", "min_duration_ms")


def bulk_rule(bulk_bytes: int = 1_000_000, filters: Optional[dict] = None) -> BulkRule:
    f = dict(filters or {})
    bad = set(f) - set(FILTER_KEYS)
    if bad:
        raise ValueError("unknown filters: %s" % sorted(bad))
    return BulkRule(int(bulk_bytes), *(int(f.get(k, 0)) for k in FILTER_KEYS), 0)


def is_bulk(nbytes: int, packets: int, dur_ms: int, bulk_bytes: int = 1_000_000,
            filters: Optional[dict] = None) -> bool:
    r = bulk_rule(bulk_bytes, filters)
    return bool(lib().orc_is_bulk(ctypes.byref(r), int(nbytes), int(packets), int(dur_ms)))


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__({E_INVAL: "invalid argument", E_CONFLICT: "conflicting prefixes",
                          E_NOMEM: "out of memory"}.get(code, "error %d" % code))
        self.code = code


class Registry:
    """Oracle-side registry: sites (addr, len, site) plus the local prefix set."""

    def __init__(self, addr, length, site, n_sites: int, local_addr, local_len):
        self.addr = np.ascontiguousarray(addr, dtype=np.uint32)
        self.length = np.ascontiguousarray(length, dtype=np.uint32)
        self.site = np.ascontiguousarray(site, dtype=np.uint32)
        self.local_addr = np.ascontiguousarray(local_addr, dtype=np.uint32)
        self.local_len = np.ascontiguousarray(local_len, dtype=np.uint32)
        self.n_sites = int(n_sites)
        h = ctypes.c_void_p()
        rc = lib().orc_registry_build(_p(self.addr), _p(self.length), _p(self.site),
                                      self.addr.shape[0], self.n_sites, ctypes.byref(h))
        if rc != OK:
            raise OracleError(rc)
        self._h = h

    @classmethod
    def from_generated(cls, reg) -> "Registry":
        return cls(reg.addr, reg.length, reg.site, reg.n_sites, reg.local_addr, reg.local_len)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().orc_registry_free(h)
            self._h = None

    @property
    def rows(self) -> int:
        return 2 * self.n_sites + 3

    def lookup(self, ips) -> np.ndarray:
        ips = np.ascontiguousarray(ips, dtype=np.uint32)
        out = np.empty(ips.shape[0], dtype=np.uint32)
        lib().orc_lookup_many(self._h, _p(ips), ips.shape[0], _p(out))
        return out

    def classify_aggregate(self, rec, bulk_bytes: int = 1_000_000,
                           threads: int = 0, window_offsets: Optional[np.ndarray] = None,
                           filters: Optional[dict] = None) -> np.ndarray:
        """Rows for each window: uint64[n_windows, rows, 8] (or [rows, 8] for one window).

        filters: optional exclusion thresholds (see BulkRule)."""
        rule = bulk_rule(bulk_bytes, filters)
        f = {k: np.ascontiguousarray(getattr(rec, k)) for k in
             ("src_ip", "dst_ip", "bytes", "packets", "first_ms", "last_ms")}
        assert f["bytes"].dtype == np.uint64 and f["src_ip"].dtype == np.uint32
        off = window_offsets if window_offsets is not None else getattr(rec, "window_offsets", None)
        if off is None:
            out = np.empty((self.rows, 8), dtype=np.uint64)
            rc = lib().orc_classify_aggregate(self._h, _p(self.local_addr), _p(self.local_len),
                                              self.local_addr.shape[0], _p(f["src_ip"]), _p(f["dst_ip"]),
                                              _p(f["bytes"]), _p(f["packets"]), _p(f["first_ms"]),
                                              _p(f["last_ms"]), f["src_ip"].shape[0], ctypes.byref(rule),
                                              threads, _p(out))
        else:
            off = np.ascontiguousarray(off, dtype=np.uint64)
            nw = off.shape[0] - 1
            out = np.empty((nw, self.rows, 8), dtype=np.uint64)
            rc = lib().orc_classify_aggregate_windows(self._h, _p(self.local_addr), _p(self.local_len),
                                                      self.local_addr.shape[0], _p(f["src_ip"]),
                                                      _p(f["dst_ip"]), _p(f["bytes"]), _p(f["packets"]),
                                                      _p(f["first_ms"]), _p(f["last_ms"]), _p(off), nw,
                                                      ctypes.byref(rule), threads, _p(out))
        if rc != OK:
            raise OracleError(rc)
        return out


RATE_BUCKETS = 10001      # 10 kbps buckets; the last one takes every rate above 100 Mbps
RATE_BUCKET_BPS = 10_000
NO_MEDIAN = 0xFFFFFFFF


def rate_bucket(rate_bps) -> np.ndarray:
    """Bucket of a rate: floor(rate / 10 kbps), the rates of the last bucket
    and above all in bucket 10000 (§III.B.2, TransRate Kernel)."""
    r = np.asarray(rate_bps, dtype=np.uint64)
    return np.minimum(r // np.uint64(RATE_BUCKET_BPS), np.uint64(RATE_BUCKETS - 1)).astype(np.uint32)


def _classify_rows(reg: "Registry", rec, bulk_bytes: int, filters: Optional[dict] = None):
    rule = bulk_rule(bulk_bytes, filters)
    f = {k: np.ascontiguousarray(getattr(rec, k))
         for k in ("src_ip", "dst_ip", "bytes", "packets", "first_ms", "last_ms")}
    n = f["src_ip"].shape[0]
    row = np.empty(n, dtype=np.uint32)
    bulk = np.empty(n, dtype=np.uint8)
    rate = np.empty(n, dtype=np.uint64)
    rc = lib().orc_classify_rows(reg._h, _p(reg.local_addr), _p(reg.local_len), reg.local_addr.shape[0],
                                 _p(f["src_ip"]), _p(f["dst_ip"]), _p(f["bytes"]), _p(f["packets"]),
                                 _p(f["first_ms"]), _p(f["last_ms"]), n, ctypes.byref(rule), _p(row), _p(bulk),
                                 _p(rate))
    if rc != OK:
        raise OracleError(rc)
    return row, bulk.astype(bool), rate


def rate_histograms(reg: "Registry", rec, window_offsets=None, bulk_bytes: int = 1_000_000,
                    filters: Optional[dict] = None) -> np.ndarray:
    """Counts of bulk-flow rates per (window, row, 10 kbps bucket): uint32[n_windows, rows, 10001]."""
    row, is_bulk, rate = _classify_rows(reg, rec, bulk_bytes, filters)
    off = window_offsets if window_offsets is not None else getattr(rec, "window_offsets", None)
    off = np.array([0, rec.n], dtype=np.uint64) if off is None else np.asarray(off, dtype=np.uint64)
    nw = off.shape[0] - 1
    out = np.zeros((nw, reg.rows, RATE_BUCKETS), dtype=np.uint32)
    for w in range(nw):
        lo, hi = int(off[w]), int(off[w + 1])
        bulk = is_bulk[lo:hi]
        np.add.at(out[w], (row[lo:hi][bulk], rate_bucket(rate[lo:hi][bulk])), 1)
    return out


def rate_medians(reg: "Registry", rec, window_offsets=None, bulk_bytes: int = 1_000_000,
                 filters: Optional[dict] = None):
    """Median bucket and bulk-flow count per (window, row).

    The median of a row's N >= 1 bulk flows is the bucket of its ceil(N/2)-th
    smallest rate (the lower median), found by sorting the flows' buckets;
    NO_MEDIAN when N = 0.  Returns (uint32[n_windows, rows], uint64[n_windows, rows]).
    """
    row, is_bulk, rate = _classify_rows(reg, rec, bulk_bytes, filters)
    off = window_offsets if window_offsets is not None else getattr(rec, "window_offsets", None)
    off = np.array([0, rec.n], dtype=np.uint64) if off is None else np.asarray(off, dtype=np.uint64)
    nw = off.shape[0] - 1
    med = np.full((nw, reg.rows), NO_MEDIAN, dtype=np.uint32)
    cnt = np.zeros((nw, reg.rows), dtype=np.uint64)
    for w in range(nw):
        lo, hi = int(off[w]), int(off[w + 1])
        bulk = is_bulk[lo:hi]
        r, b = row[lo:hi][bulk], rate_bucket(rate[lo:hi][bulk])
        order = np.lexsort((b, r))  # by row, then by bucket
        r, b = r[order], b[order]
        rows_present, start, n = np.unique(r, return_index=True, return_counts=True)
        med[w, rows_present] = b[start + (n + 1) // 2 - 1]
        cnt[w, rows_present] = n
    return med, cnt


HOST_FIELDS = ("bulk_flows", "bulk_bytes", "rate_sum_bps", "rate_min_bps", "rate_max_bps")


def host_stats(reg: "Registry", rec, bulk_bytes: int = 1_000_000, filters: Optional[dict] = None):
    """Rate statistics per remote host of a registered site (§III.B.2: rates are
    also computed for each host in a registered site), per direction.

    Over the bulk flows of the registered (site, direction) rows: key =
    remote address << 32 | row (row = 2 * site + direction; the remote
    address is the source of an inbound flow, the destination of an outbound
    one); per key the bulk flows, their bytes and rates (sum modulo 2^64,
    min, max).  Returns (uint64 keys sorted ascending, uint64[n_keys, 5]).
    """
    row, is_bulk, rate = _classify_rows(reg, rec, bulk_bytes, filters)
    sel = is_bulk & (row < 2 * reg.n_sites)
    remote = np.where(row % 2 == 0, np.asarray(rec.src_ip), np.asarray(rec.dst_ip))[sel]
    key = (remote.astype(np.uint64) << np.uint64(32)) | row[sel].astype(np.uint64)
    b = np.asarray(rec.bytes)[sel]
    r = rate[sel]
    order = np.argsort(key, kind="stable")
    key, b, r = key[order], b[order], r[order]
    keys, start = np.unique(key, return_index=True)
    out = np.zeros((keys.size, 5), dtype=np.uint64)
    if keys.size:
        out[:, 0] = np.diff(np.append(start, key.size))
        out[:, 1] = np.add.reduceat(b, start)         # uint64: wraps modulo 2^64
        out[:, 2] = np.add.reduceat(r, start)
        out[:, 3] = np.minimum.reduceat(r, start)
        out[:, 4] = np.maximum.reduceat(r, start)
    return keys, out


def host_medians(reg: "Registry", rec, bulk_bytes: int = 1_000_000, filters: Optional[dict] = None):
    """Lower-median rate bucket per remote host of a registered site, per
    direction (§III.B.2, TransRate Kernel: max, min, average and median rates
    for each host in a registered site, the median read from the host's
    10 kbps bucket array).

    Keys as in host_stats.  For a host with N bulk flows, its bucket array's
    cumulative count first reaches ceil(N/2) at the ceil(N/2)-th smallest of
    its flows' buckets: that bucket is the lower median (the convention of
    rate_medians).  Returns (uint64 keys sorted ascending, uint32 buckets).
    """
    row, is_bulk, rate = _classify_rows(reg, rec, bulk_bytes, filters)
    sel = is_bulk & (row < 2 * reg.n_sites)
    remote = np.where(row % 2 == 0, np.asarray(rec.src_ip), np.asarray(rec.dst_ip))[sel]
    key = (remote.astype(np.uint64) << np.uint64(32)) | row[sel].astype(np.uint64)
    bucket = rate_bucket(rate[sel])
    order = np.lexsort((bucket, key))  # by key, then bucket
    key, bucket = key[order], bucket[order]
    keys, start = np.unique(key, return_index=True)
    n = np.diff(np.append(start, key.size))
    med = bucket[start + (n + 1) // 2 - 1] if keys.size else np.zeros(0, dtype=np.uint32)
    return keys, med.astype(np.uint32)


def median_flags(med: np.ndarray, cnt: np.ndarray, n_sites: int, threshold_bps: int = 1_000_000,
                 min_bulk_flows: int = 0, prev: Optional[np.ndarray] = None) -> np.ndarray:
    """Median warnings per (window, site), one site and window at a time.

    bit d (d = 0 inbound, 1 outbound): the (site, d) row has at least
    max(1, min_bulk_flows) bulk flows and its median bucket's lower bound,
    bucket * 10 kbps, is below the threshold (exactly "median < threshold"
    when the threshold is a multiple of 10 kbps, as the paper's 1 Mbps is);
    bit 2 + d: bit d is set in this window and in the previous one (window
    w - 1, or `prev` for the first window): the paper's warning after two
    consecutive hours (§III.B.1, NetPerf Monitoring Thread; §IV.B).
    """
    med = np.asarray(med)
    cnt = np.asarray(cnt)
    nw = med.shape[0]
    need = max(1, int(min_bulk_flows))
    out = np.zeros((nw, n_sites), dtype=np.uint8)
    for w in range(nw):
        for s in range(n_sites):
            f = 0
            for d in (0, 1):
                m, c = int(med[w, 2 * s + d]), int(cnt[w, 2 * s + d])
                if c >= need and m * RATE_BUCKET_BPS < threshold_bps:
                    f |= 1 << d
            before = int(out[w - 1, s]) if w > 0 else (0 if prev is None else int(prev[s]))
            f |= ((f & before) & 3) << 2
            out[w, s] = f
    return out


def rate_bps(nbytes, dur_ms) -> np.ndarray:
    b = np.ascontiguousarray(nbytes, dtype=np.uint64)
    d = np.ascontiguousarray(dur_ms, dtype=np.uint32)
    out = np.empty(b.shape[0], dtype=np.uint64)
    lib().orc_rate_many(_p(b), _p(d), b.shape[0], _p(out))
    return out


def flags(rows: np.ndarray, n_sites: int, threshold_bps: int = 1_000_000,
          min_bulk_flows: int = 0) -> np.ndarray:
    """Sub-optimal flags per site (bit 0 inbound, bit 1 outbound).

    A (site, direction) is flagged when it has at least max(1, min_bulk_flows)
    bulk flows and its mean per-flow rate floor(rate_sum / bulk_flows) is
    strictly below the threshold.  The paper warns on a low rate statistic
    per site (§III.B.1, NetPerf Monitoring Thread; §IV.B); the mean is the
    reading used here.  Python integers, one (site, direction) at a time.
    """
    rows = np.asarray(rows, dtype=np.uint64)
    single = rows.ndim == 2
    if single:
        rows = rows[None]
    out = np.zeros((rows.shape[0], n_sites), dtype=np.uint8)
    need = max(1, int(min_bulk_flows))
    for w in range(rows.shape[0]):
        for s in range(n_sites):
            f = 0
            for d in (0, 1):
                r = rows[w, 2 * s + d]
                bulk, rsum = int(r[4]), int(r[5])
                if bulk >= need and rsum // bulk < threshold_bps:
                    f |= 1 << d
            out[w, s] = f
    return out[0] if single else out


def max_threads() -> int:
    return int(lib().orc_max_threads())
