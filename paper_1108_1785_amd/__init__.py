"""Python binding of libgnm (ctypes): argument marshalling only.

Every step of the classify/aggregate path runs in the library's HIP kernels
for gfx950; this module converts torch device tensors to raw pointers and the
current torch stream to a HIP stream handle.  There is no fallback: if
libgnm.so has not been built, importing works but every call raises.

Function names follow the C ABI in include/gnm.h.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgnm.so")

GNM_OK = 0
GNM_E_INVAL = -1
GNM_E_CONFLICT = -2
GNM_E_NOMEM = -3
GNM_E_HIP = -4
GNM_E_UNSUPPORTED = -5
GNM_ACCUMULATE = 0x1
GNM_REG_HOST_ONLY = 0x1
GNM_REG_FORCE_WIDE = 0x2
GNM_REG_FORCE_LINES = 0x4
GNM_REG_SHALLOW = 0x8

ACC_FIELDS = ("flows", "bytes", "packets", "duration_ms", "bulk_flows",
              "rate_sum_bps", "rate_min_bps", "rate_max_bps")
RECORD_FIELDS = {"src_ip": 4, "dst_ip": 4, "bytes": 8, "packets": 4, "first_ms": 4, "last_ms": 4}

# symbols declared in include/gnm.h
EXPORTS = ("gnm_registry_build", "gnm_registry_free", "gnm_registry_info_get", "gnm_acc_rows",
           "gnm_registry_lookup_host", "gnm_params_default", "gnm_workspace_bytes", "gnm_workspace_bytes_n", "gnm_workspace_bytes_hist",
           "gnm_host_work_bytes", "gnm_classify_aggregate",
           "gnm_classify_flag", "gnm_classify_flag_static", "gnm_static_scratch_bytes", "gnm_flag_suboptimal", "gnm_median_flags", "gnm_graph_create", "gnm_graph_launch", "gnm_graph_free", "gnm_autotune",
           "gnm_netflow_v5_workspace_bytes", "gnm_netflow_v5_decode",
           "gnm_strerror", "gnm_last_error", "gnm_version")
TUNE_MAX = 16
RATE_BUCKETS = 10001        # 10 kbps rate buckets per (site, direction) histogram
RATE_BUCKET_BPS = 10000
NO_MEDIAN = 0xFFFFFFFF


class Prefix(ctypes.Structure):
    _fields_ = [("addr", ctypes.c_uint32), ("len", ctypes.c_uint32), ("site", ctypes.c_uint32)]


class RecordsC(ctypes.Structure):
    _fields_ = [("src_ip", ctypes.c_void_p), ("dst_ip", ctypes.c_void_p),
                ("src_port", ctypes.c_void_p), ("dst_port", ctypes.c_void_p), ("proto", ctypes.c_void_p),
                ("bytes", ctypes.c_void_p), ("packets", ctypes.c_void_p),
                ("first_ms", ctypes.c_void_p), ("last_ms", ctypes.c_void_p), ("n", ctypes.c_uint64)]


class RecordsOutC(ctypes.Structure):
    _fields_ = [("src_ip", ctypes.c_void_p), ("dst_ip", ctypes.c_void_p),
                ("src_port", ctypes.c_void_p), ("dst_port", ctypes.c_void_p), ("proto", ctypes.c_void_p),
                ("bytes", ctypes.c_void_p), ("packets", ctypes.c_void_p),
                ("first_ms", ctypes.c_void_p), ("last_ms", ctypes.c_void_p), ("capacity", ctypes.c_uint64)]


class Params(ctypes.Structure):
    _fields_ = [("bulk_bytes", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("records_per_thread", ctypes.c_uint32), ("grid_blocks", ctypes.c_uint32),
                ("flush_records", ctypes.c_uint32), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_uint64), ("rate_hist", ctypes.c_void_p),
                ("min_avg_packet_bytes", ctypes.c_uint32), ("min_packets", ctypes.c_uint32),
                ("min_duration_ms", ctypes.c_uint32), ("reserved2", ctypes.c_uint32),
                ("hosts", ctypes.c_void_p)]


class HostTableC(ctypes.Structure):
    _fields_ = [("keys", ctypes.c_void_p), ("stats", ctypes.c_void_p), ("median", ctypes.c_void_p),
                ("capacity", ctypes.c_uint64), ("counters", ctypes.c_void_p), ("work", ctypes.c_void_p),
                ("work_bytes", ctypes.c_uint64)]


HOST_FIELDS = ("bulk_flows", "bulk_bytes", "rate_sum_bps", "rate_min_bps", "rate_max_bps")


def host_work_bytes(reg: "Registry", n_records: int, grid_blocks: int = 0) -> int:
    """gnm_host_work_bytes: work buffer of a host table for n_records records."""
    return int(lib().gnm_host_work_bytes(reg.handle, int(n_records), int(grid_blocks)))


class HostTable:
    """Device per-host statistics and medians (gnm_host_table) for calls of up
    to n_records records on grid_blocks workgroups (0 = automatic): room for
    `capacity` hosts, plus the work buffer."""

    def __init__(self, reg: "Registry", capacity: int, n_records: int, grid_blocks: int = 0, device=None,
                 medians: bool = True):
        import torch
        capacity = int(capacity)
        if capacity < 0:
            raise ValueError("capacity must be >= 0")
        dev = device if device is not None else "cuda"
        self.capacity = capacity
        self.keys = torch.empty(max(capacity, 1), dtype=torch.int64, device=dev)
        self.stats = torch.empty((max(capacity, 1), 5), dtype=torch.int64, device=dev)
        self.median = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev) if medians else None
        self.counters = torch.zeros(2, dtype=torch.int64, device=dev)
        wb = host_work_bytes(reg, n_records, grid_blocks)
        self._work = torch.empty(wb + 256, dtype=torch.uint8, device=dev)
        base = self._work.data_ptr()
        self.c = HostTableC(self.keys.data_ptr(), self.stats.data_ptr(),
                            self.median.data_ptr() if medians else 0, capacity, self.counters.data_ptr(),
                            (base + 255) & ~255, wb)

    def to_numpy(self):
        """(keys sorted ascending, stats [n, 5], median buckets (or None), hosts found, bulk flows of
        registered sites); keys and stats uint64, medians uint32."""
        cnt = self.counters.cpu().numpy().view(np.uint64)
        n = min(int(cnt[0]), self.capacity)
        k = self.keys[:n].cpu().numpy().view(np.uint64)
        st = self.stats[:n].cpu().numpy().view(np.uint64)
        order = np.argsort(k, kind="stable")
        med = None if self.median is None else self.median[:n].cpu().numpy().view(np.uint32)[order]
        return k[order], st[order], med, int(cnt[0]), int(cnt[1])


FILTER_KEYS = ("min_avg_packet_bytes", "min_packets", "min_duration_ms")


class TuneResult(ctypes.Structure):
    _fields_ = [("best", Params), ("best_ms", ctypes.c_float), ("n_tried", ctypes.c_uint32),
                ("ms", ctypes.c_float * TUNE_MAX), ("records_per_thread", ctypes.c_uint32 * TUNE_MAX),
                ("grid_blocks", ctypes.c_uint32 * TUNE_MAX)]


class RegistryOpts(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("root_bits", ctypes.c_uint32),
                ("list_max", ctypes.c_uint32), ("lds_bytes", ctypes.c_uint32), ("node_bits", ctypes.c_uint32)]


class RegistryInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("n_prefixes_in", "n_prefixes", "n_host_bits", "n_duplicates",
                                               "n_intervals", "n_nodes", "n_leaf_lines", "device_bytes")] + \
               [(n, ctypes.c_uint32) for n in ("n_sites", "n_local_ranges", "root_bits", "list_max",
                                               "lines_in_lds", "acc_in_lds", "lds_bytes", "cache_slots",
                                               "node_bits", "reserved")]

    def as_dict(self) -> Dict[str, int]:
        return {f: int(getattr(self, f)) for f, _ in self._fields_ if f != "reserved"}


class GnmError(RuntimeError):
    def __init__(self, code: int, where: str):
        lib = _lib_or_none()
        msg = lib.gnm_strerror(code).decode() if lib else str(code)
        detail = lib.gnm_last_error().decode() if lib else ""
        super().__init__("%s: %s%s" % (where, msg, (" (%s)" % detail) if detail else ""))
        self.code = code


_lib = None


def _lib_or_none():
    return _lib


def lib():
    """The loaded libgnm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libgnm.so is not built (run python -m paper_1108_1785_amd._build); "
                               "there is no non-HIP implementation of this path")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.gnm_registry_build.argtypes = [P, ctypes.c_uint64, ctypes.c_uint32, P, ctypes.c_uint32, P, P,
                                         ctypes.POINTER(P)]
        L.gnm_registry_build.restype = ctypes.c_int
        L.gnm_registry_free.argtypes = [P]
        L.gnm_registry_free.restype = ctypes.c_int
        L.gnm_registry_info_get.argtypes = [P, ctypes.POINTER(RegistryInfo)]
        L.gnm_registry_info_get.restype = ctypes.c_int
        L.gnm_acc_rows.argtypes = [P]
        L.gnm_acc_rows.restype = ctypes.c_uint64
        L.gnm_registry_lookup_host.argtypes = [P, P, ctypes.c_uint64, P, P]
        L.gnm_registry_lookup_host.restype = ctypes.c_int
        L.gnm_params_default.argtypes = []
        L.gnm_params_default.restype = Params
        L.gnm_workspace_bytes.argtypes = [P, ctypes.c_uint32]
        L.gnm_workspace_bytes.restype = ctypes.c_uint64
        L.gnm_workspace_bytes_n.argtypes = [P, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]
        L.gnm_workspace_bytes_n.restype = ctypes.c_uint64
        L.gnm_workspace_bytes_hist.argtypes = [P, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]
        L.gnm_workspace_bytes_hist.restype = ctypes.c_uint64
        L.gnm_host_work_bytes.argtypes = [P, ctypes.c_uint64, ctypes.c_uint32]
        L.gnm_host_work_bytes.restype = ctypes.c_uint64
        L.gnm_classify_aggregate.argtypes = [P, ctypes.POINTER(RecordsC), P, ctypes.c_uint32,
                                             ctypes.POINTER(Params), P, P]
        L.gnm_classify_aggregate.restype = ctypes.c_int
        L.gnm_classify_flag.argtypes = [P, ctypes.POINTER(RecordsC), P, ctypes.c_uint32, ctypes.POINTER(Params), P,
                                        ctypes.c_uint64, ctypes.c_uint64, P, P]
        L.gnm_classify_flag.restype = ctypes.c_int
        L.gnm_classify_flag_static.argtypes = L.gnm_classify_flag.argtypes
        L.gnm_classify_flag_static.restype = ctypes.c_int
        L.gnm_static_scratch_bytes.argtypes = []
        L.gnm_static_scratch_bytes.restype = ctypes.c_uint64
        L.gnm_flag_suboptimal.argtypes = [P, P, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, P, P]
        L.gnm_flag_suboptimal.restype = ctypes.c_int
        L.gnm_median_flags.argtypes = [P, P, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, P, P, P, P]
        L.gnm_median_flags.restype = ctypes.c_int
        L.gnm_graph_create.argtypes = [P, ctypes.POINTER(RecordsC), P, ctypes.c_uint32, ctypes.POINTER(Params), P,
                                       ctypes.c_uint64, ctypes.c_uint64, P, ctypes.POINTER(P)]
        L.gnm_graph_create.restype = ctypes.c_int
        L.gnm_graph_launch.argtypes = [P, P]
        L.gnm_graph_launch.restype = ctypes.c_int
        L.gnm_graph_free.argtypes = [P]
        L.gnm_graph_free.restype = ctypes.c_int
        L.gnm_autotune.argtypes = [P, ctypes.POINTER(RecordsC), P, ctypes.c_uint32, ctypes.POINTER(Params), P,
                                   ctypes.c_uint32, P, ctypes.POINTER(TuneResult)]
        L.gnm_autotune.restype = ctypes.c_int
        L.gnm_netflow_v5_workspace_bytes.argtypes = [ctypes.c_uint64]
        L.gnm_netflow_v5_workspace_bytes.restype = ctypes.c_uint64
        L.gnm_netflow_v5_decode.argtypes = [P, ctypes.c_uint64, P, ctypes.c_uint64, P, ctypes.c_uint64,
                                            ctypes.POINTER(RecordsOutC), P, P, P]
        L.gnm_netflow_v5_decode.restype = ctypes.c_int
        L.gnm_strerror.argtypes = [ctypes.c_int]
        L.gnm_strerror.restype = ctypes.c_char_p
        L.gnm_last_error.argtypes = []
        L.gnm_last_error.restype = ctypes.c_char_p
        L.gnm_version.argtypes = []
        L.gnm_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int, where: str):
    if rc != GNM_OK:
        raise GnmError(rc, where)


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    h = getattr(stream, "cuda_stream", stream)
    return ctypes.c_void_p(int(h) if h else 0)


def _prefix_array(addr, length, site=None):
    addr = np.asarray(addr, dtype=np.uint64).reshape(-1)
    length = np.asarray(length, dtype=np.uint64).reshape(-1)
    n = addr.shape[0]
    arr = (Prefix * max(n, 1))()
    site = np.zeros(n, dtype=np.uint64) if site is None else np.asarray(site, dtype=np.uint64).reshape(-1)
    for i, (a, l, s) in enumerate(zip(addr.tolist(), length.tolist(), site.tolist())):
        arr[i].addr, arr[i].len, arr[i].site = a, l, s
    return arr, n


class Registry:
    """gnm_registry_build / gnm_registry_free over host prefix arrays."""

    def __init__(self, addr, length, site, n_sites: int, local_addr=(), local_len=(),
                 root_bits: int = 0, list_max: int = 0, lds_bytes: int = 0,
                 host_only: bool = False, stream=None, layout: str = "auto", node_bits: int = 0):
        """layout: "auto", "wide" (GNM_REG_FORCE_WIDE), "lines" (GNM_REG_FORCE_LINES),
        "shallow" (GNM_REG_SHALLOW) or "wide-shallow" (both)."""
        L = lib()
        sites, n = _prefix_array(addr, length, site)
        local, nl = _prefix_array(local_addr, local_len)
        flags = (GNM_REG_HOST_ONLY if host_only else 0) | \
            {"auto": 0, "wide": GNM_REG_FORCE_WIDE, "lines": GNM_REG_FORCE_LINES, "shallow": GNM_REG_SHALLOW,
             "wide-shallow": GNM_REG_FORCE_WIDE | GNM_REG_SHALLOW}[layout]
        opts = RegistryOpts(flags, root_bits, list_max, lds_bytes, node_bits)
        h = ctypes.c_void_p()
        st = ctypes.c_void_p(0) if host_only else _stream_handle(stream)
        _check(L.gnm_registry_build(sites, n, int(n_sites), local, nl, ctypes.byref(opts), st,
                                    ctypes.byref(h)), "gnm_registry_build")
        self._h = h
        self.n_sites = int(n_sites)
        self.host_only = host_only

    @classmethod
    def from_generated(cls, reg, **kw) -> "Registry":
        return cls(reg.addr, reg.length, reg.site, reg.n_sites, reg.local_addr, reg.local_len, **kw)

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise RuntimeError("registry is closed")
        return self._h

    @property
    def rows(self) -> int:
        return int(lib().gnm_acc_rows(self.handle))

    def info(self) -> Dict[str, int]:
        i = RegistryInfo()
        _check(lib().gnm_registry_info_get(self.handle, ctypes.byref(i)), "gnm_registry_info_get")
        return i.as_dict()

    def lookup_host(self, ips):
        ips = np.ascontiguousarray(ips, dtype=np.uint32)
        site = np.empty(ips.shape[0], dtype=np.uint32)
        loc = np.empty(ips.shape[0], dtype=np.uint8)
        _check(lib().gnm_registry_lookup_host(self.handle, ips.ctypes.data, ips.shape[0], site.ctypes.data,
                                              loc.ctypes.data), "gnm_registry_lookup_host")
        return site, loc.astype(bool)

    def close(self):
        if getattr(self, "_h", None) is not None:
            _check(lib().gnm_registry_free(self._h), "gnm_registry_free")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr(t, elem: int, n: int, name: str, device=None) -> int:
    if t is None:
        raise ValueError("record field %s is required" % name)
    if t.element_size() != elem:
        raise ValueError("record field %s must have %d-byte elements" % (name, elem))
    if not t.is_cuda or not t.is_contiguous() or t.numel() < n:
        raise ValueError("record field %s must be a contiguous device tensor of >= %d elements" % (name, n))
    return t.data_ptr()


def records_struct(rec: Dict[str, "object"], n: Optional[int] = None) -> RecordsC:
    """SoA device tensors (src_ip, dst_ip, bytes, packets, first_ms, last_ms) -> gnm_records."""
    if n is None:
        n = int(rec["src_ip"].numel())
    c = RecordsC()
    for f, elem in RECORD_FIELDS.items():
        setattr(c, f, _ptr(rec[f], elem, n, f))
    c.n = n
    return c


def make_params(bulk_bytes: int = 1_000_000, accumulate: bool = False, records_per_thread: int = 0,
                grid_blocks: int = 0, workspace=None, rate_hist=None, filters=None, hosts=None,
                flush_records: int = 0) -> Params:
    """filters: optional dict of exclusion thresholds (FILTER_KEYS), 0 = off.
    hosts: optional HostTable (the caller keeps it alive while work is queued).
    flush_records: records a workgroup aggregates between table flushes (0 = 2^31)."""
    p = lib().gnm_params_default()
    p.bulk_bytes = int(bulk_bytes)
    p.flags = GNM_ACCUMULATE if accumulate else 0
    p.records_per_thread = int(records_per_thread)
    p.grid_blocks = int(grid_blocks)
    if not 0 <= int(flush_records) < 2**32:
        raise ValueError("flush_records must fit 32 bits")
    p.flush_records = int(flush_records)
    if workspace is not None:
        if not workspace.is_cuda or not workspace.is_contiguous():
            raise ValueError("workspace must be a contiguous device tensor")
        p.workspace = workspace.data_ptr()
        p.workspace_bytes = workspace.numel() * workspace.element_size()
    if rate_hist is not None:
        if not rate_hist.is_cuda or not rate_hist.is_contiguous() or rate_hist.element_size() != 4:
            raise ValueError("rate_hist must be a contiguous device tensor of 32-bit counts")
        p.rate_hist = rate_hist.data_ptr()
    f = dict(filters or {})
    if set(f) - set(FILTER_KEYS):
        raise ValueError("unknown filters: %s" % sorted(set(f) - set(FILTER_KEYS)))
    for k in FILTER_KEYS:
        v = int(f.get(k, 0))
        if not 0 <= v < 2**32:
            raise ValueError("%s must fit 32 bits" % k)
        setattr(p, k, v)
    if hosts is not None:
        if not isinstance(hosts, HostTable):
            raise ValueError("hosts must be a HostTable")
        p.hosts = ctypes.addressof(hosts.c)
    return p


def rate_hist_words(reg: Registry, n_windows: int = 1) -> int:
    """Counts in the rate histograms of n_windows windows: n_windows * 2 * n_sites * 10001."""
    return int(n_windows) * 2 * reg.n_sites * RATE_BUCKETS


def make_rate_hist(reg: Registry, n_windows: int = 1, device=None):
    """A device int32 tensor [n_windows, 2 * n_sites, 10001] for the rate histograms."""
    import torch
    return torch.empty((int(n_windows), 2 * reg.n_sites, RATE_BUCKETS), dtype=torch.int32,
                       device=device if device is not None else "cuda")


def workspace_bytes(reg: Registry, grid_blocks: int = 0) -> int:
    """gnm_workspace_bytes: scratch size for a launch of grid_blocks workgroups (0 = automatic)."""
    return int(lib().gnm_workspace_bytes(reg.handle, int(grid_blocks)))


def workspace_bytes_n(reg: Registry, n_records: int, n_windows: int = 1, grid_blocks: int = 0) -> int:
    """gnm_workspace_bytes_n: scratch size for a call over n_records records in n_windows windows."""
    return int(lib().gnm_workspace_bytes_n(reg.handle, int(n_records), int(n_windows), int(grid_blocks)))


def workspace_bytes_hist(reg: Registry, n_records: int, n_windows: int = 1, grid_blocks: int = 0) -> int:
    """gnm_workspace_bytes_hist: scratch size for a call with rate histograms, whose keys it also holds."""
    return int(lib().gnm_workspace_bytes_hist(reg.handle, int(n_records), int(n_windows), int(grid_blocks)))


def make_workspace(reg: Registry, grid_blocks: int = 0, device=None, n_records: Optional[int] = None,
                   n_windows: int = 1, hist: bool = False):
    """A device byte tensor of gnm_workspace_bytes(reg, grid_blocks) bytes, or, with
    n_records, of gnm_workspace_bytes_n (which also holds the spilled rows of a
    table too large for LDS), or with hist as well, of gnm_workspace_bytes_hist
    (which also holds the staged histogram keys); 256-byte aligned (torch's
    allocations are)."""
    import torch
    if hist and n_records is None:
        raise ValueError("a workspace for staged histograms needs n_records")
    if hist:
        nb = workspace_bytes_hist(reg, n_records, n_windows, grid_blocks)
    else:
        nb = workspace_bytes(reg, grid_blocks) if n_records is None else \
            workspace_bytes_n(reg, n_records, n_windows, grid_blocks)
    t = torch.empty(max(nb, 1), dtype=torch.uint8, device=device if device is not None else "cuda")
    if t.data_ptr() % 256:
        raise RuntimeError("device allocation not 256-byte aligned")
    return t


def classify_aggregate(reg: Registry, rec, acc, window_offsets=None, n_windows: int = 1,
                       bulk_bytes: int = 1_000_000, accumulate: bool = False,
                       records_per_thread: int = 0, grid_blocks: int = 0, stream=None,
                       n: Optional[int] = None, workspace=None, rate_hist=None, filters=None,
                       hosts=None, flush_records: int = 0) -> None:
    """gnm_classify_aggregate: acc is a device tensor of n_windows*rows*8 64-bit words.

    workspace: optional device tensor from make_workspace() (faster table merge).
    rate_hist: optional device tensor from make_rate_hist() (bulk-rate histograms).
    filters: optional exclusion thresholds, e.g. {"min_avg_packet_bytes": 100}.
    hosts: optional HostTable for per-host statistics.
    """
    c, off, p = _classify_args(reg, rec, acc, window_offsets, n_windows, bulk_bytes, accumulate, records_per_thread,
                               grid_blocks, n, workspace, rate_hist, filters, hosts, flush_records)
    _check(lib().gnm_classify_aggregate(reg.handle, ctypes.byref(c), ctypes.c_void_p(off), int(n_windows),
                                        ctypes.byref(p), ctypes.c_void_p(acc.data_ptr()),
                                        _stream_handle(stream)), "gnm_classify_aggregate")


def _classify_args(reg, rec, acc, window_offsets, n_windows, bulk_bytes, accumulate, records_per_thread,
                   grid_blocks, n, workspace, rate_hist, filters, hosts, flush_records=0):
    c = rec if isinstance(rec, RecordsC) else records_struct(rec, n)
    if acc.element_size() * acc.numel() < n_windows * reg.rows * 64 or not acc.is_cuda:
        raise ValueError("acc must be a device tensor of n_windows * rows * 64 bytes")
    off = 0
    if window_offsets is not None:
        if window_offsets.element_size() != 8 or window_offsets.numel() < n_windows + 1 or not window_offsets.is_cuda:
            raise ValueError("window_offsets must be a device tensor of n_windows+1 64-bit offsets")
        off = window_offsets.data_ptr()
    if rate_hist is not None and rate_hist.numel() < rate_hist_words(reg, n_windows):
        raise ValueError("rate_hist must hold n_windows * 2 * n_sites * 10001 counts")
    p = make_params(bulk_bytes, accumulate, records_per_thread, grid_blocks, workspace, rate_hist, filters, hosts,
                    flush_records)
    return c, off, p


def classify_flag(reg: Registry, rec, acc, flags, threshold_bps: int = 1_000_000, min_bulk_flows: int = 0,
                  window_offsets=None, n_windows: int = 1, bulk_bytes: int = 1_000_000, accumulate: bool = False,
                  records_per_thread: int = 0, grid_blocks: int = 0, stream=None, n: Optional[int] = None,
                  workspace=None, rate_hist=None, filters=None, hosts=None, flush_records: int = 0) -> None:
    """gnm_classify_flag: classify_aggregate then flag_suboptimal in one call (the flag
    test fused into the table merge when a workspace is given); same arguments as
    those two."""
    if flags.element_size() != 1 or flags.numel() < n_windows * reg.n_sites or not flags.is_cuda:
        raise ValueError("flags must be a device uint8 tensor of n_windows * n_sites bytes")
    c, off, p = _classify_args(reg, rec, acc, window_offsets, n_windows, bulk_bytes, accumulate, records_per_thread,
                               grid_blocks, n, workspace, rate_hist, filters, hosts, flush_records)
    _check(lib().gnm_classify_flag(reg.handle, ctypes.byref(c), ctypes.c_void_p(off), int(n_windows),
                                   ctypes.byref(p), ctypes.c_void_p(acc.data_ptr()), int(threshold_bps),
                                   int(min_bulk_flows), ctypes.c_void_p(flags.data_ptr()),
                                   _stream_handle(stream)), "gnm_classify_flag")


def classify_flag_static(reg: Registry, rec, acc, flags, threshold_bps: int = 1_000_000, min_bulk_flows: int = 0,
                         window_offsets=None, n_windows: int = 1, bulk_bytes: int = 1_000_000,
                         accumulate: bool = False, records_per_thread: int = 0, grid_blocks: int = 0, stream=None,
                         n: Optional[int] = None, rate_hist=None, filters=None, hosts=None,
                         flush_records: int = 0) -> None:
    """gnm_classify_flag_static: gnm_classify_flag with its workspace in the
    library's static device scratch (no workspace argument; the call allocates
    nothing).  Calls whose work overlaps on one GPU race on that scratch."""
    if flags.element_size() != 1 or flags.numel() < n_windows * reg.n_sites or not flags.is_cuda:
        raise ValueError("flags must be a device uint8 tensor of n_windows * n_sites bytes")
    c, off, p = _classify_args(reg, rec, acc, window_offsets, n_windows, bulk_bytes, accumulate, records_per_thread,
                               grid_blocks, n, None, rate_hist, filters, hosts, flush_records)
    _check(lib().gnm_classify_flag_static(reg.handle, ctypes.byref(c), ctypes.c_void_p(off), int(n_windows),
                                          ctypes.byref(p), ctypes.c_void_p(acc.data_ptr()), int(threshold_bps),
                                          int(min_bulk_flows), ctypes.c_void_p(flags.data_ptr()),
                                          _stream_handle(stream)), "gnm_classify_flag_static")


def static_scratch_bytes() -> int:
    """gnm_static_scratch_bytes: size of the static scratch of classify_flag_static."""
    return int(lib().gnm_static_scratch_bytes())


def flag_suboptimal(reg: Registry, acc, n_windows: int, flags, threshold_bps: int = 1_000_000,
                    min_bulk_flows: int = 0, stream=None) -> None:
    """gnm_flag_suboptimal: flags is a device uint8 tensor of n_windows*n_sites bytes."""
    if flags.element_size() != 1 or flags.numel() < n_windows * reg.n_sites or not flags.is_cuda:
        raise ValueError("flags must be a device uint8 tensor of n_windows * n_sites bytes")
    _check(lib().gnm_flag_suboptimal(reg.handle, ctypes.c_void_p(acc.data_ptr()), int(n_windows),
                                     int(threshold_bps), int(min_bulk_flows), ctypes.c_void_p(flags.data_ptr()),
                                     _stream_handle(stream)), "gnm_flag_suboptimal")


def median_flags(reg: Registry, rate_hist, n_windows: int, flags, threshold_bps: int = 1_000_000,
                 min_bulk_flows: int = 0, prev_flags=None, median_bucket=None, stream=None) -> None:
    """gnm_median_flags: lower medians of the rate histograms and the two-window warning.

    flags: device uint8 tensor of n_windows*n_sites bytes (bits 0/1 low median,
    bits 2/3 low in this window and the previous one); prev_flags: optional
    device uint8 tensor of n_sites bytes for the window before the first;
    median_bucket: optional device 32-bit tensor of n_windows*2*n_sites buckets.
    """
    if not rate_hist.is_cuda or rate_hist.element_size() != 4 or rate_hist.numel() < rate_hist_words(reg, n_windows):
        raise ValueError("rate_hist must be a device tensor of n_windows * 2 * n_sites * 10001 counts")
    if flags.element_size() != 1 or flags.numel() < n_windows * reg.n_sites or not flags.is_cuda:
        raise ValueError("flags must be a device uint8 tensor of n_windows * n_sites bytes")
    prev = 0
    if prev_flags is not None:
        if prev_flags.element_size() != 1 or prev_flags.numel() < reg.n_sites or not prev_flags.is_cuda:
            raise ValueError("prev_flags must be a device uint8 tensor of n_sites bytes")
        prev = prev_flags.data_ptr()
    med = 0
    if median_bucket is not None:
        if (median_bucket.element_size() != 4 or median_bucket.numel() < 2 * n_windows * reg.n_sites
                or not median_bucket.is_cuda):
            raise ValueError("median_bucket must be a device 32-bit tensor of n_windows * 2 * n_sites entries")
        med = median_bucket.data_ptr()
    _check(lib().gnm_median_flags(reg.handle, ctypes.c_void_p(rate_hist.data_ptr()), int(n_windows),
                                  int(threshold_bps), int(min_bulk_flows), ctypes.c_void_p(prev),
                                  ctypes.c_void_p(med), ctypes.c_void_p(flags.data_ptr()), _stream_handle(stream)),
           "gnm_median_flags")


class Graph:
    """gnm_graph_create / gnm_graph_launch / gnm_graph_free: one captured step.

    Holds references to every tensor baked into the graph so they outlive it.
    """

    def __init__(self, reg: Registry, rec, acc, window_offsets=None, n_windows: int = 1, flags=None,
                 threshold_bps: int = 1_000_000, min_bulk_flows: int = 0, n: Optional[int] = None, **params):
        self._keep = (reg, rec, acc, window_offsets, flags, params.get("workspace"), params.get("rate_hist"),
                      params.get("hosts"))
        self._rec = rec if isinstance(rec, RecordsC) else records_struct(rec, n)
        self._p = make_params(**params)
        off = 0 if window_offsets is None else window_offsets.data_ptr()
        fl = 0 if flags is None else flags.data_ptr()
        h = ctypes.c_void_p()
        _check(lib().gnm_graph_create(reg.handle, ctypes.byref(self._rec), ctypes.c_void_p(off), int(n_windows),
                                      ctypes.byref(self._p), ctypes.c_void_p(acc.data_ptr()), int(threshold_bps),
                                      int(min_bulk_flows), ctypes.c_void_p(fl), ctypes.byref(h)),
               "gnm_graph_create")
        self._h = h

    def launch(self, stream=None) -> None:
        _check(lib().gnm_graph_launch(self._h, _stream_handle(stream)), "gnm_graph_launch")

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().gnm_graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(reg: Registry, rec, acc, window_offsets=None, n_windows: int = 1, reps: int = 3,
             stream=None, n: Optional[int] = None, **params) -> Dict[str, object]:
    """gnm_autotune: fastest launch shape for this registry and these records.

    Returns {"records_per_thread", "grid_blocks", "best_ms", "tried": [(rpt, grid, ms), ...]}.
    """
    c = rec if isinstance(rec, RecordsC) else records_struct(rec, n)
    p = make_params(**params)
    off = 0 if window_offsets is None else window_offsets.data_ptr()
    out = TuneResult()
    _check(lib().gnm_autotune(reg.handle, ctypes.byref(c), ctypes.c_void_p(off), int(n_windows), ctypes.byref(p),
                              ctypes.c_void_p(acc.data_ptr()), int(reps), _stream_handle(stream),
                              ctypes.byref(out)), "gnm_autotune")
    tried = [(int(out.records_per_thread[i]), int(out.grid_blocks[i]), float(out.ms[i]))
             for i in range(out.n_tried)]
    return {"records_per_thread": int(out.best.records_per_thread), "grid_blocks": int(out.best.grid_blocks),
            "best_ms": float(out.best_ms), "tried": tried}


OUT_FIELDS = {"src_ip": 4, "dst_ip": 4, "src_port": 2, "dst_port": 2, "proto": 1, "bytes": 8, "packets": 4,
              "first_ms": 4, "last_ms": 4}


def make_records_out(capacity: int, device=None, ports: bool = True) -> Dict[str, "object"]:
    """Device tensors to decode up to `capacity` records into (ports and proto optional)."""
    import torch
    dt = {4: torch.int32, 2: torch.int16, 1: torch.uint8, 8: torch.int64}
    dev = device if device is not None else "cuda"
    return {f: torch.empty(int(capacity), dtype=dt[w], device=dev) for f, w in OUT_FIELDS.items()
            if ports or f not in ("src_port", "dst_port", "proto")}


def netflow_v5_workspace_bytes(n_datagrams: int) -> int:
    return int(lib().gnm_netflow_v5_workspace_bytes(int(n_datagrams)))


def netflow_v5_decode(datagrams, offsets, out: Dict[str, "object"], workspace=None, counts=None,
                      stream=None):
    """gnm_netflow_v5_decode: datagrams is a device uint8 tensor, offsets a
    device 64-bit tensor of n+1 offsets, out a dict from make_records_out().
    Returns a device int64 tensor [records carried, datagrams rejected]."""
    import torch
    n = offsets.numel() - 1
    if n < 0 or offsets.element_size() != 8 or not offsets.is_cuda or not datagrams.is_cuda:
        raise ValueError("offsets must be a device tensor of n+1 64-bit offsets; datagrams a device tensor")
    cap = None
    c = RecordsOutC()
    for f, w in OUT_FIELDS.items():
        t = out.get(f)
        if t is None:
            if f in ("src_port", "dst_port", "proto"):
                continue
            raise ValueError("missing output field %s" % f)
        if not t.is_cuda or not t.is_contiguous() or t.element_size() != w:
            raise ValueError("output field %s must be a contiguous device tensor of %d-byte items" % (f, w))
        cap = t.numel() if cap is None else min(cap, t.numel())
        setattr(c, f, t.data_ptr())
    c.capacity = cap
    need = netflow_v5_workspace_bytes(n)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=datagrams.device)
    if counts is None:
        counts = torch.empty(2, dtype=torch.int64, device=datagrams.device)
    _check(lib().gnm_netflow_v5_decode(ctypes.c_void_p(datagrams.data_ptr()),
                                       datagrams.numel() * datagrams.element_size(),
                                       ctypes.c_void_p(offsets.data_ptr()), n,
                                       ctypes.c_void_p(workspace.data_ptr()),
                                       workspace.numel() * workspace.element_size(), ctypes.byref(c),
                                       ctypes.c_void_p(counts.data_ptr()), ctypes.c_void_p(counts.data_ptr() + 8),
                                       _stream_handle(stream)), "gnm_netflow_v5_decode")
    return counts


def version() -> str:
    return lib().gnm_version().decode()


def acc_to_numpy(acc) -> np.ndarray:
    """Device acc tensor (int64 words) -> host uint64 array [..., rows, 8]."""
    return acc.detach().cpu().numpy().view(np.uint64)
