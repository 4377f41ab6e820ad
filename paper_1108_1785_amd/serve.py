"""Served form: a request loop with admission by device memory and continuous
batching over the C ABI.

The paper processes one window per hourly launch (§III.B.1, NetPerf
Monitoring Thread).  Here windows arrive at any time:

* admission — each window needs room for its records in a device ring arena
  (the memory budget); a window waits until earlier windows free enough
  contiguous space, and one larger than the whole arena is rejected;
* overlap — admitted windows are copied host->device on a copy stream while
  earlier windows are being classified on the compute stream;
* continuous batching — whenever fewer than `max_inflight` launches are
  running, every admitted window whose copy has finished, consecutive in the
  arena, goes into one persistent classify launch (gnm_classify_flag with
  window offsets: the classify launch, then the table merge with the flag
  test);
* isolation — every window has its own accumulator rows, so a window's result
  is the same alone and in any mix.

The scheduler is independent of the device: it drives an executor object
(GpuExecutor for the library; tests may substitute a fake one).
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from typing import Deque, Dict, List, Optional, Tuple

import numpy as np

RECORD_FIELDS = ("src_ip", "dst_ip", "bytes", "packets", "first_ms", "last_ms")
RECORD_BYTES = 28  # device bytes per record in the arena (the fields read)


class AdmissionError(RuntimeError):
    """A window that can never fit the device arena."""


class RingArena:
    """First-in first-out allocator of record slots in a ring of `capacity`.

    Allocations are contiguous and non-empty; they are freed in allocation
    order (batches complete in launch order).  The occupied region runs from
    the oldest allocation to the newest, wrapping past the end at most once.
    """

    def __init__(self, capacity: int):
        self.capacity = int(capacity)
        self.live: Deque[Tuple[int, int]] = collections.deque()  # (offset, n), oldest first

    @property
    def head(self) -> int:
        """Where the next allocation would start if it fits without wrapping."""
        return self.live[-1][0] + self.live[-1][1] if self.live else 0

    def alloc(self, n: int) -> Optional[int]:
        if n <= 0:
            raise ValueError("allocations are non-empty")
        if n > self.capacity:
            raise AdmissionError("window of %d records exceeds the arena of %d" % (n, self.capacity))
        if not self.live:
            off = 0
        else:
            tail, head = self.live[0][0], self.head
            if self.live[-1][0] >= tail:  # occupied [tail, head)
                if self.capacity - head >= n:
                    off = head
                elif tail >= n:
                    off = 0
                else:
                    return None
            else:  # wrapped: occupied [tail, capacity) and [0, head)
                if tail - head >= n:
                    off = head
                else:
                    return None
        self.live.append((off, n))
        return off

    def free_oldest(self) -> None:
        self.live.popleft()

    @property
    def used(self) -> int:
        return sum(n for _, n in self.live)


class Request:
    __slots__ = ("rid", "records", "n", "t_arrival", "future", "offset", "copy_event", "ready", "t_done")

    def __init__(self, rid: int, records, n: int, t_arrival: float, ready=None):
        self.rid, self.records, self.n, self.t_arrival = rid, records, n, t_arrival
        self.future: Future = Future()
        self.offset = -1
        self.copy_event = None
        self.ready = ready  # device event after which the records may be read (None: at once)
        self.t_done = 0.0


def pin_records(rec, lo: int = 0, hi: Optional[int] = None) -> Dict[str, object]:
    """Pinned host torch tensors of records [lo, hi) of a SoA record set.

    `rec` has numpy fields src_ip, dst_ip, packets, first_ms, last_ms (32-bit)
    and bytes (64-bit).  Pinned memory lets the copy stream move a window to
    the device asynchronously.
    """
    import torch
    hi = rec.n if hi is None else hi
    out = {}
    for f in RECORD_FIELDS:
        a = np.ascontiguousarray(getattr(rec, f)[lo:hi])
        a = a.view(np.int64 if f == "bytes" else np.int32)
        t = torch.empty(a.shape, dtype=torch.int64 if f == "bytes" else torch.int32, pin_memory=True)
        t.numpy()[:] = a
        out[f] = t
    return out


class GpuExecutor:
    """Device side of the server: arena buffers, streams and launches via libgnm."""

    def __init__(self, reg, capacity: Optional[int] = None, max_batch_windows: int = 1024, max_inflight: int = 2,
                 bulk_bytes: int = 1_000_000, threshold_bps: int = 1_000_000, min_bulk_flows: int = 0,
                 device: str = "cuda:0", mem_budget_bytes: Optional[int] = None, free_fraction: float = 0.25):
        """Arena of `capacity` records; else `mem_budget_bytes` / 28 B; else a
        `free_fraction` of the device memory free now (admission by free HBM)."""
        import torch

        from . import lib, make_workspace
        lib()
        self.torch, self.reg, self.dev = torch, reg, device
        if capacity is None:
            if mem_budget_bytes is None:
                free, _ = torch.cuda.mem_get_info(torch.device(device))
                mem_budget_bytes = int(free * free_fraction)
            capacity = int(mem_budget_bytes) // RECORD_BYTES
        if capacity <= 0:
            raise ValueError("arena capacity must be positive")
        self.capacity, self.max_w = int(capacity), int(max_batch_windows)
        self.bulk_bytes, self.threshold, self.min_bulk = bulk_bytes, threshold_bps, min_bulk_flows
        self.rows, self.n_sites = reg.rows, reg.n_sites
        i32, i64 = torch.int32, torch.int64
        self.buf = {f: torch.empty(self.capacity, dtype=i64 if f == "bytes" else i32, device=device)
                    for f in RECORD_FIELDS}
        self.copy_stream = torch.cuda.Stream(device=device)     # default priority
        self.compute_stream = torch.cuda.Stream(device=device)  # default priority
        self.slots = []
        for _ in range(max_inflight):
            self.slots.append({
                "acc": torch.empty((self.max_w, self.rows, 8), dtype=i64, device=device),
                "flags": torch.empty(self.max_w * self.n_sites, dtype=torch.uint8, device=device),
                "off_host": torch.empty(self.max_w + 1, dtype=i64, pin_memory=True),
                "off_dev": torch.empty(self.max_w + 1, dtype=i64, device=device),
                "acc_host": torch.empty((self.max_w, self.rows, 8), dtype=i64, pin_memory=True),
                "flags_host": torch.empty(self.max_w * self.n_sites, dtype=torch.uint8, pin_memory=True),
                "ws": make_workspace(reg, device=device),
                "event": None, "busy": False,
            })

    def thread_init(self) -> None:
        """Called once on the scheduler thread before it issues device work."""
        self.torch.cuda.set_device(self.torch.device(self.dev))

    def producer_event(self, records):
        """Called by submit() on the caller's thread.  Records already in device
        memory may still be being written by work the caller queued on its
        current stream (a decode kernel, a copy): an event recorded there now
        orders the staging copy after that work.  None for host records."""
        torch = self.torch
        if not any(getattr(records.get(f), "is_cuda", False) for f in RECORD_FIELDS):
            return None
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream(torch.device(self.dev)))
        return ev

    def _wait_ready(self, reqs: List[Request]) -> None:
        for r in reqs:
            if r.ready is not None:
                self.copy_stream.wait_event(r.ready)

    def start_copy(self, req: Request):
        """Asynchronous host->device copy of the request's records into the arena."""
        torch = self.torch
        if req.n == 0:
            return None
        self._wait_ready([req])
        with torch.cuda.stream(self.copy_stream):
            for f in RECORD_FIELDS:
                self.buf[f][req.offset:req.offset + req.n].copy_(req.records[f], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.copy_stream)
        return ev

    def start_copy_group(self, reqs: List[Request]) -> None:
        """Stage requests that were admitted together and sit back to back in the
        arena.  Device-resident records go in with one concatenating copy per
        field for the whole group (one event for all of them), rather than a
        copy per field and window; host records keep their own copies."""
        torch = self.torch
        live = [r for r in reqs if r.n]
        on_device = all(getattr(r.records[f], "is_cuda", False) for r in live for f in RECORD_FIELDS)
        contiguous = all(b.offset == a.offset + a.n for a, b in zip(live, live[1:]))
        if len(live) < 2 or not on_device or not contiguous:
            for r in reqs:
                r.copy_event = self.start_copy(r)
            return
        lo, hi = live[0].offset, live[-1].offset + live[-1].n
        self._wait_ready(live)
        with torch.cuda.stream(self.copy_stream):
            for f in RECORD_FIELDS:
                torch.cat([r.records[f][:r.n] for r in live], out=self.buf[f][lo:hi])
            ev = torch.cuda.Event()
            ev.record(self.copy_stream)
        for r in reqs:
            r.copy_event = ev if r.n else None

    @staticmethod
    def done(event) -> bool:
        return event is None or event.query()

    def free_slot(self) -> Optional[int]:
        for i, s in enumerate(self.slots):
            if not s["busy"]:
                return i
        return None

    def launch(self, slot: int, batch: List[Request]) -> None:
        """One persistent classify launch over consecutive arena windows, then flags and D2H."""
        from . import classify_flag, records_struct
        torch = self.torch
        s = self.slots[slot]
        base = batch[0].offset
        total = batch[-1].offset + batch[-1].n - base
        nw = len(batch)
        offs = np.zeros(nw + 1, dtype=np.int64)
        np.cumsum([r.n for r in batch], out=offs[1:])
        s["off_host"][:nw + 1].copy_(torch.from_numpy(offs))
        st = self.compute_stream
        with torch.cuda.stream(st):
            for r in batch:  # the launch reads records only after their copies
                if r.copy_event is not None:
                    st.wait_event(r.copy_event)
            s["off_dev"][:nw + 1].copy_(s["off_host"][:nw + 1], non_blocking=True)
            view = {f: self.buf[f][base:base + max(total, 1)] for f in RECORD_FIELDS}
            rec = records_struct(view, total)
            classify_flag(self.reg, rec, s["acc"], s["flags"], self.threshold, self.min_bulk,
                          window_offsets=s["off_dev"], n_windows=nw, bulk_bytes=self.bulk_bytes,
                          workspace=s["ws"], stream=st)
            s["acc_host"][:nw].copy_(s["acc"][:nw], non_blocking=True)
            s["flags_host"][:nw * self.n_sites].copy_(s["flags"][:nw * self.n_sites], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
        s["event"], s["busy"], s["batch"] = ev, True, batch

    def poll(self, slot: int) -> Optional[Tuple[np.ndarray, np.ndarray]]:
        """Per-window tables and flags of a finished launch (None while running)."""
        s = self.slots[slot]
        if not s["busy"] or not s["event"].query():
            return None
        nw = len(s["batch"])
        acc = s["acc_host"][:nw].numpy().view(np.uint64).copy()
        flags = s["flags_host"][:nw * self.n_sites].numpy().reshape(nw, self.n_sites).copy()
        s["busy"], s["event"], s["batch"] = False, None, None
        return acc, flags


class WindowResult:
    __slots__ = ("acc", "flags", "latency_s", "n_records", "rid")

    def __init__(self, rid, acc, flags, latency_s, n_records):
        self.rid, self.acc, self.flags, self.latency_s, self.n_records = rid, acc, flags, latency_s, n_records


class Server:
    """Continuously batching request loop over an executor (see module doc)."""

    def __init__(self, executor, capacity: Optional[int] = None, max_batch_windows: Optional[int] = None,
                 idle_sleep_s: float = 20e-6):
        self.ex = executor
        self.arena = RingArena(capacity if capacity is not None else executor.capacity)
        self.max_w = max_batch_windows if max_batch_windows is not None else executor.max_w
        self.idle = idle_sleep_s
        self.waiting: Deque[Request] = collections.deque()   # not yet admitted
        self.copying: Deque[Request] = collections.deque()   # admitted, copy in flight or done
        self.inflight: Deque[Tuple[int, List[Request]]] = collections.deque()  # (slot, batch)
        self.lock = threading.Lock()
        self.wake = threading.Event()
        self.stop = False
        self.next_id = 0
        self.stats = collections.Counter()
        self.thread = threading.Thread(target=self._loop, name="gnm-serve", daemon=True)
        self.thread.start()

    def submit(self, records: Dict[str, object], n: Optional[int] = None,
               t_arrival: Optional[float] = None) -> Future:
        """Queue one window; the future resolves to a WindowResult."""
        if n is None:
            n = int(len(records["src_ip"]))
        if n > self.arena.capacity:
            f: Future = Future()
            f.set_exception(AdmissionError("window of %d records exceeds the arena of %d"
                                           % (n, self.arena.capacity)))
            return f
        mark = getattr(self.ex, "producer_event", None)
        ready = mark(records) if mark is not None and n else None
        with self.lock:
            req = Request(self.next_id, records, n, time.perf_counter() if t_arrival is None else t_arrival, ready)
            self.next_id += 1
            self.waiting.append(req)
        self.wake.set()
        return req.future

    def close(self, timeout: float = 60.0) -> None:
        self.stop = True
        self.wake.set()
        self.thread.join(timeout)

    # ------------------------------------------------------------ scheduler
    def _admit(self) -> bool:
        # admit what the arena can take now, then stage it: runs of windows
        # that landed back to back are staged together
        group: List[Request] = []
        while True:
            with self.lock:
                if not self.waiting:
                    break
                req = self.waiting[0]
                off = self._alloc(req)
                if off is None:
                    self.stats["admission_waits"] += 1
                    break
                self.waiting.popleft()
            req.offset = off
            group.append(req)
        if not group:
            return False
        stage = getattr(self.ex, "start_copy_group", None)
        run: List[Request] = []
        for req in group + [None]:
            if req is not None and (not run or not req.n or not run[-1].n or
                                    req.offset == run[-1].offset + run[-1].n):
                run.append(req)
                continue
            self.copying.extend(run)  # pending before staging: a failure fails them too
            if stage is not None:
                stage(run)
            else:
                for r in run:
                    r.copy_event = self.ex.start_copy(r)
            run = [req] if req is not None else []
        return True

    def _alloc(self, req: Request) -> Optional[int]:
        # empty windows take no arena space and sit at the current head
        return self.arena.head if req.n == 0 else self.arena.alloc(req.n)

    def _launch(self) -> bool:
        if not self.copying:
            return False
        slot = self.ex.free_slot()
        if slot is None:
            return False
        batch: List[Request] = []
        for req in self.copying:
            if len(batch) >= self.max_w or not self.ex.done(req.copy_event):
                break
            if batch and req.offset != batch[-1].offset + batch[-1].n:
                break  # the arena wrapped: next launch
            batch.append(req)
        if not batch:
            return False
        self.ex.launch(slot, batch)  # on failure the batch is still pending and gets failed
        for _ in batch:
            self.copying.popleft()
        self.inflight.append((slot, batch))
        self.stats["launches"] += 1
        self.stats["windows"] += len(batch)
        return True

    def _complete(self) -> bool:
        if not self.inflight:
            return False
        slot, batch = self.inflight[0]
        res = self.ex.poll(slot)
        if res is None:
            return False
        self.inflight.popleft()
        acc, flags = res
        now = time.perf_counter()
        with self.lock:
            for req in batch:
                if req.n:
                    self.arena.free_oldest()
        for i, req in enumerate(batch):
            req.t_done = now
            req.future.set_result(WindowResult(req.rid, acc[i], flags[i], now - req.t_arrival, req.n))
        return True

    def _loop(self) -> None:
        init = getattr(self.ex, "thread_init", None)
        if init is not None:
            init()
        while True:
            try:
                busy = self._complete()
                busy |= self._admit()
                busy |= self._launch()
            except Exception as e:  # fail every pending request rather than hang
                self._fail_all(e)
                return
            if self.stop and not (self.waiting or self.copying or self.inflight):
                return
            if not busy:
                if not (self.waiting or self.copying or self.inflight):
                    self.wake.wait(0.01)
                    self.wake.clear()
                else:
                    time.sleep(self.idle)

    def _fail_all(self, e: Exception) -> None:
        with self.lock:
            reqs = list(self.waiting) + list(self.copying) + [r for _, b in self.inflight for r in b]
            self.waiting.clear()
            self.copying.clear()
            self.inflight.clear()
        for r in reqs:
            if not r.future.done():
                r.future.set_exception(e)
