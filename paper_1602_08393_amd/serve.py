"""Serving loop binding (wmh_server_* in include/wmh.h) and an open-loop request driver.

The loop itself runs in libwmh: a worker thread admits queued requests as slots and device
memory free up and overlaps their walks on the device.  This module only marshals arguments
and, for benchmarking, submits requests at their scheduled (Poisson) arrival times.
"""
from __future__ import annotations

import ctypes
import gc
import time
from dataclasses import dataclass, field

import numpy as np

from . import wmh


def now_ns() -> int:
    return int(wmh.load().wmh_server_now_ns())


class PinnedBuffer:
    """Page-locked host memory from wmh_host_alloc, released when the object is collected."""

    def __init__(self, nbytes: int):
        self._lib = wmh.load()
        self.ptr = ctypes.c_void_p()
        st = self._lib.wmh_host_alloc(nbytes, ctypes.byref(self.ptr))
        if st != 0:
            raise wmh.WMHError(st, f"wmh_host_alloc of {nbytes} bytes")
        self.nbytes = nbytes

    def array(self, shape, dtype) -> np.ndarray:
        dtype = np.dtype(dtype)
        n = int(np.prod(shape))
        if n == 0:
            return np.zeros(shape, dtype=dtype)
        raw = (ctypes.c_uint8 * (n * dtype.itemsize)).from_address(self.ptr.value)
        return np.frombuffer(raw, dtype=dtype, count=n).reshape(shape)

    def __del__(self, _void=ctypes.c_void_p):
        # _void is bound at definition: at interpreter exit the module's globals may be gone
        if getattr(self, "ptr", None) and self.ptr.value:
            self._lib.wmh_host_free(self.ptr)
            self.ptr = _void()


def pinned_like(a: np.ndarray, pins: list) -> np.ndarray:
    """A copy of `a` in page-locked memory; its owner is appended to `pins`."""
    buf = PinnedBuffer(max(a.nbytes, 1))
    pins.append(buf)
    out = buf.array(a.shape, a.dtype)
    out[...] = a
    return out


@dataclass
class Request:
    row_ptr: np.ndarray  # u64 [N+1]
    col: np.ndarray      # u32 [nnz]
    val: np.ndarray      # u32 [nnz]
    sig: np.ndarray      # u16 [N, k], written on completion
    ticket: int = 0
    pins: list = field(default_factory=list)  # owners of page-locked buffers

    @property
    def n_rows(self) -> int:
        return len(self.row_ptr) - 1


class Server:
    """A serving loop on a context's device and bounds."""

    def __init__(self, ctx: "wmh.Context", k: int, seed: int = 0, slots: int = 8,
                 mem_budget: int = 0, mode: str = "auto", stream_depth: int = 0,
                 build_index: bool = False, group_rows: int = 0):
        self._lib = wmh.load()
        self.ctx = ctx
        self.k = k
        cfg = wmh.ServerConfig()
        cfg.k = k
        cfg.slots = slots
        cfg.seed = seed & 0xFFFFFFFFFFFFFFFF
        cfg.mem_budget = mem_budget
        cfg.mode = wmh.MODES[mode]
        cfg.stream_depth = stream_depth
        cfg.build_index = int(bool(build_index))
        cfg.group_rows = group_rows
        self._ptr = ctypes.c_void_p()
        ctx._check(self._lib.wmh_server_create(ctx._ptr, ctypes.byref(cfg),
                                               ctypes.byref(self._ptr)), "wmh_server_create")
        self._live: dict[int, Request] = {}

    def close(self):
        if self._ptr:
            self._lib.wmh_server_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def make_request(self, row_ptr, col, val, pinned: bool = False) -> Request:
        """A request over these rows; with `pinned` its buffers are copied to page-locked
        memory, so the loop's copies in and out are asynchronous DMA."""
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.uint64)
        col = np.ascontiguousarray(col, dtype=np.uint32)
        val = np.ascontiguousarray(val, dtype=np.uint32)
        sig = np.zeros((len(row_ptr) - 1, self.k), dtype=np.uint16)
        if not pinned:
            return Request(row_ptr, col, val, sig)
        pins: list = []
        return Request(pinned_like(row_ptr, pins), pinned_like(col, pins),
                       pinned_like(val, pins), pinned_like(sig, pins), pins=pins)

    def submit(self, req: Request, arrival_ns: int = 0) -> int:
        t = ctypes.c_uint64()
        st = self._lib.wmh_server_submit(self._ptr, req.row_ptr.ctypes.data,
                                         req.col.ctypes.data if len(req.col) else None,
                                         req.val.ctypes.data if len(req.val) else None,
                                         req.n_rows, len(req.col),
                                         req.sig.ctypes.data if req.sig.size else None,
                                         ctypes.c_uint64(arrival_ns), ctypes.byref(t))
        self.ctx._check(st, "wmh_server_submit")
        req.ticket = t.value
        self._live[t.value] = req  # keeps the buffers alive until completion
        return t.value

    def wait(self, ticket: int) -> float:
        lat = ctypes.c_double()
        st = self._lib.wmh_server_wait(self._ptr, ticket, ctypes.byref(lat))
        self._live.pop(ticket, None)
        self.ctx._check(st, "wmh_server_wait")
        return lat.value

    def poll(self, ticket: int):
        done, lat = ctypes.c_int(), ctypes.c_double()
        st = self._lib.wmh_server_poll(self._ptr, ticket, ctypes.byref(done), ctypes.byref(lat))
        if done.value:
            self._live.pop(ticket, None)
        self.ctx._check(st, "wmh_server_poll")
        return (lat.value if done.value else None)

    def drain(self):
        self.ctx._check(self._lib.wmh_server_drain(self._ptr), "wmh_server_drain")

    def reserve(self, max_rows: int, max_nnz: int):
        """Sizes every slot's buffers for requests of up to max_rows rows and max_nnz
        nonzeros (wmh_server_reserve), so that admitting them allocates nothing."""
        self.ctx._check(self._lib.wmh_server_reserve(self._ptr, ctypes.c_uint64(max_rows),
                                                     ctypes.c_uint64(max_nnz)),
                        "wmh_server_reserve")

    def reset_stats(self):
        self.ctx._check(self._lib.wmh_server_reset_stats(self._ptr), "wmh_server_reset_stats")

    def stats(self) -> dict:
        s = wmh.ServingStats()
        self.ctx._check(self._lib.wmh_server_stats(self._ptr, ctypes.byref(s)),
                        "wmh_server_stats")
        return {name: getattr(s, name) for name, _ in wmh.ServingStats._fields_}


def requests_from_corpus(ds, row_lists, server: Server, pinned: bool = False) -> list[Request]:
    """One Request per list of corpus row indices (rows copied out of the corpus, into
    page-locked buffers with `pinned`)."""
    out = []
    rp = ds.row_ptr.astype(np.int64)
    for rows in row_lists:
        rows = np.asarray(rows, dtype=np.int64)
        lengths = rp[rows + 1] - rp[rows]
        row_ptr = np.zeros(len(rows) + 1, dtype=np.uint64)
        row_ptr[1:] = np.cumsum(lengths)
        if lengths.sum():
            idx = np.concatenate([np.arange(a, b) for a, b in zip(rp[rows], rp[rows + 1])])
        else:
            idx = np.zeros(0, dtype=np.int64)
        out.append(server.make_request(row_ptr, ds.col[idx], ds.val[idx], pinned=pinned))
    return out


class RangeRequests:
    """Requests over runs of consecutive corpus rows without copying the rows: the corpus's
    col and val sit once in page-locked memory and each request points into them; its row_ptr
    (rebased to 0) and its signatures use one of `ring` page-locked buffer pairs in turn.  A
    pair is reused only once the request that last used it has completed."""

    def __init__(self, server: Server, ds, max_rows: int, ring: int = 512):
        self.server = server
        self.k = server.k
        self.rp = ds.row_ptr.astype(np.uint64)
        self.pins: list = []
        self.col = pinned_like(ds.col, self.pins)
        self.val = pinned_like(ds.val, self.pins)
        self.row_ptr_buf = [PinnedBuffer((max_rows + 1) * 8) for _ in range(ring)]
        self.sig_buf = [PinnedBuffer(max(max_rows * self.k * 2, 2)) for _ in range(ring)]
        self.last: list = [None] * ring
        self.n = 0
        self.reused_waits = 0

    def make(self, start: int, n_rows: int) -> Request:
        i = self.n % len(self.row_ptr_buf)
        self.n += 1
        prev = self.last[i]
        if prev is not None and prev.ticket in self.server._live:
            if self.server.poll(prev.ticket) is None:  # still in flight: wait for it
                self.reused_waits += 1
                self.server.wait(prev.ticket)
        lo, hi = int(self.rp[start]), int(self.rp[start + n_rows])
        row_ptr = self.row_ptr_buf[i].array((n_rows + 1,), np.uint64)
        np.subtract(self.rp[start:start + n_rows + 1], np.uint64(lo), out=row_ptr)
        sig = self.sig_buf[i].array((n_rows, self.k), np.uint16)
        req = Request(row_ptr, self.col[lo:hi], self.val[lo:hi], sig)
        self.last[i] = req
        return req


def run_open_loop(server: Server, requests, arrivals_s: np.ndarray) -> dict:
    """Submits request i at t0 + arrivals_s[i] (open loop: the schedule never waits for
    completions) with that scheduled time as its arrival, then drains and returns stats, with
    the driver's own lateness (actual submission after the scheduled time) added: latencies
    count from the scheduled time, so a late driver shows up as queueing.  Python's cyclic
    garbage collector is paused while requests are submitted, so none of its passes delays
    the schedule.  `requests` is a list of Requests or a function of i that makes request i
    (called before its due time)."""
    late = np.zeros(len(arrivals_s))
    gc_was_on = gc.isenabled()
    gc.collect()
    gc.disable()
    try:
        t0 = now_ns() + 2_000_000
        for i, a in enumerate(arrivals_s):
            req = requests(i) if callable(requests) else requests[i]
            due = t0 + int(a * 1e9)
            while True:
                left = due - now_ns()
                if left <= 0:
                    break
                time.sleep(min(left, 2_000_000) / 1e9 if left > 200_000 else 0)
            late[i] = (now_ns() - due) * 1e-6
            server.submit(req, arrival_ns=due)
        server.drain()
        for ticket in list(server._live):
            server.wait(ticket)
    finally:
        if gc_was_on:
            gc.enable()
    st = server.stats()
    if len(late):
        st["driver_late_p99_ms"] = float(np.quantile(late, 0.99))
        st["driver_late_max_ms"] = float(late.max())
    return st
