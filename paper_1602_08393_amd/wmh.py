"""Python binding of libwmh (include/wmh.h): argument marshalling only.

Every computation runs in the library's HIP kernels; torch supplies device memory and streams.
If ``libwmh.so`` has not been built this module raises on first use -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwmh.so")

CAP = 65535

STATUS = {0: "WMH_OK", -1: "WMH_E_ARG", -2: "WMH_E_NO_BOUNDS", -3: "WMH_E_COL_RANGE",
          -4: "WMH_E_UNSORTED", -5: "WMH_E_BOUND", -6: "WMH_E_OVERFLOW", -7: "WMH_E_NOMEM",
          -8: "WMH_E_DEVICE", -9: "WMH_E_ROW_PTR"}
NOALLOC_SCRATCH_BYTES = 16 << 20  # WMH_NOALLOC_SCRATCH_BYTES: wmh_hash_noalloc's static array
MODES = {"auto": 0, "plain": 1, "batched": 2, "indexed": 3, "split": 4, "plain_shared": 5}
WALKS = {"auto": 0, "shared": 1, "rows": 2, "ballot": 3, "index": 4}
VALUES = {"auto": 0, "exact": 1, "coarse": 2}  # wmh_opts.values: dense rows in LDS

EXPORTED = ["wmh_opts_init", "wmh_create", "wmh_destroy", "wmh_set_bounds", "wmh_hash",
            "wmh_hash_noalloc",
            "wmh_estimate", "wmh_estimate_pair", "wmh_collisions", "wmh_bounds_info", "wmh_bounds_tables",
            "wmh_draws", "wmh_last_kernel_ms", "wmh_last_mode", "wmh_last_plan",
            "wmh_tune", "wmh_tune_save", "wmh_tune_load", "wmh_pack_words", "wmh_sig_bits",
            "wmh_pack", "wmh_unpack", "wmh_packed_collisions", "wmh_packed_estimate",
            "wmh_choose_scale", "wmh_quantize", "wmh_lsh_build", "wmh_lsh_query",
            "wmh_lsh_destroy",
            "wmh_last_error", "wmh_status_string",
            "wmh_server_create", "wmh_server_submit", "wmh_server_poll", "wmh_server_wait",
            "wmh_server_drain", "wmh_server_stats", "wmh_server_reset_stats",
            "wmh_server_reserve",
            "wmh_server_now_ns", "wmh_server_destroy",
            "wmh_host_alloc", "wmh_host_free"]


class WmhOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("batch_rows", ctypes.c_uint32),
                ("validate", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("sync", ctypes.c_int32), ("rows_per_block", ctypes.c_uint32),
                ("hashes_per_tile", ctypes.c_uint32), ("stream_depth", ctypes.c_uint32),
                ("waves_per_block", ctypes.c_uint32), ("profile", ctypes.c_int32),
                ("walk", ctypes.c_int32), ("steps_per_lane", ctypes.c_uint32),
                ("index_batch", ctypes.c_uint32), ("index_claim", ctypes.c_uint32),
                ("hash_groups", ctypes.c_uint32), ("values", ctypes.c_int32),
                ("coarse_bits", ctypes.c_uint32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("slots", ctypes.c_uint32), ("seed", ctypes.c_uint64),
                ("mem_budget", ctypes.c_uint64), ("mode", ctypes.c_int32),
                ("stream_depth", ctypes.c_uint32), ("build_index", ctypes.c_int32),
                ("group_rows", ctypes.c_uint32), ("reserved", ctypes.c_uint32 * 2)]


class ServingStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("queued", ctypes.c_uint64),
                ("max_queued", ctypes.c_uint64), ("peak_bytes", ctypes.c_uint64),
                ("hashes", ctypes.c_uint64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("p999_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("busy_s", ctypes.c_double), ("hashes_per_s", ctypes.c_double),
                ("rejected", ctypes.c_uint64), ("max_on_device", ctypes.c_uint64),
                ("max_computing", ctypes.c_uint64), ("overlap_s", ctypes.c_double),
                ("loads", ctypes.c_uint64)]


class TuneResult(ctypes.Structure):
    _fields_ = [("rows_per_block", ctypes.c_uint32), ("hashes_per_tile", ctypes.c_uint32),
                ("waves_per_block", ctypes.c_uint32), ("stream_depth", ctypes.c_uint32),
                ("best_ms", ctypes.c_float), ("default_ms", ctypes.c_float),
                ("candidates", ctypes.c_uint32), ("steps_class", ctypes.c_int32),
                ("walk", ctypes.c_int32), ("steps_per_lane", ctypes.c_uint32),
                ("index_batch", ctypes.c_uint32), ("index_claim", ctypes.c_uint32),
                ("hash_groups", ctypes.c_uint32), ("values", ctypes.c_int32),
                ("reserved", ctypes.c_uint32 * 2)]


class WMHError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__(f"{self.name}: {detail}")


_lib = None


def load() -> ctypes.CDLL:
    """Loads libwmh.so; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                           "python -m paper_1602_08393_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
    L.wmh_opts_init.argtypes = [ctypes.POINTER(WmhOpts)]
    L.wmh_opts_init.restype = None
    L.wmh_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
    L.wmh_create.restype = ctypes.c_int
    L.wmh_destroy.argtypes = [vp]
    L.wmh_destroy.restype = None
    L.wmh_set_bounds.argtypes = [vp, vp, u32]
    L.wmh_set_bounds.restype = ctypes.c_int
    L.wmh_hash.argtypes = [vp, vp, vp, vp, u64, u64, u32, u64, vp, vp, ctypes.POINTER(WmhOpts)]
    L.wmh_hash.restype = ctypes.c_int
    L.wmh_hash_noalloc.argtypes = [vp, vp, vp, vp, u64, u64, u32, u64, vp, vp,
                                   ctypes.POINTER(WmhOpts)]
    L.wmh_hash_noalloc.restype = ctypes.c_int
    L.wmh_estimate.argtypes = [vp, vp, vp, u64, u32, vp, vp, vp]
    L.wmh_estimate.restype = ctypes.c_int
    L.wmh_estimate_pair.argtypes = [vp, vp, u32, ctypes.POINTER(u32),
                                    ctypes.POINTER(ctypes.c_double)]
    L.wmh_estimate_pair.restype = ctypes.c_int
    L.wmh_collisions.argtypes = [vp, vp, u64, vp, u64, u32, vp, vp]
    L.wmh_collisions.restype = ctypes.c_int
    L.wmh_bounds_info.argtypes = [vp, ctypes.POINTER(u32), ctypes.POINTER(u64),
                                  ctypes.POINTER(u32), ctypes.POINTER(u64)]
    L.wmh_bounds_info.restype = ctypes.c_int
    L.wmh_bounds_tables.argtypes = [vp, u32, vp, vp, ctypes.POINTER(u32), ctypes.POINTER(u64),
                                    ctypes.POINTER(u64)]
    L.wmh_bounds_tables.restype = ctypes.c_int
    L.wmh_last_kernel_ms.argtypes = [vp, ctypes.POINTER(ctypes.c_float),
                                     ctypes.POINTER(ctypes.c_float)]
    L.wmh_last_kernel_ms.restype = ctypes.c_int
    L.wmh_last_mode.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.wmh_last_mode.restype = ctypes.c_int
    L.wmh_last_plan.argtypes = [vp, ctypes.POINTER(WmhOpts)]
    L.wmh_last_plan.restype = ctypes.c_int
    L.wmh_tune.argtypes = [vp, vp, vp, vp, u64, u64, u32, u64, vp, vp, u32,
                           ctypes.POINTER(TuneResult)]
    L.wmh_tune.restype = ctypes.c_int
    L.wmh_tune_save.argtypes = [vp, ctypes.c_char_p]
    L.wmh_tune_save.restype = ctypes.c_int
    L.wmh_tune_load.argtypes = [vp, ctypes.c_char_p]
    L.wmh_tune_load.restype = ctypes.c_int
    L.wmh_pack_words.argtypes = [u32, u32]
    L.wmh_pack_words.restype = ctypes.c_uint32
    L.wmh_sig_bits.argtypes = [vp, vp, u64, u32, ctypes.POINTER(u32), ctypes.POINTER(u32), vp]
    L.wmh_sig_bits.restype = ctypes.c_int
    L.wmh_pack.argtypes = [vp, vp, u64, u32, u32, vp, ctypes.POINTER(u64), vp]
    L.wmh_pack.restype = ctypes.c_int
    L.wmh_unpack.argtypes = [vp, vp, u64, u32, u32, vp, vp]
    L.wmh_unpack.restype = ctypes.c_int
    L.wmh_packed_collisions.argtypes = [vp, vp, u64, vp, u64, u32, u32, vp, vp]
    L.wmh_packed_collisions.restype = ctypes.c_int
    L.wmh_packed_estimate.argtypes = [vp, vp, vp, u64, u32, u32, vp, vp, vp]
    L.wmh_packed_estimate.restype = ctypes.c_int
    L.wmh_choose_scale.argtypes = [vp, u32, u32, u32, u32, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double), vp]
    L.wmh_choose_scale.restype = ctypes.c_int
    L.wmh_quantize.argtypes = [vp, vp, vp, u64, ctypes.c_double, vp, ctypes.POINTER(u64), vp]
    L.wmh_quantize.restype = ctypes.c_int
    L.wmh_lsh_build.argtypes = [vp, vp, u64, u32, u32, u32, vp, ctypes.POINTER(vp)]
    L.wmh_lsh_build.restype = ctypes.c_int
    L.wmh_lsh_query.argtypes = [vp, vp, u64, u32, u32, vp, vp, vp]
    L.wmh_lsh_query.restype = ctypes.c_int
    L.wmh_lsh_destroy.argtypes = [vp]
    L.wmh_lsh_destroy.restype = None
    L.wmh_draws.argtypes = [vp, u64, u32, u32, u32, vp, vp, vp, vp]
    L.wmh_draws.restype = ctypes.c_int
    L.wmh_server_create.argtypes = [vp, ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
    L.wmh_server_create.restype = ctypes.c_int
    L.wmh_server_submit.argtypes = [vp, vp, vp, vp, u64, u64, vp, u64, ctypes.POINTER(u64)]
    L.wmh_server_submit.restype = ctypes.c_int
    L.wmh_server_poll.argtypes = [vp, u64, ctypes.POINTER(ctypes.c_int),
                                  ctypes.POINTER(ctypes.c_double)]
    L.wmh_server_poll.restype = ctypes.c_int
    L.wmh_server_wait.argtypes = [vp, u64, ctypes.POINTER(ctypes.c_double)]
    L.wmh_server_wait.restype = ctypes.c_int
    L.wmh_server_drain.argtypes = [vp]
    L.wmh_server_drain.restype = ctypes.c_int
    L.wmh_server_stats.argtypes = [vp, ctypes.POINTER(ServingStats)]
    L.wmh_server_stats.restype = ctypes.c_int
    L.wmh_server_reset_stats.argtypes = [vp]
    L.wmh_server_reset_stats.restype = ctypes.c_int
    L.wmh_server_now_ns.argtypes = []
    L.wmh_server_now_ns.restype = ctypes.c_uint64
    L.wmh_server_destroy.argtypes = [vp]
    L.wmh_server_destroy.restype = None
    L.wmh_host_alloc.argtypes = [ctypes.c_size_t, ctypes.POINTER(vp)]
    L.wmh_host_alloc.restype = ctypes.c_int
    L.wmh_host_free.argtypes = [vp]
    L.wmh_host_free.restype = None
    L.wmh_last_error.argtypes = [vp]
    L.wmh_last_error.restype = ctypes.c_char_p
    L.wmh_status_string.argtypes = [ctypes.c_int]
    L.wmh_status_string.restype = ctypes.c_char_p
    _lib = L
    return L


def choose_scale(m, limit: int = 0, components: int = 0, steps: int = 0):
    """Host-only scale choice (see wmh_choose_scale): (alpha, efficiency, integer bounds)."""
    m = np.ascontiguousarray(m, dtype=np.float64)
    mq = np.zeros(len(m), dtype=np.uint32)
    a, eff = ctypes.c_double(), ctypes.c_double()
    st = load().wmh_choose_scale(m.ctypes.data, len(m), limit, components, steps,
                                 ctypes.byref(a), ctypes.byref(eff), mq.ctypes.data)
    if st != 0:
        raise WMHError(st, "wmh_choose_scale")
    return a.value, eff.value, mq


def estimate_pair(a, b):
    """Host-only estimate of one pair of host signatures (see wmh_estimate_pair): (count, jhat)."""
    a = np.ascontiguousarray(a, dtype=np.uint16)
    b = np.ascontiguousarray(b, dtype=np.uint16)
    if a.shape != b.shape or a.ndim != 1:
        raise ValueError("two signatures of the same length expected")
    count, jhat = ctypes.c_uint32(), ctypes.c_double()
    st = load().wmh_estimate_pair(a.ctypes.data, b.ctypes.data, len(a), ctypes.byref(count),
                                  ctypes.byref(jhat))
    if st != 0:
        raise WMHError(st, "wmh_estimate_pair")
    return count.value, jhat.value


def bounds_tables(m: np.ndarray) -> dict:
    """Host-only: prefix sums, bucket table, shift and threshold (no device needed)."""
    L = load()
    m = np.ascontiguousarray(m, dtype=np.uint32)
    shift, nb, thr = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint64()
    st = L.wmh_bounds_tables(m.ctypes.data, len(m), None, None, ctypes.byref(shift),
                             ctypes.byref(nb), ctypes.byref(thr))
    if st != 0:
        raise WMHError(st, "wmh_bounds_tables")
    prefix = np.zeros(len(m) + 1, dtype=np.uint64)
    bucket = np.zeros(nb.value + 1, dtype=np.uint32)
    st = L.wmh_bounds_tables(m.ctypes.data, len(m), prefix.ctypes.data, bucket.ctypes.data,
                             None, None, None)
    if st != 0:
        raise WMHError(st, "wmh_bounds_tables")
    return {"prefix": prefix, "bucket": bucket, "shift": shift.value, "n_buckets": nb.value,
            "threshold": thr.value}


def _torch():
    import torch
    return torch


@dataclass
class DeviceRows:
    """CSR rows resident on the device (torch tensors; unsigned data in signed containers)."""
    row_ptr: object  # int64 [N+1]
    col: object      # int32 [nnz]
    val: object      # int32 [nnz]
    n_rows: int
    nnz: int


def upload_rows(row_ptr: np.ndarray, col: np.ndarray, val: np.ndarray, device="cuda") \
        -> DeviceRows:
    torch = _torch()
    rp = torch.from_numpy(np.ascontiguousarray(row_ptr, dtype=np.uint64).view(np.int64))
    c = torch.from_numpy(np.ascontiguousarray(col, dtype=np.uint32).view(np.int32))
    v = torch.from_numpy(np.ascontiguousarray(val, dtype=np.uint32).view(np.int32))
    n = len(row_ptr) - 1
    return DeviceRows(rp.to(device), c.to(device), v.to(device), n, len(col))


def upload_dataset(ds, device="cuda") -> DeviceRows:
    return upload_rows(ds.row_ptr, ds.col, ds.val, device)


def sig_to_numpy(sig) -> np.ndarray:
    return sig.cpu().numpy().view(np.uint16)


class LshIndex:
    """A (K, L) banding index owned by a Context (see wmh_lsh_build / wmh_lsh_query)."""

    def __init__(self, ctx: "Context", ptr, k: int):
        self._ctx, self._ptr, self.k = ctx, ptr, k

    def query(self, q, max_out: int, stream=None):
        """(candidates int32 [Q, max_out], counts int32 [Q]) as device tensors; rows in
        increasing order, count 0xFFFFFFFF (-1 as int32) when a query overflows."""
        torch = _torch()
        nq = q.shape[0]
        out = torch.full((nq, max(max_out, 1)), -1, dtype=torch.int32, device=q.device)
        cnt = torch.empty(nq, dtype=torch.int32, device=q.device)
        self._ctx._check(self._ctx._lib.wmh_lsh_query(self._ptr, q.data_ptr(), nq, self.k,
                                                      max_out, out.data_ptr(), cnt.data_ptr(),
                                                      self._ctx._stream(stream)), "wmh_lsh_query")
        return out, cnt

    def close(self):
        if self._ptr:
            self._ctx._lib.wmh_lsh_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """One libwmh context on a HIP device."""

    def __init__(self, device: int = 0):
        self._lib = load()
        self._ptr = ctypes.c_void_p()
        self.device = device
        self._check(self._lib.wmh_create(device, ctypes.byref(self._ptr)), "wmh_create")

    def close(self):
        if self._ptr:
            self._lib.wmh_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, status: int, what: str):
        if status != 0:
            detail = ""
            if self._ptr:
                detail = self._lib.wmh_last_error(self._ptr).decode()
            raise WMHError(status, f"{what}: {detail}")

    def last_error(self) -> str:
        return self._lib.wmh_last_error(self._ptr).decode()

    def _stream(self, stream):
        if stream is not None:
            return ctypes.c_void_p(int(stream))
        torch = _torch()
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    # -- calls --------------------------------------------------------------------------------
    def set_bounds(self, m: np.ndarray):
        m = np.ascontiguousarray(m, dtype=np.uint32)
        self._check(self._lib.wmh_set_bounds(self._ptr, m.ctypes.data, len(m)), "wmh_set_bounds")

    def bounds_info(self) -> dict:
        D, M, shift, nb = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_uint64()
        self._check(self._lib.wmh_bounds_info(self._ptr, ctypes.byref(D), ctypes.byref(M),
                                              ctypes.byref(shift), ctypes.byref(nb)),
                    "wmh_bounds_info")
        return {"D": D.value, "M": M.value, "shift": shift.value, "n_buckets": nb.value}

    @staticmethod
    def make_opts(mode="auto", batch_rows=0, validate=True, use_graph=True, sync=True,
                  rows_per_block=0, hashes_per_tile=0, stream_depth=0, waves_per_block=0,
                  profile=False, walk=0, steps_per_lane=0, index_batch=0,
                  index_claim=0, hash_groups=0, values=0, coarse_bits=0) -> WmhOpts:
        o = WmhOpts()
        load().wmh_opts_init(ctypes.byref(o))
        o.mode = MODES[mode] if isinstance(mode, str) else int(mode)
        if batch_rows:
            o.batch_rows = batch_rows
        o.validate = int(bool(validate))
        o.use_graph = int(bool(use_graph))
        o.sync = int(bool(sync))
        o.rows_per_block = rows_per_block
        o.hashes_per_tile = hashes_per_tile
        o.stream_depth = 0xFFFFFFFF if stream_depth is None else stream_depth
        o.waves_per_block = waves_per_block
        o.profile = int(bool(profile))
        o.walk = WALKS[walk] if isinstance(walk, str) else int(walk)
        o.steps_per_lane = steps_per_lane
        o.index_batch = index_batch
        o.index_claim = {"counter": 1, "stride": 2}.get(index_claim, index_claim)
        o.hash_groups = hash_groups
        o.values = VALUES[values] if isinstance(values, str) else int(values)
        o.coarse_bits = coarse_bits
        return o

    def last_kernel_ms(self) -> tuple[float, float]:
        """(walk_ms, stream_ms) of the last profiled wmh_hash call."""
        w, st = ctypes.c_float(), ctypes.c_float()
        self._check(self._lib.wmh_last_kernel_ms(self._ptr, ctypes.byref(w), ctypes.byref(st)),
                    "wmh_last_kernel_ms")
        return w.value, st.value

    def last_mode(self) -> str:
        """Name of the path ("plain", "batched", "indexed", "split") the last wmh_hash call
        took."""
        m = ctypes.c_int32()
        self._check(self._lib.wmh_last_mode(self._ptr, ctypes.byref(m)), "wmh_last_mode")
        return {v: k for k, v in MODES.items()}[m.value]

    def last_plan(self) -> dict:
        """Mode and batched tile plan of the last wmh_hash call."""
        o = WmhOpts()
        self._check(self._lib.wmh_last_plan(self._ptr, ctypes.byref(o)), "wmh_last_plan")
        return {"mode": {v: k for k, v in MODES.items()}[o.mode],
                "rows_per_block": o.rows_per_block, "hashes_per_tile": o.hashes_per_tile,
                "stream_depth": o.stream_depth, "waves_per_block": o.waves_per_block,
                "walk": {v: k for k, v in WALKS.items()}.get(o.walk, o.walk),
                "steps_per_lane": o.steps_per_lane, "index_batch": o.index_batch,
                "index_claim": o.index_claim, "hash_groups": o.hash_groups,
                "values": {1: "exact", 2: "coarse"}.get(o.values),
                "coarse_bits": o.coarse_bits}

    def tune(self, rows: DeviceRows, k: int, seed: int = 0, reps: int = 3, stream=None) -> dict:
        """Autotunes the batched tile plan on these rows (see wmh_tune); returns the result and
        leaves the signatures of the last candidate in a scratch tensor."""
        torch = _torch()
        sig = torch.empty((rows.n_rows, k), dtype=torch.int16, device=rows.row_ptr.device)
        r = TuneResult()
        st = self._lib.wmh_tune(self._ptr, rows.row_ptr.data_ptr(), rows.col.data_ptr(),
                                rows.val.data_ptr(), rows.n_rows, rows.nnz, k, seed,
                                sig.data_ptr(), self._stream(stream), reps, ctypes.byref(r))
        self._check(st, "wmh_tune")
        return {"rows_per_block": r.rows_per_block, "hashes_per_tile": r.hashes_per_tile,
                "waves_per_block": r.waves_per_block, "stream_depth": r.stream_depth,
                "best_ms": r.best_ms, "default_ms": r.default_ms, "candidates": r.candidates,
                "steps_class": r.steps_class,
                "walk": {v: k for k, v in WALKS.items()}.get(r.walk, r.walk),
                "steps_per_lane": r.steps_per_lane, "index_batch": r.index_batch,
                "index_claim": r.index_claim, "hash_groups": r.hash_groups,
                "values": {1: "exact", 2: "coarse"}.get(r.values)}

    def tune_save(self, path: str):
        self._check(self._lib.wmh_tune_save(self._ptr, os.fsencode(path)), "wmh_tune_save")

    def tune_load(self, path: str):
        self._check(self._lib.wmh_tune_load(self._ptr, os.fsencode(path)), "wmh_tune_load")

    def hash_into(self, rows: DeviceRows, k: int, seed: int, sig, stream=None, opts=None):
        """Raw call: sig is a device int16 tensor of N*k elements."""
        if opts is None:
            opts = self.make_opts()
        st = self._lib.wmh_hash(self._ptr, rows.row_ptr.data_ptr(), rows.col.data_ptr(),
                                rows.val.data_ptr(), rows.n_rows, rows.nnz, k,
                                ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), sig.data_ptr(),
                                self._stream(stream), ctypes.byref(opts))
        self._check(st, "wmh_hash")
        return sig

    def hash_noalloc_into(self, rows: DeviceRows, k: int, seed: int, sig, stream=None,
                          opts=None):
        """wmh_hash_noalloc (the batched walk with its scratch in the library's static device
        array; allocates nothing): sig is a device int16 tensor of N*k elements."""
        if opts is None:
            opts = self.make_opts(mode="batched")
        st = self._lib.wmh_hash_noalloc(self._ptr, rows.row_ptr.data_ptr(), rows.col.data_ptr(),
                                        rows.val.data_ptr(), rows.n_rows, rows.nnz, k,
                                        ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF),
                                        sig.data_ptr(), self._stream(stream), ctypes.byref(opts))
        self._check(st, "wmh_hash_noalloc")
        return sig

    def hash(self, rows: DeviceRows, k: int, seed: int = 0, stream=None, **opt_kwargs):
        """Signatures [N, k] as a device int16 tensor (reinterpret as uint16)."""
        torch = _torch()
        sig = torch.empty((rows.n_rows, k), dtype=torch.int16,
                          device=rows.row_ptr.device)
        return self.hash_into(rows, k, seed, sig, stream, self.make_opts(**opt_kwargs))

    def draws(self, seed: int, j0: int, n_hashes: int, depth: int, device="cuda", stream=None):
        """(pos uint64, comp uint32, off uint64) as numpy arrays [n_hashes, depth]."""
        torch = _torch()
        pos = torch.empty((n_hashes, depth), dtype=torch.int64, device=device)
        comp = torch.empty((n_hashes, depth), dtype=torch.int32, device=device)
        off = torch.empty((n_hashes, depth), dtype=torch.int64, device=device)
        self._check(self._lib.wmh_draws(self._ptr, ctypes.c_uint64(seed), j0, n_hashes, depth,
                                        pos.data_ptr(), comp.data_ptr(), off.data_ptr(),
                                        self._stream(stream)), "wmh_draws")
        return (pos.cpu().numpy().view(np.uint64), comp.cpu().numpy().view(np.uint32),
                off.cpu().numpy().view(np.uint64))

    def estimate(self, A, B, stream=None):
        """Row-aligned pairs: (count uint32 [n], jhat float64 [n]) as device tensors."""
        torch = _torch()
        n, k = A.shape
        count = torch.empty(n, dtype=torch.int32, device=A.device)
        jhat = torch.empty(n, dtype=torch.float64, device=A.device)
        self._check(self._lib.wmh_estimate(self._ptr, A.data_ptr(), B.data_ptr(), n, k,
                                           count.data_ptr(), jhat.data_ptr(),
                                           self._stream(stream)), "wmh_estimate")
        return count, jhat

    def quantize(self, x, col, alpha: float, stream=None):
        """(uint32 values as an int32 tensor, number clipped) from device float32 x."""
        torch = _torch()
        out = torch.empty(x.shape[0], dtype=torch.int32, device=x.device)
        clipped = ctypes.c_uint64()
        self._check(self._lib.wmh_quantize(self._ptr, x.data_ptr(), col.data_ptr(), x.shape[0],
                                           alpha, out.data_ptr(), ctypes.byref(clipped),
                                           self._stream(stream)), "wmh_quantize")
        return out, clipped.value

    def lsh_index(self, sig, K: int, L: int, stream=None) -> "LshIndex":
        """(K, L) banding index over device signatures [N, k] (see wmh_lsh_build)."""
        n, k = sig.shape
        ptr = ctypes.c_void_p()
        self._check(self._lib.wmh_lsh_build(self._ptr, sig.data_ptr(), n, k, K, L,
                                            self._stream(stream), ctypes.byref(ptr)),
                    "wmh_lsh_build")
        return LshIndex(self, ptr, k)

    # -- b-bit signatures ------------------------------------------------------------------

    def sig_bits(self, sig, stream=None) -> tuple[int, int]:
        """(smallest lossless width, largest value) of device signatures [N, k]."""
        n, k = sig.shape
        b, m = ctypes.c_uint32(), ctypes.c_uint32()
        self._check(self._lib.wmh_sig_bits(self._ptr, sig.data_ptr(), n, k, ctypes.byref(b),
                                           ctypes.byref(m), self._stream(stream)), "wmh_sig_bits")
        return b.value, m.value

    def pack(self, sig, bits: int, stream=None):
        """(packed int32 tensor [N, W], number of saturated values)."""
        torch = _torch()
        n, k = sig.shape
        words = self._lib.wmh_pack_words(k, bits)
        packed = torch.empty((n, max(words, 1)), dtype=torch.int32, device=sig.device)
        sat = ctypes.c_uint64()
        self._check(self._lib.wmh_pack(self._ptr, sig.data_ptr(), n, k, bits, packed.data_ptr(),
                                       ctypes.byref(sat), self._stream(stream)), "wmh_pack")
        return packed, sat.value

    def unpack(self, packed, k: int, bits: int, stream=None):
        torch = _torch()
        n = packed.shape[0]
        sig = torch.empty((n, k), dtype=torch.int16, device=packed.device)
        self._check(self._lib.wmh_unpack(self._ptr, packed.data_ptr(), n, k, bits, sig.data_ptr(),
                                         self._stream(stream)), "wmh_unpack")
        return sig

    def packed_collisions(self, A, B, k: int, bits: int, stream=None):
        torch = _torch()
        na, nb = A.shape[0], B.shape[0]
        counts = torch.empty((na, nb), dtype=torch.int32, device=A.device)
        self._check(self._lib.wmh_packed_collisions(self._ptr, A.data_ptr(), na, B.data_ptr(), nb,
                                                    k, bits, counts.data_ptr(),
                                                    self._stream(stream)), "wmh_packed_collisions")
        return counts

    def packed_estimate(self, A, B, k: int, bits: int, stream=None):
        torch = _torch()
        n = A.shape[0]
        count = torch.empty(n, dtype=torch.int32, device=A.device)
        jhat = torch.empty(n, dtype=torch.float64, device=A.device)
        self._check(self._lib.wmh_packed_estimate(self._ptr, A.data_ptr(), B.data_ptr(), n, k,
                                                  bits, count.data_ptr(), jhat.data_ptr(),
                                                  self._stream(stream)), "wmh_packed_estimate")
        return count, jhat

    def collisions(self, A, B, stream=None):
        """All pairs: counts [NA, NB] (uint32 in an int32 tensor)."""
        torch = _torch()
        na, k = A.shape
        nb = B.shape[0]
        counts = torch.empty((na, nb), dtype=torch.int32, device=A.device)
        self._check(self._lib.wmh_collisions(self._ptr, A.data_ptr(), na, B.data_ptr(), nb, k,
                                             counts.data_ptr(), self._stream(stream)),
                    "wmh_collisions")
        return counts
