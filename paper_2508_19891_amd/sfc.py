"""ctypes binding of libsfc (the C ABI in include/sfc.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libsfc.  Device buffers are torch CUDA tensors (torch supplies
memory and streams); every function raises if the library is not built or if
a call returns an error status.  There is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsfc.so")

SFC_OK = 0
SFC_ERR_INVALID = -1
SFC_ERR_DOMAIN = -2
SFC_ERR_NOMEM = -3
SFC_ERR_CAPACITY = -4
SFC_ERR_DEVICE = -5
SFC_ERR_UNSUPPORTED = -6
SFC_ERR_SCRATCH = -7   # more than sfc_query_batch_static's fixed scratch

MORTON = 0
HILBERT = 1
MORTON3 = 2   # points in [0,1)^3, d = 3 Morton keys
BINARY = 0
LEARNED = 1
STREE = 2   # static search tree over the keys
L2 = 0      # closed Euclidean ball of radius delta
LINF = 1    # closed axis-parallel square window of half side delta

EXPORTS = [
    "sfc_default_options", "sfc_status_string", "sfc_build", "sfc_query_batch", "sfc_size",
    "sfc_index_view", "sfc_index_copy", "sfc_keys", "sfc_query_ranges",
    "sfc_last_query_stats", "sfc_free", "sfc_profile_enable", "sfc_profile_reset",
    "sfc_profile_only",
    "sfc_profile_read", "sfc_pool_trim", "sfc_set_search", "sfc_learned_fit",
    "sfc_learned_info_get", "sfc_learned_params", "sfc_learned_grad",
    "sfc_learned_shrink_windows", "sfc_build_sets", "sfc_query_sets", "sfc_graph_build",
    "sfc_graph_query", "sfc_graph_launch", "sfc_graph_wait", "sfc_graph_free",
    "sfc_autotune_build", "sfc_autotune_query", "sfc_tune_pin", "sfc_debug_chunk_tiles",
    "sfc_insert", "sfc_erase", "sfc_query_epochs", "sfc_hold_epochs", "sfc_retire",
    "sfc_compact", "sfc_update_info_get", "sfc_learned_route", "sfc_query_retry",
    "sfc_query_async", "sfc_occupancy_copy", "sfc_set_metric", "sfc_set_cell_filter",
    "sfc_cells_copy", "sfc_debug_sort_path", "sfc_insert_runs", "sfc_query_batch_static",
    "sfc_query_scratch_size", "sfc_query_async_on",
]

NPARAM = 1153


class SfcError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


class DomainError(SfcError):
    pass


class CapacityError(SfcError):
    def __init__(self, status, what, total):
        super().__init__(status, what)
        self.total = total


class Options(ctypes.Structure):
    _fields_ = [
        ("curve", ctypes.c_int),
        ("search", ctypes.c_int),
        ("refine", ctypes.c_int),
        ("learn_steps", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("alloc", ctypes.c_void_p),
        ("release", ctypes.c_void_p),
        ("alloc_ctx", ctypes.c_void_p),
        ("early_term", ctypes.c_int),
        ("metric", ctypes.c_int),
    ]


# sfc_options.alloc / release: device memory hooks (alloc returns NULL on failure).
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class LearnedInfo(ctypes.Structure):
    _fields_ = [("fitted", ctypes.c_int), ("steps", ctypes.c_uint32),
                ("loss_init", ctypes.c_float), ("loss_final", ctypes.c_float),
                ("leaves", ctypes.c_uint32), ("leaves_nonempty", ctypes.c_uint32),
                ("max_leaf", ctypes.c_uint32), ("mean_window", ctypes.c_double),
                ("max_window", ctypes.c_uint32), ("endpoints_last", ctypes.c_uint64),
                ("fallbacks_last", ctypes.c_uint64), ("pieces", ctypes.c_uint32),
                ("search_steps", ctypes.c_double)]


class QueryStats(ctypes.Structure):
    _fields_ = [("queries", ctypes.c_uint64), ("rows", ctypes.c_uint64),
                ("candidates", ctypes.c_uint64), ("reported", ctypes.c_uint64),
                ("pruned", ctypes.c_uint64)]


class UpdateInfo(ctypes.Structure):
    _fields_ = [("epoch", ctypes.c_uint32), ("oldest", ctypes.c_uint32),
                ("next_id", ctypes.c_uint32), ("hold", ctypes.c_uint32),
                ("stored", ctypes.c_uint64), ("live", ctypes.c_uint64),
                ("dead", ctypes.c_uint64), ("droppable", ctypes.c_uint64),
                ("merges", ctypes.c_uint64), ("compactions", ctypes.c_uint64)]


_lib = None


def lib() -> ctypes.CDLL:
    """Opens libsfc.so (built by build_lib.py); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2508_19891_amd.build_lib")
    L = ctypes.CDLL(LIB_PATH)
    vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    L.sfc_default_options.argtypes = [ctypes.POINTER(Options)]
    L.sfc_default_options.restype = None
    L.sfc_status_string.argtypes = [i32]
    L.sfc_status_string.restype = ctypes.c_char_p
    L.sfc_build.argtypes = [vp, u64, ctypes.POINTER(Options), ctypes.POINTER(vp)]
    L.sfc_build.restype = i32
    L.sfc_query_batch.argtypes = [vp, vp, vp, u64, vp, vp, u64, ctypes.POINTER(u64)]
    L.sfc_query_batch.restype = i32
    L.sfc_query_batch_static.argtypes = [vp, vp, vp, u64, vp, vp, u64, ctypes.POINTER(u64)]
    L.sfc_query_batch_static.restype = i32
    L.sfc_size.argtypes = [vp]
    L.sfc_size.restype = u64
    L.sfc_index_view.argtypes = [vp, vp, vp, vp, ctypes.POINTER(u64)]
    L.sfc_index_view.restype = i32
    L.sfc_index_copy.argtypes = [vp, vp, vp, vp]
    L.sfc_index_copy.restype = i32
    L.sfc_keys.argtypes = [vp, u64, i32, vp, vp]
    L.sfc_keys.restype = i32
    L.sfc_query_ranges.argtypes = [vp, vp, vp, u64, vp, vp, vp, vp, vp]
    L.sfc_query_ranges.restype = i32
    L.sfc_last_query_stats.argtypes = [vp, ctypes.POINTER(QueryStats)]
    L.sfc_last_query_stats.restype = i32
    L.sfc_free.argtypes = [vp]
    L.sfc_free.restype = None
    L.sfc_profile_enable.argtypes = [i32]
    L.sfc_profile_enable.restype = None
    L.sfc_profile_only.argtypes = [ctypes.c_char_p]
    L.sfc_profile_only.restype = None
    L.sfc_profile_reset.argtypes = []
    L.sfc_profile_reset.restype = None
    L.sfc_profile_read.argtypes = [vp, vp, vp, i32]
    L.sfc_profile_read.restype = i32
    L.sfc_pool_trim.argtypes = []
    L.sfc_pool_trim.restype = None
    L.sfc_set_search.argtypes = [vp, i32]
    L.sfc_set_search.restype = i32
    L.sfc_set_metric.argtypes = [vp, i32]
    L.sfc_set_metric.restype = i32
    L.sfc_set_cell_filter.argtypes = [vp, i32]
    L.sfc_set_cell_filter.restype = i32
    L.sfc_cells_copy.argtypes = [vp, vp, u64]
    L.sfc_cells_copy.restype = i32
    L.sfc_learned_fit.argtypes = [vp, i32]
    L.sfc_learned_fit.restype = i32
    L.sfc_learned_info_get.argtypes = [vp, ctypes.POINTER(LearnedInfo)]
    L.sfc_learned_info_get.restype = i32
    L.sfc_learned_params.argtypes = [vp, vp]
    L.sfc_learned_params.restype = i32
    L.sfc_learned_grad.argtypes = [vp, vp, vp, u32, vp, vp]
    L.sfc_learned_grad.restype = i32
    L.sfc_learned_shrink_windows.argtypes = [vp]
    L.sfc_learned_shrink_windows.restype = i32
    L.sfc_build_sets.argtypes = [vp, vp, u32, ctypes.POINTER(Options), ctypes.POINTER(vp)]
    L.sfc_build_sets.restype = i32
    L.sfc_query_sets.argtypes = [vp, vp, vp, vp, u64, vp, vp, u64, ctypes.POINTER(u64)]
    L.sfc_query_sets.restype = i32
    L.sfc_graph_build.argtypes = [vp, vp, ctypes.POINTER(vp)]
    L.sfc_graph_build.restype = i32
    L.sfc_graph_query.argtypes = [vp, vp, vp, vp, u64, u64, vp, vp, u64, ctypes.POINTER(vp)]
    L.sfc_graph_query.restype = i32
    L.sfc_graph_launch.argtypes = [vp]
    L.sfc_graph_launch.restype = i32
    L.sfc_graph_wait.argtypes = [vp, ctypes.POINTER(u64)]
    L.sfc_graph_wait.restype = i32
    L.sfc_graph_free.argtypes = [vp]
    L.sfc_graph_free.restype = None
    L.sfc_autotune_build.argtypes = [vp, u64, vp, u32, ctypes.POINTER(Options),
                                     ctypes.POINTER(i32), vp]
    L.sfc_autotune_build.restype = i32
    L.sfc_autotune_query.argtypes = [vp, vp, vp, vp, u64, vp, vp, u64, ctypes.POINTER(i32), vp]
    L.sfc_autotune_query.restype = i32
    L.sfc_tune_pin.argtypes = [i32, u64, i32]
    L.sfc_tune_pin.restype = i32
    L.sfc_debug_sort_path.argtypes = [i32, ctypes.POINTER(i32)]
    L.sfc_debug_sort_path.restype = i32
    L.sfc_debug_chunk_tiles.argtypes = [u64]
    L.sfc_debug_chunk_tiles.restype = i32
    L.sfc_insert.argtypes = [vp, vp, u64, vp]
    L.sfc_insert.restype = i32
    L.sfc_insert_runs.argtypes = [vp, vp, ctypes.POINTER(u64), u32, vp]
    L.sfc_insert_runs.restype = i32
    L.sfc_erase.argtypes = [vp, vp, u64, ctypes.POINTER(u64)]
    L.sfc_erase.restype = i32
    L.sfc_query_epochs.argtypes = [vp, vp, vp, vp, u64, vp, vp, u64, ctypes.POINTER(u64)]
    L.sfc_query_epochs.restype = i32
    L.sfc_hold_epochs.argtypes = [vp, i32]
    L.sfc_hold_epochs.restype = i32
    L.sfc_retire.argtypes = [vp, u32]
    L.sfc_retire.restype = i32
    L.sfc_compact.argtypes = [vp]
    L.sfc_compact.restype = i32
    L.sfc_update_info_get.argtypes = [vp, ctypes.POINTER(UpdateInfo)]
    L.sfc_update_info_get.restype = i32
    L.sfc_learned_route.argtypes = [vp, vp, u64, vp, vp]
    L.sfc_learned_route.restype = i32
    L.sfc_query_retry.argtypes = [vp, vp, vp, u64, ctypes.POINTER(u64)]
    L.sfc_query_retry.restype = i32
    L.sfc_query_async.argtypes = [vp, vp, vp, vp, u64, u64, vp, vp, u64, vp]
    L.sfc_query_async.restype = i32
    L.sfc_query_scratch_size.argtypes = [vp, u64, u64, ctypes.POINTER(u64)]
    L.sfc_query_scratch_size.restype = i32
    L.sfc_query_async_on.argtypes = [vp, vp, vp, u64, vp, vp, vp, u64, u64, vp, vp, u64, vp]
    L.sfc_query_async_on.restype = i32
    L.sfc_occupancy_copy.argtypes = [vp, vp, u64]
    L.sfc_occupancy_copy.restype = i32
    _lib = L
    return L


def status_string(status: int) -> str:
    return lib().sfc_status_string(status).decode()


def _check(status: int, what: str):
    if status == SFC_OK:
        return
    if status == SFC_ERR_DOMAIN:
        raise DomainError(status, what)
    raise SfcError(status, what)


def _dev(t: torch.Tensor, dtype: torch.dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ptr(t: torch.Tensor | None):
    return None if t is None or t.numel() == 0 else ctypes.c_void_p(t.data_ptr())


def current_stream_handle() -> int:
    return torch.cuda.current_stream().cuda_stream


# ---- the entry points, one per C function ------------------------------------------


def sfc_keys(xy: torch.Tensor, curve: int = MORTON) -> torch.Tensor:
    """Curve keys of the points (n, 2) float64, or (n, 3) for MORTON3 ->
    (n,) uint64 (as int64 bits)."""
    xy = _dev(xy, torch.float64, "xy")
    n = xy.shape[0]
    keys = torch.empty(n, dtype=torch.int64, device=xy.device)
    _check(lib().sfc_keys(_ptr(xy), n, curve, ctypes.c_void_p(current_stream_handle()),
                          _ptr(keys)), "sfc_keys")
    return keys


class Index:
    """An index built by sfc_build; freed by close() or on garbage collection."""

    def __init__(self, xy: torch.Tensor, curve: int = MORTON, search: int = BINARY,
                 refine: bool = False, learn_steps: int = -1, set_off=None,
                 early_term: bool = False, metric: int = L2, allocator=None):
        """set_off (host sequence of n_sets + 1 offsets): build independent
        point sets with sfc_build_sets; query them with query_sets.  metric:
        L2 (ball of radius delta) or LINF (square window of half side
        delta).  allocator: an object with alloc(nbytes) -> device address
        (0 on failure) and release(address), used for every device
        allocation of the index (sfc_options.alloc / release)."""
        xy = _dev(xy, torch.float64, "xy")
        self.dim = 3 if curve == MORTON3 else 2
        if xy.ndim != 2 or xy.shape[1] != self.dim:
            raise ValueError(f"xy must have shape (n, {self.dim})")
        L = lib()
        opt = Options()
        L.sfc_default_options(ctypes.byref(opt))
        opt.curve = curve
        opt.search = search
        opt.refine = 1 if refine else 0
        opt.learn_steps = learn_steps
        opt.early_term = 1 if early_term else 0
        opt.metric = metric
        opt.stream = current_stream_handle()
        self._hooks = None
        if allocator is not None:
            self._hooks = (ALLOC_FN(lambda nbytes, ctx: allocator.alloc(nbytes) or None),
                           RELEASE_FN(lambda ptr, ctx: allocator.release(ptr)))
            opt.alloc = ctypes.cast(self._hooks[0], ctypes.c_void_p)
            opt.release = ctypes.cast(self._hooks[1], ctypes.c_void_p)
        h = ctypes.c_void_p()
        if set_off is None:
            _check(L.sfc_build(_ptr(xy), xy.shape[0], ctypes.byref(opt), ctypes.byref(h)),
                   "sfc_build")
            self.n_sets = 0
        else:
            import numpy as np
            so = np.ascontiguousarray(set_off, np.uint64)
            if int(so[-1]) != xy.shape[0]:
                raise ValueError("set_off[-1] must equal the number of points")
            _check(L.sfc_build_sets(_ptr(xy), so.ctypes.data_as(ctypes.c_void_p), len(so) - 1,
                                    ctypes.byref(opt), ctypes.byref(h)), "sfc_build_sets")
            self.n_sets = len(so) - 1
        self._h = h
        self.curve = curve
        self.search = search
        self.metric = metric
        self.device = xy.device

    def close(self):
        if getattr(self, "_h", None):
            lib().sfc_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("index is closed")
        return self._h

    def size(self) -> int:
        return int(lib().sfc_size(self.handle))

    def sorted_arrays(self):
        """Copies of the sorted (keys int64-bits, ids int32-bits, xy (n,2))."""
        n = self.size()
        keys = torch.empty(n, dtype=torch.int64, device=self.device)
        ids = torch.empty(n, dtype=torch.int32, device=self.device)
        xy = torch.empty((n, self.dim), dtype=torch.float64, device=self.device)
        _check(lib().sfc_index_copy(self.handle, _ptr(keys), _ptr(ids), _ptr(xy)),
               "sfc_index_copy")
        return keys, ids, xy

    def query(self, q: torch.Tensor, delta: torch.Tensor, ids_cap: int | None = None,
              out_ids: torch.Tensor | None = None, out_offsets: torch.Tensor | None = None):
        """Batched queries; returns (offsets int64[m+1], ids int32[total]).

        Without ids_cap/out_ids a first guess of the output size that is too
        small is followed by the library's write-only retry into a buffer of
        the exact size."""
        q = _dev(q, torch.float64, "q")
        delta = _dev(delta, torch.float64, "delta")
        m = q.shape[0]
        if q.ndim != 2 or q.shape[1] != self.dim or delta.shape != (m,):
            raise ValueError(f"q must be (m, {self.dim}) and delta (m,)")
        offsets = out_offsets if out_offsets is not None else torch.empty(
            m + 1, dtype=torch.int64, device=self.device)
        auto = ids_cap is None and out_ids is None   # may retry with the exact size
        if out_ids is None:
            cap = ids_cap if ids_cap is not None else max(16 * m, 1024)
            out_ids = torch.empty(cap, dtype=torch.int32, device=self.device)
        total = ctypes.c_uint64(0)
        st = lib().sfc_query_batch(self.handle, _ptr(q), _ptr(delta), m, _ptr(offsets),
                                   _ptr(out_ids), out_ids.numel(), ctypes.byref(total))
        if st == SFC_ERR_CAPACITY and auto:
            out_ids, st = self._retry(offsets, total, lambda o, t: lib().sfc_query_batch(
                self.handle, _ptr(q), _ptr(delta), m, _ptr(offsets), _ptr(o), o.numel(),
                ctypes.byref(t)))
        if st == SFC_ERR_CAPACITY:
            raise CapacityError(st, "sfc_query_batch", int(total.value))
        _check(st, "sfc_query_batch")
        return offsets, out_ids[: int(total.value)]

    def query_static(self, q: torch.Tensor, delta: torch.Tensor, out_ids: torch.Tensor,
                     out_offsets: torch.Tensor):
        """sfc_query_batch_static into caller buffers (the library's fixed
        scratch, no allocation); returns (offsets, ids[:total])."""
        q = _dev(q, torch.float64, "q")
        delta = _dev(delta, torch.float64, "delta")
        m = q.shape[0]
        if q.ndim != 2 or q.shape[1] != self.dim or delta.shape != (m,):
            raise ValueError(f"q must be (m, {self.dim}) and delta (m,)")
        if out_offsets.numel() < m + 1:
            raise ValueError("out_offsets must hold m + 1 entries")
        total = ctypes.c_uint64(0)
        st = lib().sfc_query_batch_static(self.handle, _ptr(q), _ptr(delta), m,
                                          _ptr(out_offsets), _ptr(out_ids), out_ids.numel(),
                                          ctypes.byref(total))
        if st == SFC_ERR_CAPACITY:
            raise CapacityError(st, "sfc_query_batch_static", int(total.value))
        _check(st, "sfc_query_batch_static")
        return out_offsets[: m + 1], out_ids[: int(total.value)]

    def _retry(self, offsets, total, rerun):
        """After SFC_ERR_CAPACITY: an ids buffer of the exact size, filled by
        the kept batch's write pass (sfc_query_retry), or by rerunning the
        batch when the library kept none.  Returns (ids buffer, status)."""
        out_ids = torch.empty(max(int(total.value), 1), dtype=torch.int32, device=self.device)
        st = lib().sfc_query_retry(self.handle, _ptr(offsets), _ptr(out_ids), out_ids.numel(),
                                   ctypes.byref(total))
        if st == SFC_ERR_UNSUPPORTED:
            st = rerun(out_ids, total)
        return out_ids, st

    def query_retry(self, offsets: torch.Tensor, out_ids: torch.Tensor) -> int:
        """sfc_query_retry into caller buffers; returns the total."""
        total = ctypes.c_uint64(0)
        st = lib().sfc_query_retry(self.handle, _ptr(offsets), _ptr(out_ids), out_ids.numel(),
                                   ctypes.byref(total))
        if st == SFC_ERR_CAPACITY:
            raise CapacityError(st, "sfc_query_retry", int(total.value))
        _check(st, "sfc_query_retry")
        return int(total.value)

    def query_sets(self, q: torch.Tensor, delta: torch.Tensor, qset: torch.Tensor,
                   out_ids: torch.Tensor | None = None, out_offsets: torch.Tensor | None = None):
        """Queries of an index of point sets; qset (m,) int32 holds each
        query's set.  Returns (offsets int64[m+1], ids int32[total])."""
        q = _dev(q, torch.float64, "q")
        delta = _dev(delta, torch.float64, "delta")
        qset = _dev(qset, torch.int32, "qset")
        m = q.shape[0]
        offsets = out_offsets if out_offsets is not None else torch.empty(
            m + 1, dtype=torch.int64, device=self.device)
        cap_given = out_ids is not None
        if out_ids is None:
            out_ids = torch.empty(max(16 * m, 1024), dtype=torch.int32, device=self.device)
        total = ctypes.c_uint64(0)
        args = (self.handle, _ptr(q), _ptr(delta), _ptr(qset), m, _ptr(offsets))
        st = lib().sfc_query_sets(*args, _ptr(out_ids), out_ids.numel(), ctypes.byref(total))
        if st == SFC_ERR_CAPACITY and not cap_given:
            out_ids, st = self._retry(offsets, total, lambda o, t: lib().sfc_query_sets(
                *args, _ptr(o), o.numel(), ctypes.byref(t)))
        if st == SFC_ERR_CAPACITY:
            raise CapacityError(st, "sfc_query_sets", int(total.value))
        _check(st, "sfc_query_sets")
        return offsets, out_ids[: int(total.value)]

    def query_epochs(self, q: torch.Tensor, delta: torch.Tensor, qepoch: torch.Tensor,
                     out_ids: torch.Tensor | None = None,
                     out_offsets: torch.Tensor | None = None):
        """Queries answered at per-query epochs qepoch (m,) int32 (uint32
        values).  Returns (offsets int64[m+1], ids int32[total])."""
        q = _dev(q, torch.float64, "q")
        delta = _dev(delta, torch.float64, "delta")
        qepoch = _dev(qepoch, torch.int32, "qepoch")
        m = q.shape[0]
        offsets = out_offsets if out_offsets is not None else torch.empty(
            m + 1, dtype=torch.int64, device=self.device)
        cap_given = out_ids is not None
        if out_ids is None:
            out_ids = torch.empty(max(16 * m, 1024), dtype=torch.int32, device=self.device)
        total = ctypes.c_uint64(0)
        args = (self.handle, _ptr(q), _ptr(delta), _ptr(qepoch), m, _ptr(offsets))
        st = lib().sfc_query_epochs(*args, _ptr(out_ids), out_ids.numel(), ctypes.byref(total))
        if st == SFC_ERR_CAPACITY and not cap_given:
            out_ids, st = self._retry(offsets, total, lambda o, t: lib().sfc_query_epochs(
                *args, _ptr(o), o.numel(), ctypes.byref(t)))
        if st == SFC_ERR_CAPACITY:
            raise CapacityError(st, "sfc_query_epochs", int(total.value))
        _check(st, "sfc_query_epochs")
        return offsets, out_ids[: int(total.value)]

    def query_async(self, q: torch.Tensor, delta: torch.Tensor, qepoch: torch.Tensor | None,
                    max_rows: int, out_offsets: torch.Tensor, out_ids: torch.Tensor,
                    flags: torch.Tensor):
        """Queues a batch (sfc_query_async) and returns at once; the caller
        keeps the tensors alive until the stream has passed the batch, then
        reads flags[0] and out_offsets[-1]."""
        q = _dev(q, torch.float64, "q")
        delta = _dev(delta, torch.float64, "delta")
        if qepoch is not None:
            qepoch = _dev(qepoch, torch.int32, "qepoch")
        _check(lib().sfc_query_async(self.handle, _ptr(q), _ptr(delta), _ptr(qepoch), q.shape[0],
                                     max_rows, _ptr(out_offsets), _ptr(out_ids), out_ids.numel(),
                                     _ptr(flags)), "sfc_query_async")

    def query_scratch_bytes(self, m: int, max_rows: int) -> int:
        """Scratch bytes of one sfc_query_async_on batch."""
        b = ctypes.c_uint64(0)
        _check(lib().sfc_query_scratch_size(self.handle, m, max_rows, ctypes.byref(b)),
               "sfc_query_scratch_size")
        return int(b.value)

    def query_async_on(self, stream: torch.cuda.Stream, scratch: torch.Tensor, q: torch.Tensor,
                       delta: torch.Tensor, qepoch: torch.Tensor | None, max_rows: int,
                       out_offsets: torch.Tensor, out_ids: torch.Tensor, flags: torch.Tensor):
        """Queues a batch on `stream` with its own scratch (sfc_query_async_on)
        and returns at once; the caller keeps every tensor alive until the
        stream has passed the batch."""
        q = _dev(q, torch.float64, "q")
        delta = _dev(delta, torch.float64, "delta")
        if qepoch is not None:
            qepoch = _dev(qepoch, torch.int32, "qepoch")
        _check(lib().sfc_query_async_on(self.handle, ctypes.c_void_p(stream.cuda_stream),
                                        _ptr(scratch), scratch.numel() * scratch.element_size(),
                                        _ptr(q), _ptr(delta), _ptr(qepoch), q.shape[0], max_rows,
                                        _ptr(out_offsets), _ptr(out_ids), out_ids.numel(),
                                        _ptr(flags)), "sfc_query_async_on")

    def occupancy(self) -> torch.Tensor:
        """The early-termination bitmap (int32 words)."""
        out = torch.empty(699051, dtype=torch.int32, device=self.device)
        _check(lib().sfc_occupancy_copy(self.handle, _ptr(out), out.numel()),
               "sfc_occupancy_copy")
        return out

    def insert(self, xy: torch.Tensor, want_ids: bool = True):
        """Inserts points (k, 2); returns their ids (int32 tensor) or None."""
        xy = _dev(xy, torch.float64, "xy")
        if xy.ndim != 2 or xy.shape[1] != self.dim:
            raise ValueError(f"xy must have shape (k, {self.dim})")
        k = xy.shape[0]
        ids = torch.empty(k, dtype=torch.int32, device=self.device) if want_ids else None
        _check(lib().sfc_insert(self.handle, _ptr(xy), k, _ptr(ids)), "sfc_insert")
        return ids

    def insert_runs(self, xy: torch.Tensor, run_off, want_ids: bool = True):
        """Inserts consecutive batches xy[run_off[r]:run_off[r+1]] as if by one
        insert call each, in order (one sort, one merge); returns the ids
        (int32 tensor) or None."""
        xy = _dev(xy, torch.float64, "xy")
        if xy.ndim != 2 or xy.shape[1] != self.dim:
            raise ValueError(f"xy must have shape (k, {self.dim})")
        off = [int(v) for v in run_off]
        if len(off) < 2 or off[-1] != xy.shape[0]:
            raise ValueError("run_off must end at the number of points")
        arr = (ctypes.c_uint64 * len(off))(*off)
        ids = (torch.empty(xy.shape[0], dtype=torch.int32, device=self.device)
               if want_ids else None)
        _check(lib().sfc_insert_runs(self.handle, _ptr(xy), arr, len(off) - 1, _ptr(ids)),
               "sfc_insert_runs")
        return ids

    def erase(self, ids: torch.Tensor) -> int:
        """Erases ids (k,) int32; returns the number of entries erased."""
        ids = _dev(ids, torch.int32, "ids")
        cnt = ctypes.c_uint64(0)
        _check(lib().sfc_erase(self.handle, _ptr(ids), ids.numel(), ctypes.byref(cnt)),
               "sfc_erase")
        return int(cnt.value)

    def hold_epochs(self, hold: bool = True):
        _check(lib().sfc_hold_epochs(self.handle, 1 if hold else 0), "sfc_hold_epochs")

    def retire(self, epoch: int):
        _check(lib().sfc_retire(self.handle, epoch), "sfc_retire")

    def compact(self):
        _check(lib().sfc_compact(self.handle), "sfc_compact")

    def update_info(self) -> dict:
        u = UpdateInfo()
        _check(lib().sfc_update_info_get(self.handle, ctypes.byref(u)), "sfc_update_info_get")
        return {f: int(getattr(u, f)) for f, _ in UpdateInfo._fields_}

    def query_ranges(self, q: torch.Tensor, delta: torch.Tensor):
        """Per query four slots of (key_lo, key_hi, begin, end) and the number
        of ranges; tensors of shape (m, 4) and (m,)."""
        q = _dev(q, torch.float64, "q")
        delta = _dev(delta, torch.float64, "delta")
        m = q.shape[0]
        dev = self.device
        klo = torch.zeros((m, 4), dtype=torch.int64, device=dev)
        khi = torch.zeros((m, 4), dtype=torch.int64, device=dev)
        b = torch.zeros((m, 4), dtype=torch.int64, device=dev)
        e = torch.zeros((m, 4), dtype=torch.int64, device=dev)
        nr = torch.zeros(m, dtype=torch.int32, device=dev)
        _check(lib().sfc_query_ranges(self.handle, _ptr(q), _ptr(delta), m, _ptr(klo), _ptr(khi),
                                      _ptr(b), _ptr(e), _ptr(nr)), "sfc_query_ranges")
        return klo, khi, b, e, nr

    def set_cell_filter(self, on: bool):
        """Decide candidates from their grid cell where the cell settles the
        test (default), or run the exact test on every candidate."""
        _check(lib().sfc_set_cell_filter(self.handle, 1 if on else 0), "sfc_set_cell_filter")

    def cells(self) -> torch.Tensor:
        """Grid cells of the sorted points (int64 bits of the packed words)."""
        out = torch.empty(max(self.size(), 1), dtype=torch.int64, device=self.device)
        _check(lib().sfc_cells_copy(self.handle, _ptr(out), out.numel()), "sfc_cells_copy")
        return out[:self.size()]

    def set_metric(self, metric: int):
        _check(lib().sfc_set_metric(self.handle, metric), "sfc_set_metric")
        self.metric = metric

    def set_search(self, search: int):
        _check(lib().sfc_set_search(self.handle, search), "sfc_set_search")
        self.search = search

    def learned_fit(self, steps: int = -1):
        _check(lib().sfc_learned_fit(self.handle, steps), "sfc_learned_fit")

    def learned_info(self) -> dict:
        i = LearnedInfo()
        _check(lib().sfc_learned_info_get(self.handle, ctypes.byref(i)), "sfc_learned_info_get")
        return {f: getattr(i, f) for f, _ in LearnedInfo._fields_}

    def learned_params(self):
        import numpy as np
        out = np.zeros(NPARAM, np.float32)
        _check(lib().sfc_learned_params(self.handle, out.ctypes.data_as(ctypes.c_void_p)),
               "sfc_learned_params")
        return out

    def learned_route(self, keys: torch.Tensor):
        """(direct, table) leaves of keys (int64 tensor holding uint64 bits)."""
        keys = _dev(keys, torch.int64, "keys")
        d = torch.empty(keys.numel(), dtype=torch.int32, device=self.device)
        t = torch.empty_like(d)
        _check(lib().sfc_learned_route(self.handle, _ptr(keys), keys.numel(), _ptr(d), _ptr(t)),
               "sfc_learned_route")
        return d, t

    def learned_shrink_windows(self):
        _check(lib().sfc_learned_shrink_windows(self.handle), "sfc_learned_shrink_windows")

    def last_stats(self) -> dict:
        s = QueryStats()
        _check(lib().sfc_last_query_stats(self.handle, ctypes.byref(s)), "sfc_last_query_stats")
        return {"queries": s.queries, "rows": s.rows, "candidates": s.candidates,
                "reported": s.reported, "pruned": s.pruned}


class Graph:
    """A recorded construction or query batch (sfc_graph_*).  Keeps the
    tensors it was recorded with alive; launch() enqueues a replay, wait()
    synchronises and returns the total (query graphs)."""

    def __init__(self, index: Index, handle, keep):
        self.index = index
        self._g = handle
        self._keep = keep

    @classmethod
    def build(cls, index: Index, xy: torch.Tensor) -> "Graph":
        xy = _dev(xy, torch.float64, "xy")
        g = ctypes.c_void_p()
        _check(lib().sfc_graph_build(index.handle, _ptr(xy), ctypes.byref(g)), "sfc_graph_build")
        return cls(index, g, (xy,))

    @classmethod
    def query(cls, index: Index, q: torch.Tensor, delta: torch.Tensor, max_rows: int,
              ids_cap: int, qset: torch.Tensor | None = None) -> "Graph":
        q = _dev(q, torch.float64, "q")
        delta = _dev(delta, torch.float64, "delta")
        if qset is not None:
            qset = _dev(qset, torch.int32, "qset")
        m = q.shape[0]
        offsets = torch.empty(m + 1, dtype=torch.int64, device=index.device)
        ids = torch.empty(max(ids_cap, 1), dtype=torch.int32, device=index.device)
        g = ctypes.c_void_p()
        _check(lib().sfc_graph_query(index.handle, _ptr(q), _ptr(delta), _ptr(qset), m, max_rows,
                                     _ptr(offsets), _ptr(ids), ids_cap, ctypes.byref(g)),
               "sfc_graph_query")
        obj = cls(index, g, (q, delta, qset))
        obj.offsets, obj.ids = offsets, ids
        return obj

    def launch(self):
        _check(lib().sfc_graph_launch(self._g), "sfc_graph_launch")

    def wait(self) -> int:
        total = ctypes.c_uint64(0)
        st = lib().sfc_graph_wait(self._g, ctypes.byref(total))
        if st == SFC_ERR_CAPACITY:
            raise CapacityError(st, "sfc_graph_wait", int(total.value))
        _check(st, "sfc_graph_wait")
        return int(total.value)

    def result(self):
        total = self.wait()
        return self.offsets, self.ids[:total]

    def close(self):
        if getattr(self, "_g", None):
            lib().sfc_graph_free(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def debug_chunk_tiles(tiles: int):
    """Test hook: compaction chunk size in tiles of 64 rows (0 = default)."""
    _check(lib().sfc_debug_chunk_tiles(tiles), "sfc_debug_chunk_tiles")


def debug_sort_path(force_plain: int = -1) -> int:
    """Test hook: force_plain 1 makes every build use the plain radix sort, 0
    restores the chunked sort (-1 leaves it); returns 1 if the last build fell
    back from the chunked sort to the plain one."""
    fell = ctypes.c_int(0)
    _check(lib().sfc_debug_sort_path(force_plain, ctypes.byref(fell)), "sfc_debug_sort_path")
    return fell.value


def autotune_build(xy: torch.Tensor, curve: int = MORTON, set_off=None):
    """Times the radix passes' keys-per-thread shapes on these points and
    records the fastest for their size; returns (best, {shape: ms})."""
    import numpy as np
    xy = _dev(xy, torch.float64, "xy")
    L = lib()
    opt = Options()
    L.sfc_default_options(ctypes.byref(opt))
    opt.curve = curve
    opt.stream = current_stream_handle()
    best = ctypes.c_int(0)
    ms = (ctypes.c_double * 5)()
    so = None if set_off is None else np.ascontiguousarray(set_off, np.uint64)
    _check(L.sfc_autotune_build(_ptr(xy), xy.shape[0],
                                None if so is None else so.ctypes.data_as(ctypes.c_void_p),
                                0 if so is None else len(so) - 1, ctypes.byref(opt),
                                ctypes.byref(best), ms), "sfc_autotune_build")
    return best.value, dict(zip((8, 12, 16, 20, 24), list(ms)))


TUNE_SORT_ITEMS = 0
TUNE_TEST_SHAPE = 1


def tune_pin(what: int, size: int, value: int) -> None:
    """Pins a launch shape for the size bucket of `size` (TUNE_SORT_ITEMS:
    8, 12, 16, 20 or 24 keys of a radix tile per 256; TUNE_TEST_SHAPE: 0..4);
    value -1 removes the pin."""
    _check(lib().sfc_tune_pin(what, size, value), "sfc_tune_pin")


def autotune_query(index: Index, q: torch.Tensor, delta: torch.Tensor,
                   qset: torch.Tensor | None = None, ids_cap: int | None = None):
    """Times the test kernel's shapes on this batch and records the fastest
    for its candidate-row bucket; returns (best, [ms per shape])."""
    q = _dev(q, torch.float64, "q")
    delta = _dev(delta, torch.float64, "delta")
    if qset is not None:
        qset = _dev(qset, torch.int32, "qset")
    m = q.shape[0]
    offsets = torch.empty(m + 1, dtype=torch.int64, device=index.device)
    if ids_cap is None:
        off, ids = (index.query(q, delta) if qset is None else index.query_sets(q, delta, qset))
        ids_cap = ids.numel() + 1
    ids = torch.empty(max(ids_cap, 1), dtype=torch.int32, device=index.device)
    best = ctypes.c_int(0)
    ms = (ctypes.c_double * 5)()
    _check(lib().sfc_autotune_query(index.handle, _ptr(q), _ptr(delta), _ptr(qset), m,
                                    _ptr(offsets), _ptr(ids), ids_cap, ctypes.byref(best), ms),
           "sfc_autotune_query")
    return best.value, list(ms)


def sfc_build(xy: torch.Tensor, curve: int = MORTON, search: int = BINARY,
              refine: bool = False) -> Index:
    return Index(xy, curve, search, refine)


def sfc_query_batch(index: Index, q: torch.Tensor, delta: torch.Tensor, **kw):
    return index.query(q, delta, **kw)


def sfc_free(index: Index):
    index.close()


def learned_grad(params, x, t):
    """(gradient float32[1153], loss) of one batch through the GPU trainer's
    backward code (host numpy arrays in and out)."""
    import numpy as np
    p = np.ascontiguousarray(params, np.float32)
    x = np.ascontiguousarray(x, np.float32)
    t = np.ascontiguousarray(t, np.float32)
    g = np.zeros(NPARAM, np.float32)
    loss = np.zeros(1, np.float32)
    vp = ctypes.c_void_p
    _check(lib().sfc_learned_grad(p.ctypes.data_as(vp), x.ctypes.data_as(vp),
                                  t.ctypes.data_as(vp), len(x), g.ctypes.data_as(vp),
                                  loss.ctypes.data_as(vp)), "sfc_learned_grad")
    return g, float(loss[0])


def profile_enable(on: bool = True):
    lib().sfc_profile_enable(1 if on else 0)


def profile_only(name: str | None):
    """Time only the launches of kernel `name` (None: every kernel)."""
    lib().sfc_profile_only(name.encode() if name else None)


def profile_reset():
    lib().sfc_profile_reset()


def profile_read() -> dict:
    """{kernel name: (launches, total ms)} of the launches since the last reset."""
    L = lib()
    k = L.sfc_profile_read(None, None, None, 0)
    names = (ctypes.c_char_p * max(k, 1))()
    launches = (ctypes.c_uint64 * max(k, 1))()
    ms = (ctypes.c_double * max(k, 1))()
    k = L.sfc_profile_read(names, launches, ms, k)
    return {names[i].decode(): (int(launches[i]), float(ms[i])) for i in range(k)}


def u64(t: torch.Tensor):
    """View of an int64 tensor holding uint64 bit patterns as numpy uint64."""
    return t.detach().cpu().numpy().view("uint64")
