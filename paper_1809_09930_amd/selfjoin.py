"""Python binding of libselfjoin (the C ABI in include/selfjoin.h).

Argument marshalling only: every step of the join runs in the HIP library.
PyTorch provides device memory and the current stream.  Importing this
module raises if the built library is missing -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libselfjoin.so")

SJ_OK = 0
SJ_ERR_INVALID_ARG = -1
SJ_ERR_OUT_OF_MEMORY = -2
SJ_ERR_DEVICE = -3
SJ_ERR_KEY_OVERFLOW = -4
SJ_ERR_STATE = -5
SJ_ERR_RANGE = -6
SJ_MAX_DIM = 128

SJ_PREC_FP32 = 0
SJ_PREC_FP16 = 1
SJ_PREC_BF16 = 2
PRECISIONS = {"fp32": SJ_PREC_FP32, "fp16": SJ_PREC_FP16, "bf16": SJ_PREC_BF16}

SJ_FP32_AUTO = 0
SJ_FP32_DIFFERENCE = 1
SJ_FP32_NORM = 2
FP32_FORMS = {"auto": SJ_FP32_AUTO, "difference": SJ_FP32_DIFFERENCE, "norm": SJ_FP32_NORM}
SJ_UNITS_CELL = 1
SJ_UNITS_SMALL_CELLS = 2

EXPORTED = ("selfjoin_default_options", "selfjoin_build_index", "selfjoin_build_query",
            "selfjoin_run",
            "selfjoin_fetch_pairs", "selfjoin_fetch_offsets", "selfjoin_fetch_offsets_noalloc",
            "selfjoin_get_info",
            "selfjoin_get_perm",
            "selfjoin_free", "selfjoin_last_error", "selfjoin_run_batched",
            "selfjoin_batch_replay", "selfjoin_batch_range", "selfjoin_batch_fetch",
            "selfjoin_batch_get_info", "selfjoin_batch_free", "selfjoin_release_cache")


class SjOptions(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32),
                ("k", ctypes.c_int32),
                ("k_min", ctypes.c_uint32),
                ("k_max", ctypes.c_uint32),
                ("reorder", ctypes.c_uint32),
                ("shortc", ctypes.c_uint32),
                ("precision", ctypes.c_uint32),
                ("batch_pairs", ctypes.c_uint64),
                ("min_batches", ctypes.c_uint32),
                ("autotune", ctypes.c_uint32),
                ("mem_budget", ctypes.c_uint64),
                ("fp32_form", ctypes.c_uint32),
                ("sortidu", ctypes.c_uint32)]


class SjInfo(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32),
                ("d", ctypes.c_uint32),
                ("n", ctypes.c_uint64),
                ("epsilon", ctypes.c_double),
                ("k", ctypes.c_uint32),
                ("precision", ctypes.c_uint32),
                ("n_cells", ctypes.c_uint64),
                ("candidates", ctypes.c_uint64),
                ("evaluated", ctypes.c_uint64),
                ("rechecks", ctypes.c_uint64),
                ("pairs", ctypes.c_uint64),
                ("batches", ctypes.c_uint32),
                ("result_on_host", ctypes.c_uint32),
                ("ms_build", ctypes.c_float),
                ("ms_join", ctypes.c_float),
                ("ms_sort", ctypes.c_float),
                ("ms_run", ctypes.c_float),
                ("join_launches", ctypes.c_uint32),
                ("fp32_form", ctypes.c_uint32),
                ("units", ctypes.c_uint32)]


class SjJob(ctypes.Structure):
    _fields_ = [("points", ctypes.c_void_p),
                ("n", ctypes.c_uint64),
                ("d", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32),
                ("epsilon", ctypes.c_double)]


class SjBatchInfo(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32),
                ("njobs", ctypes.c_uint32),
                ("pairs", ctypes.c_uint64),
                ("candidates", ctypes.c_uint64),
                ("evaluated", ctypes.c_uint64),
                ("rechecks", ctypes.c_uint64),
                ("capacity", ctypes.c_uint64),
                ("n_wu", ctypes.c_uint64),
                ("tile_candidates", ctypes.c_uint32),
                ("queue_grab", ctypes.c_uint32),
                ("grid", ctypes.c_uint32),
                ("tuned", ctypes.c_uint32),
                ("ms_build", ctypes.c_float),
                ("ms_estimate", ctypes.c_float),
                ("ms_graph", ctypes.c_float),
                ("ms_host_build", ctypes.c_float),
                ("ms_host_prepare", ctypes.c_float),
                ("ms_tune", ctypes.c_float)]


class SelfJoinError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("selfjoin error %d: %s" % (code, msg))
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libselfjoin.so and declare its signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libselfjoin.so is not built (run "
                          "`python -m paper_1809_09930_amd.build`); "
                          "there is no CPU fallback")
    lib = ctypes.CDLL(path)
    vp, u64, u32, dbl = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double
    lib.selfjoin_default_options.argtypes = [ctypes.POINTER(SjOptions)]
    lib.selfjoin_default_options.restype = None
    lib.selfjoin_build_index.argtypes = [vp, u64, u32, dbl, ctypes.POINTER(SjOptions), vp,
                                         ctypes.POINTER(vp)]
    lib.selfjoin_build_index.restype = ctypes.c_int
    lib.selfjoin_build_query.argtypes = [vp, vp, u64, vp, ctypes.POINTER(vp)]
    lib.selfjoin_build_query.restype = ctypes.c_int
    lib.selfjoin_run.argtypes = [vp, vp, ctypes.POINTER(u64)]
    lib.selfjoin_run.restype = ctypes.c_int
    lib.selfjoin_fetch_pairs.argtypes = [vp, u64, u64, vp, vp, vp, ctypes.POINTER(u64), vp]
    lib.selfjoin_fetch_offsets.argtypes = [vp, vp, vp]
    lib.selfjoin_fetch_offsets.restype = ctypes.c_int
    lib.selfjoin_fetch_offsets_noalloc.argtypes = [vp, vp, vp]
    lib.selfjoin_fetch_offsets_noalloc.restype = ctypes.c_int
    lib.selfjoin_fetch_pairs.restype = ctypes.c_int
    lib.selfjoin_get_info.argtypes = [vp, ctypes.POINTER(SjInfo)]
    lib.selfjoin_get_info.restype = ctypes.c_int
    lib.selfjoin_get_perm.argtypes = [vp, vp, u32]
    lib.selfjoin_get_perm.restype = ctypes.c_int
    lib.selfjoin_free.argtypes = [vp]
    lib.selfjoin_free.restype = None
    lib.selfjoin_last_error.argtypes = []
    lib.selfjoin_last_error.restype = ctypes.c_char_p
    lib.selfjoin_run_batched.argtypes = [ctypes.POINTER(SjJob), u32, ctypes.POINTER(SjOptions), vp,
                                         ctypes.POINTER(vp)]
    lib.selfjoin_run_batched.restype = ctypes.c_int
    lib.selfjoin_batch_replay.argtypes = [vp, ctypes.POINTER(ctypes.c_float)]
    lib.selfjoin_batch_replay.restype = ctypes.c_int
    lib.selfjoin_batch_range.argtypes = [vp, u32, ctypes.POINTER(u64), ctypes.POINTER(u64)]
    lib.selfjoin_batch_range.restype = ctypes.c_int
    lib.selfjoin_batch_fetch.argtypes = [vp, u32, u64, u64, vp, vp, vp, ctypes.POINTER(u64), vp]
    lib.selfjoin_batch_fetch.restype = ctypes.c_int
    lib.selfjoin_batch_get_info.argtypes = [vp, ctypes.POINTER(SjBatchInfo)]
    lib.selfjoin_batch_get_info.restype = ctypes.c_int
    lib.selfjoin_batch_free.argtypes = [vp]
    lib.selfjoin_batch_free.restype = None
    lib.selfjoin_release_cache.argtypes = [ctypes.POINTER(u64)]
    lib.selfjoin_release_cache.restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc):
    if rc != SJ_OK:
        msg = _lib.selfjoin_last_error()
        raise SelfJoinError(rc, msg.decode() if msg else "")


def default_options() -> SjOptions:
    o = SjOptions()
    load_library().selfjoin_default_options(ctypes.byref(o))
    return o


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def selfjoin_build_index(points, epsilon: float, k: int = 0, reorder: bool = True,
                         shortc: bool = True, batch_pairs: int = 0, min_batches: int = 0,
                         mem_budget: int = 0, k_min: int = 4, k_max: int = 8,
                         precision="fp32", fp32_form="auto", sortidu: bool = False,
                         stream=None):
    """Build the grid index over a float32 [n, d] tensor (CUDA or CPU).
    Returns an opaque handle (int)."""
    import torch
    lib = load_library()
    if points.dtype != torch.float32 or points.dim() != 2:
        raise ValueError("points must be a float32 [n, d] tensor")
    points = points.contiguous()
    o = default_options()
    o.k = int(k)
    o.k_min, o.k_max = int(k_min), int(k_max)
    o.reorder = 1 if reorder else 0
    o.shortc = 1 if shortc else 0
    o.batch_pairs = int(batch_pairs)
    o.min_batches = int(min_batches)
    o.mem_budget = int(mem_budget)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.fp32_form = FP32_FORMS[fp32_form] if isinstance(fp32_form, str) else int(fp32_form)
    o.sortidu = 1 if sortidu else 0
    h = ctypes.c_void_p()
    n, d = points.shape
    ptr = points.data_ptr() if points.numel() else None
    _check(lib.selfjoin_build_index(ptr, n, d, float(epsilon), ctypes.byref(o),
                                    _stream_handle(stream), ctypes.byref(h)))
    return h.value


def selfjoin_build_query(entries, queries, stream=None):
    """Query handle of the general join Q join_eps E: the float32 [m, d]
    tensor `queries` (CUDA or CPU) against the index `entries` (a handle of
    selfjoin_build_index, which must outlive the query handle).  Run, fetch
    and free it like any handle; its pairs are (query row, row of E)."""
    import torch
    lib = load_library()
    if queries.dtype != torch.float32 or queries.dim() != 2:
        raise ValueError("queries must be a float32 [m, d] tensor")
    queries = queries.contiguous()
    h = ctypes.c_void_p()
    ptr = queries.data_ptr() if queries.numel() else None
    _check(lib.selfjoin_build_query(entries, ptr, queries.shape[0], _stream_handle(stream),
                                    ctypes.byref(h)))
    return h.value


def selfjoin_run(handle, stream=None) -> int:
    total = ctypes.c_uint64()
    _check(load_library().selfjoin_run(handle, _stream_handle(stream), ctypes.byref(total)))
    return total.value


def selfjoin_fetch_pairs(handle, first: int, out_i=None, out_j=None, out_dist=None,
                         max_pairs: int | None = None, stream=None) -> int:
    """Copy result pairs [first, first + max_pairs) into the given tensors
    (uint32 stored as int32 / float32; CUDA or CPU).  Returns pairs written."""
    sizes = [t.numel() for t in (out_i, out_j, out_dist) if t is not None]
    if max_pairs is None:
        max_pairs = min(sizes) if sizes else 0
    for t in (out_i, out_j, out_dist):
        if t is not None and (t.numel() < max_pairs or not t.is_contiguous()):
            raise ValueError("output tensors must be contiguous with room for max_pairs")
    nw = ctypes.c_uint64()
    ptr = lambda t: None if t is None else t.data_ptr()  # noqa: E731
    _check(load_library().selfjoin_fetch_pairs(handle, int(first), int(max_pairs), ptr(out_i),
                                               ptr(out_j), ptr(out_dist), ctypes.byref(nw),
                                               _stream_handle(stream)))
    return nw.value


def selfjoin_fetch_offsets(handle, offsets, stream=None) -> None:
    """CSR row starts of the sorted result into an int64 tensor of n + 1
    entries (CUDA or CPU): the neighbours of point i are the j column
    [offsets[i], offsets[i + 1])."""
    if not offsets.is_contiguous():
        raise ValueError("offsets must be contiguous")
    _check(load_library().selfjoin_fetch_offsets(handle, offsets.data_ptr(),
                                                 _stream_handle(stream)))


def selfjoin_fetch_offsets_noalloc(handle, offsets, stream=None) -> None:
    """As selfjoin_fetch_offsets, with every temporary in the library's fixed
    per-device array: the call allocates no memory."""
    if not offsets.is_contiguous():
        raise ValueError("offsets must be contiguous")
    _check(load_library().selfjoin_fetch_offsets_noalloc(handle, offsets.data_ptr(),
                                                         _stream_handle(stream)))


def selfjoin_release_cache() -> int:
    """Free the device blocks the library keeps cached for the current
    device; returns the bytes freed."""
    out = ctypes.c_uint64(0)
    _check(load_library().selfjoin_release_cache(ctypes.byref(out)))
    return out.value


def selfjoin_get_info(handle) -> dict:
    info = SjInfo()
    info.struct_size = ctypes.sizeof(SjInfo)
    _check(load_library().selfjoin_get_info(handle, ctypes.byref(info)))
    return {name: getattr(info, name) for name, _ in SjInfo._fields_
            if name not in ("struct_size", "reserved")}


def selfjoin_get_perm(handle, d: int):
    arr = (ctypes.c_uint32 * d)()
    _check(load_library().selfjoin_get_perm(handle, arr, d))
    return list(arr)


def selfjoin_run_batched(points_list, eps_list, precision="fp16", autotune: bool = False,
                         k: int = 0, reorder: bool = True, stream=None):
    """Run len(points_list) independent self-joins in one persistent launch
    (float32 [n, d] tensors, CUDA or CPU).  Returns an opaque batch handle."""
    import torch
    lib = load_library()
    pts = [p.contiguous() for p in points_list]
    for p in pts:
        if p.dtype != torch.float32 or p.dim() != 2:
            raise ValueError("points must be float32 [n, d] tensors")
    jobs = (SjJob * len(pts))()
    for i, (p, e) in enumerate(zip(pts, eps_list)):
        jobs[i].points = p.data_ptr() if p.numel() else None
        jobs[i].n, jobs[i].d = p.shape
        jobs[i].epsilon = float(e)
    o = default_options()
    o.k = int(k)
    o.reorder = 1 if reorder else 0
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.autotune = 1 if autotune else 0
    h = ctypes.c_void_p()
    _check(lib.selfjoin_run_batched(jobs, len(pts), ctypes.byref(o), _stream_handle(stream),
                                    ctypes.byref(h)))
    return h.value


def selfjoin_batch_replay(batch) -> float:
    ms = ctypes.c_float()
    _check(load_library().selfjoin_batch_replay(batch, ctypes.byref(ms)))
    return ms.value


def selfjoin_batch_range(batch, job: int):
    first, count = ctypes.c_uint64(), ctypes.c_uint64()
    _check(load_library().selfjoin_batch_range(batch, job, ctypes.byref(first),
                                               ctypes.byref(count)))
    return first.value, count.value


def selfjoin_batch_fetch(batch, job: int, first: int, out_i=None, out_j=None, out_dist=None,
                         max_pairs: int | None = None, stream=None) -> int:
    sizes = [t.numel() for t in (out_i, out_j, out_dist) if t is not None]
    if max_pairs is None:
        max_pairs = min(sizes) if sizes else 0
    nw = ctypes.c_uint64()
    ptr = lambda t: None if t is None else t.data_ptr()  # noqa: E731
    _check(load_library().selfjoin_batch_fetch(batch, job, int(first), int(max_pairs),
                                               ptr(out_i), ptr(out_j), ptr(out_dist),
                                               ctypes.byref(nw), _stream_handle(stream)))
    return nw.value


def selfjoin_batch_get_info(batch) -> dict:
    info = SjBatchInfo()
    info.struct_size = ctypes.sizeof(SjBatchInfo)
    _check(load_library().selfjoin_batch_get_info(batch, ctypes.byref(info)))
    return {name: getattr(info, name) for name, _ in SjBatchInfo._fields_
            if name != "struct_size"}


def selfjoin_batch_free(batch) -> None:
    if batch:
        load_library().selfjoin_batch_free(batch)


def selfjoin_free(handle) -> None:
    if handle:
        load_library().selfjoin_free(handle)


class SelfJoin:
    """Convenience wrapper: build on construction, run, fetch all pairs."""

    def __init__(self, points, epsilon: float, **opts):
        self.n, self.d = points.shape
        self.handle = selfjoin_build_index(points, epsilon, **opts)
        self.total = None

    def run(self) -> int:
        self.total = selfjoin_run(self.handle)
        return self.total

    def pairs(self, with_dist: bool = False, device="cuda"):
        """All result pairs as (i, j[, dist]) tensors, sorted by (i, j)."""
        import torch
        if self.total is None:
            self.run()
        m = self.total
        oi = torch.empty(m, dtype=torch.int32, device=device)
        oj = torch.empty(m, dtype=torch.int32, device=device)
        od = torch.empty(m, dtype=torch.float32, device=device) if with_dist else None
        if m:
            got = selfjoin_fetch_pairs(self.handle, 0, oi, oj, od, max_pairs=m)
            assert got == m
        return (oi, oj, od) if with_dist else (oi, oj)

    def info(self) -> dict:
        return selfjoin_get_info(self.handle)

    def perm(self):
        return selfjoin_get_perm(self.handle, self.d)

    def close(self):
        selfjoin_free(self.handle)
        self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                self.close()
        except Exception:
            pass
