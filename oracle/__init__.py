"""Plain CPU oracle for the Euclidean epsilon self-join.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product library never does, and
this package imports nothing from it.

Contents (each function cites the passage of Gowanlock & Karsin, "GPU
Accelerated Similarity Self-Join for Multi-Dimensional Data", it follows):

* ``bruteforce``      O1: nested-loop join, FP64 canonical predicate (C).
* ``rows``            O1 for selected query rows (C).
* ``grid_join``       O2: grid-index join over k indexed dimensions (C).
* ``cell_coords``     grid cell coordinates (C; Figure 1/2 pins).
* ``grid_candidates`` the points one query's grid search visits (C).
* ``sortidu_candidates`` the same with SORTIDU's search along u (C).
* ``rows_smallest``   K smallest distances per row (C; eps calibration).
* ``bruteforce_np``   O1': numpy twin of O1 (same rounding sequence).
* ``exact_int_join``  O0: exact integer join for data on a 2^-g grid.
* ``join``            O1q: nested-loop general join Q join_eps E (C).
* ``reorder_perm``    REORDER: variance-ranked dimension order.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_GCC_FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
              "-shared", "-fPIC", "-Wall"]

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *_GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    u64, u32, f64, i64 = (ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double,
                          ctypes.c_int64)
    lib.oracle_bruteforce.argtypes = [P, u64, u32, f64, P, P, P, P, u64]
    lib.oracle_bruteforce.restype = i64
    lib.oracle_join.argtypes = [P, u64, P, u64, u32, f64, P, P, P, P, u64]
    lib.oracle_join.restype = i64
    lib.oracle_rows.argtypes = [P, u64, u32, f64, P, u64, P, P, P, u64]
    lib.oracle_rows.restype = i64
    lib.oracle_rows_smallest.argtypes = [P, u64, u32, P, u64, u32, P]
    lib.oracle_rows_smallest.restype = ctypes.c_int
    lib.oracle_cell_coords.argtypes = [P, u64, u32, f64, u32, P, ctypes.c_int,
                                       f64, P]
    lib.oracle_cell_coords.restype = ctypes.c_int
    lib.oracle_grid.argtypes = [P, u64, u32, f64, u32, P, ctypes.c_int, f64,
                                P, P, u64, P]
    lib.oracle_grid.restype = i64
    lib.oracle_grid_candidates.argtypes = [P, u64, u32, f64, u32, P,
                                           ctypes.c_int, f64, u64, P, u64]
    lib.oracle_grid_candidates.restype = i64
    lib.oracle_sortidu_candidates.argtypes = [P, u64, u32, f64, u32, P, ctypes.c_int, f64,
                                              u32, u64, P, u64]
    lib.oracle_sortidu_candidates.restype = i64
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _points(P):
    P = np.ascontiguousarray(P, dtype=np.float32)
    if P.ndim != 2:
        raise ValueError("points must be a 2-D [n][d] array")
    return P


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def bruteforce(P, eps: float, with_dist: bool = False):
    """O1 (Section 3.1): every ordered pair (i, j) with the FP64 canonical
    squared distance <= fl(eps*eps), in ascending (i, j) order.
    Returns (i, j) or (i, j, s) as numpy arrays."""
    P = _points(P)
    n, d = P.shape
    lib = _load()
    counts = np.zeros(max(n, 1), dtype=np.uint64)
    total = lib.oracle_bruteforce(_ptr(P), n, d, float(eps), _ptr(counts),
                                  None, None, None, 0)
    if total < 0:
        raise MemoryError("oracle_bruteforce failed")
    oi = np.empty(total, dtype=np.uint32)
    oj = np.empty(total, dtype=np.uint32)
    os_ = np.empty(total, dtype=np.float64) if with_dist else None
    got = lib.oracle_bruteforce(_ptr(P), n, d, float(eps), None, _ptr(oi),
                                _ptr(oj), _ptr(os_), total)
    assert got == total
    return (oi, oj, os_) if with_dist else (oi, oj)


def join(Q, E, eps: float, with_dist: bool = False):
    """O1q (Section 3.1, the similarity join Q join_eps E): every pair (q, e)
    of a row of Q and a row of E with the FP64 canonical squared distance
    <= fl(eps*eps), in ascending (q, e) order.  The self-join is join(P, P).
    Returns (q, e) or (q, e, s) as numpy arrays."""
    Q = _points(Q)
    E = _points(E)
    m, d = Q.shape
    n, d2 = E.shape
    if m and n and d != d2:
        raise ValueError("Q and E must have the same number of dimensions")
    d = d if m else d2
    lib = _load()
    total = lib.oracle_join(_ptr(Q), m, _ptr(E), n, d, float(eps), None,
                            None, None, None, 0)
    if total < 0:
        raise MemoryError("oracle_join failed")
    oi = np.empty(total, dtype=np.uint32)
    oj = np.empty(total, dtype=np.uint32)
    os_ = np.empty(total, dtype=np.float64) if with_dist else None
    got = lib.oracle_join(_ptr(Q), m, _ptr(E), n, d, float(eps), None,
                          _ptr(oi), _ptr(oj), _ptr(os_), total)
    assert got == total
    return (oi, oj, os_) if with_dist else (oi, oj)


def rows(P, eps: float, query_rows, with_dist: bool = False):
    """O1 restricted to the listed query rows (Section 3.1).  Returns
    (counts per listed row, concatenated j arrays[, distances])."""
    P = _points(P)
    n, d = P.shape
    q = np.ascontiguousarray(query_rows, dtype=np.uint64)
    lib = _load()
    counts = np.zeros(max(len(q), 1), dtype=np.uint64)
    total = lib.oracle_rows(_ptr(P), n, d, float(eps), _ptr(q), len(q),
                            _ptr(counts), None, None, 0)
    oj = np.empty(total, dtype=np.uint32)
    os_ = np.empty(total, dtype=np.float64) if with_dist else None
    got = lib.oracle_rows(_ptr(P), n, d, float(eps), _ptr(q), len(q), None,
                          _ptr(oj), _ptr(os_), total)
    assert got == total
    counts = counts[:len(q)]
    return (counts, oj, os_) if with_dist else (counts, oj)


def rows_smallest(P, query_rows, K: int):
    """K smallest canonical squared distances from each listed row to the
    other points, ascending (+inf padded)."""
    P = _points(P)
    n, d = P.shape
    q = np.ascontiguousarray(query_rows, dtype=np.uint64)
    out = np.empty((len(q), K), dtype=np.float64)
    _load().oracle_rows_smallest(_ptr(P), n, d, _ptr(q), len(q), K, _ptr(out))
    return out


def cell_coords(P, eps: float, dims, origin_zero: bool = False,
                width_factor: float = 1.0 + 2.0 ** -20):
    """Grid cell coordinates over the listed dims (Section 3.2.1): cells of
    side eps*width_factor, origin 0 or the per-dimension minimum."""
    P = _points(P)
    n, d = P.shape
    dims = np.ascontiguousarray(dims, dtype=np.uint32)
    out = np.empty((n, len(dims)), dtype=np.int64)
    _load().oracle_cell_coords(_ptr(P), n, d, float(eps), len(dims),
                               _ptr(dims), int(origin_zero),
                               float(width_factor), _ptr(out))
    return out


def grid_join(P, eps: float, dims, origin_zero: bool = False,
              width_factor: float = 1.0 + 2.0 ** -20):
    """O2 (Sections 3.2.1 and 4.1, Algorithm 1): grid over the listed k dims,
    3^k adjacent cells per query found by binary search, FP64 canonical
    predicate over all dimensions.  Returns (i, j, n_candidates)."""
    P = _points(P)
    n, d = P.shape
    dims = np.ascontiguousarray(dims, dtype=np.uint32)
    lib = _load()
    cand = np.zeros(1, dtype=np.uint64)
    total = lib.oracle_grid(_ptr(P), n, d, float(eps), len(dims), _ptr(dims),
                            int(origin_zero), float(width_factor), None, None,
                            0, _ptr(cand))
    if total < 0:
        raise RuntimeError("oracle_grid failed (%d)" % total)
    oi = np.empty(total, dtype=np.uint32)
    oj = np.empty(total, dtype=np.uint32)
    got = lib.oracle_grid(_ptr(P), n, d, float(eps), len(dims), _ptr(dims),
                          int(origin_zero), float(width_factor), _ptr(oi),
                          _ptr(oj), total, _ptr(cand))
    assert got == total
    return oi, oj, int(cand[0])


def grid_candidates(P, eps: float, dims, query: int,
                    origin_zero: bool = False,
                    width_factor: float = 1.0 + 2.0 ** -20):
    """Candidate point ids the grid search visits for one query (Algorithm 1,
    getAdjCells and the loop over adjacent cells)."""
    P = _points(P)
    n, d = P.shape
    dims = np.ascontiguousarray(dims, dtype=np.uint32)
    lib = _load()
    cnt = lib.oracle_grid_candidates(_ptr(P), n, d, float(eps), len(dims),
                                     _ptr(dims), int(origin_zero),
                                     float(width_factor), int(query), None, 0)
    out = np.empty(max(cnt, 0), dtype=np.uint32)
    lib.oracle_grid_candidates(_ptr(P), n, d, float(eps), len(dims),
                               _ptr(dims), int(origin_zero), float(width_factor),
                               int(query), _ptr(out), len(out))
    return out


def sortidu_candidates(P, eps: float, dims, u: int, query: int,
                       origin_zero: bool = False,
                       width_factor: float = 1.0 + 2.0 ** -20):
    """SORTIDU (Section 4.3): candidate ids one query visits when every cell
    is sorted by the un-indexed dimension u -- a binary search to the first
    point within eps along u, then a scan until one is farther.  Cells in the
    order of the 3^k offsets, points in increasing u inside each."""
    P = _points(P)
    n, d = P.shape
    dims = np.ascontiguousarray(dims, dtype=np.uint32)
    lib = _load()
    args = (_ptr(P), n, d, float(eps), len(dims), _ptr(dims), int(origin_zero),
            float(width_factor), int(u), int(query))
    cnt = lib.oracle_sortidu_candidates(*args, None, 0)
    if cnt < 0:
        raise ValueError("oracle_sortidu_candidates failed (%d)" % cnt)
    out = np.empty(cnt, dtype=np.uint32)
    got = lib.oracle_sortidu_candidates(*args, _ptr(out), len(out))
    assert got == cnt
    return out


def bruteforce_np(P, eps: float):
    """O1' (Section 3.1): numpy twin of O1 with the same rounding sequence --
    per query row, acc = acc + diff*diff one dimension at a time in original
    order (no pairwise summation, no FMA).  Returns (i, j)."""
    P = _points(P)
    n, d = P.shape
    X = P.astype(np.float64)
    eps2 = float(eps) * float(eps)
    out_i, out_j = [], []
    for i in range(n):
        acc = np.zeros(n, dtype=np.float64)
        for t in range(d):
            diff = X[i, t] - X[:, t]
            acc = acc + diff * diff
        js = np.nonzero(acc <= eps2)[0]
        out_i.append(np.full(len(js), i, dtype=np.uint32))
        out_j.append(js.astype(np.uint32))
    if not out_i:
        return np.empty(0, np.uint32), np.empty(0, np.uint32)
    return np.concatenate(out_i), np.concatenate(out_j)


def exact_int_join(A, T: int, B=None):
    """O0: the join in exact integer arithmetic for data on a 2^-g grid.
    A = P * 2^g as int64, T = floor(eps2 * 2^(2g)); pair iff
    sum_t (A_i,t - A_j,t)^2 <= T.  With B given, the general join A join B
    (rows i of A, rows j of B) instead of the self-join of A.  The caller
    keeps |A|, |B| < 2^30 and d small enough that the int64 sums cannot
    overflow (asserted).  Returns (i, j)."""
    A = np.ascontiguousarray(A, dtype=np.int64)
    B = A if B is None else np.ascontiguousarray(B, dtype=np.int64)
    n, d = A.shape
    if n and len(B):
        span = max(int(A.max()), int(B.max())) - min(int(A.min()), int(B.min()))
        assert span * span * d < 2 ** 62, "int64 sums could overflow"
    out_i, out_j = [], []
    for i in range(n):
        acc = np.zeros(len(B), dtype=np.int64)
        for t in range(d):
            diff = B[:, t] - A[i, t]
            acc += diff * diff
        js = np.nonzero(acc <= T)[0]
        out_i.append(np.full(len(js), i, dtype=np.uint32))
        out_j.append(js.astype(np.uint32))
    if not out_i:
        return np.empty(0, np.uint32), np.empty(0, np.uint32)
    return np.concatenate(out_i), np.concatenate(out_j)


def reorder_sample_rows(n: int, stride: int = 100, full_below: int = 10_000):
    """The deterministic variance sample: every stride-th point from 0, or all
    points when n <= full_below (Section 4.2 asks for a 1% sample without
    fixing how it is drawn)."""
    if n <= full_below:
        return np.arange(n)
    return np.arange(0, n, stride)


def reorder_perm(P, stride: int = 100, full_below: int = 10_000):
    """REORDER (Section 4.2): estimate each dimension's variance on a 1%
    sample and order the dimensions from highest to lowest variance.
    Variance is the unbiased FP64 estimate; equal variances keep the lower
    original index first.  Returns (perm, variances) with perm[r] the
    original index of the r-th reordered dimension."""
    P = _points(P)
    S = P[reorder_sample_rows(P.shape[0], stride, full_below)].astype(np.float64)
    if S.shape[0] < 2:
        var = np.zeros(P.shape[1])
    else:
        var = np.var(S, axis=0, ddof=1)
    perm = np.argsort(-var, kind="stable")
    return perm.astype(np.uint32), var


def calibrate_eps(P, target: float, query_rows, k0: int | None = None):
    """Epsilon for a target selectivity S_D (Section 5.2: S_D is the mean
    number of neighbours per point excluding the point itself).

    Over the listed query rows, take m = round(target * #rows) and eps2* = the
    m-th smallest canonical squared distance among all (query, other point)
    pairs, found exactly by growing per-row lists of smallest distances until
    no row can hide a smaller value.  eps is the smallest binary64 with
    fl(eps*eps) >= eps2*.  Returns (eps, achieved S_D on the sample)."""
    q = np.asarray(query_rows, dtype=np.int64)
    m = max(1, int(round(target * len(q))))
    K = int(k0 or max(64, 4 * int(math.ceil(target))))
    redo = np.arange(len(q))
    lists = [None] * len(q)
    while True:
        sm = rows_smallest(P, q[redo], K)
        for r, row in zip(redo, sm):
            lists[r] = row
        allv = np.concatenate(lists)
        allv = allv[np.isfinite(allv)]
        if len(allv) < m:
            raise ValueError("not enough pairs for the target")
        t = np.partition(allv, m - 1)[m - 1]
        kth = np.array([row[-1] for row in lists])
        full = np.array([len(row) == K and np.isfinite(row[-1]) for row in lists])
        redo = np.nonzero(full & (kth <= t))[0]
        if len(redo) == 0:
            break
        K *= 4
    eps = float(np.sqrt(t))
    while eps * eps < t:
        eps = float(np.nextafter(eps, np.inf))
    while True:  # smallest such eps
        prev = float(np.nextafter(eps, 0.0))
        if prev * prev >= t:
            eps = prev
        else:
            break
    eps2 = eps * eps
    achieved = float(np.count_nonzero(allv <= eps2)) / len(q)
    return eps, achieved
