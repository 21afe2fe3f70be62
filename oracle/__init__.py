"""FP64 CPU oracle for cRMSD (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports it, and this package never imports the
product.  The arithmetic lives in ``crmsd_oracle.c`` (plain C, FP64, OpenMP):
the definition of cRMSD (Algorithms, Eq. 1) evaluated with an explicit Kabsch
superposition (one-sided Jacobi SVD of the 3x3 correlation matrix, proper
rotation, explicit residual), and the definition of dRMSD (Algorithms, Eq. 5)
as a direct sum over atom pairs.  Every function takes float32 or float64
coordinates and promotes them exactly to float64.  ``cmo*`` give the contact map overlap (Algorithms, Eq. 6-7)
with integer contact counts.  ``kmedoids`` clusters a
packed float32 score matrix (K-means with member centres, the representative
by the smallest <R>/f) with plain FP64 sums of the scores.

Parity status: pinned (see ``tests/test_oracle_*.py``: invariants, closed
forms, library-routine equalities, brute force on tiny inputs, finite
differences for the gradient).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "crmsd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_crmsd.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
               "-ffp-contract=off", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    lp = ctypes.POINTER(ctypes.c_int64)
    i64, cint = ctypes.c_int64, ctypes.c_int
    lib.oracle_crmsd_pair.restype = ctypes.c_double
    lib.oracle_crmsd_pair.argtypes = [dp, dp, i64]
    lib.oracle_kabsch_rotation.restype = None
    lib.oracle_kabsch_rotation.argtypes = [dp, dp, i64, dp]
    lib.oracle_max_threads.restype = cint
    lib.oracle_crmsd_matrix.argtypes = [dp, i64, i64, dp, cint]
    lib.oracle_crmsd_pairs.argtypes = [dp, i64, i64, lp, lp, i64, dp, cint]
    lib.oracle_crmsd_cross.argtypes = [dp, i64, dp, i64, i64, dp, cint]
    lib.oracle_crmsd_grad_pair.argtypes = [dp, dp, i64, dp, dp, dp]
    lib.oracle_crmsd_matrix_grad.argtypes = [dp, i64, i64, dp, dp, cint]
    lib.oracle_crmsd_cross_grad.argtypes = [dp, i64, dp, i64, i64, dp, dp, dp, cint]
    lib.oracle_crmsd_matrix_grad_rows.argtypes = [dp, i64, i64, dp, lp, i64, dp, cint]
    lib.oracle_drmsd_pair.restype = ctypes.c_double
    lib.oracle_drmsd_pair.argtypes = [dp, dp, i64]
    lib.oracle_drmsd_matrix.argtypes = [dp, i64, i64, dp, cint]
    lib.oracle_drmsd_pairs.argtypes = [dp, i64, i64, lp, lp, i64, dp, cint]
    lib.oracle_cmo_pair.restype = ctypes.c_double
    lib.oracle_cmo_pair.argtypes = [dp, dp, i64, ctypes.c_double]
    lib.oracle_cmo_matrix.argtypes = [dp, i64, i64, ctypes.c_double, dp, cint]
    lib.oracle_cmo_pairs.argtypes = [dp, i64, i64, ctypes.c_double, lp, lp, i64, dp, cint]
    lib.oracle_cmo_matrix.restype = cint
    lib.oracle_cmo_pairs.restype = cint
    lib.oracle_cmo_near_ties.argtypes = [dp, i64, i64, ctypes.c_double, ctypes.c_double, lp]
    lib.oracle_cmo_near_ties.restype = cint
    i32p = ctypes.POINTER(ctypes.c_int32)
    fp = ctypes.POINTER(ctypes.c_float)
    lib.oracle_kmedoids.argtypes = [fp, i64, i64, i32p, i64, i32p, i32p, lp, dp, lp, dp]
    lib.oracle_kmedoids.restype = cint
    for f in ("oracle_crmsd_matrix", "oracle_crmsd_pairs", "oracle_crmsd_cross",
              "oracle_crmsd_grad_pair", "oracle_crmsd_matrix_grad", "oracle_crmsd_cross_grad",
              "oracle_crmsd_matrix_grad_rows", "oracle_drmsd_matrix", "oracle_drmsd_pairs"):
        getattr(lib, f).restype = cint
    _lib = lib
    return lib


def _d(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _p(x):
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"{what}: oracle rejected its arguments (code {rc})")


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def crmsd(a, b) -> float:
    """cRMSD of two [L,3] models."""
    a, b = _d(a), _d(b)
    assert a.shape == b.shape and a.ndim == 2 and a.shape[1] == 3
    return float(_load().oracle_crmsd_pair(_p(a), _p(b), a.shape[0]))


def rotation(a, b) -> np.ndarray:
    """Optimal proper rotation R with R (a - mean a) ~ (b - mean b)."""
    a, b = _d(a), _d(b)
    R = np.zeros((3, 3))
    _load().oracle_kabsch_rotation(_p(a), _p(b), a.shape[0], _p(R))
    return R


def crmsd_matrix(x, threads: int = 0) -> np.ndarray:
    """Packed upper triangle [N(N-1)/2] (i<j, row-major) of an [N,L,3] ensemble."""
    x = _d(x)
    N, L = x.shape[0], x.shape[1]
    out = np.zeros(N * (N - 1) // 2)
    _check(_load().oracle_crmsd_matrix(_p(x), N, L, _p(out), threads), "crmsd_matrix")
    return out


def crmsd_pairs(x, I, J, threads: int = 0) -> np.ndarray:
    """cRMSD of selected pairs (I[p], J[p]) of one ensemble."""
    x = _d(x)
    I = np.ascontiguousarray(I, dtype=np.int64)
    J = np.ascontiguousarray(J, dtype=np.int64)
    out = np.zeros(I.shape[0])
    lp = ctypes.POINTER(ctypes.c_int64)
    _check(_load().oracle_crmsd_pairs(_p(x), x.shape[0], x.shape[1], I.ctypes.data_as(lp),
                                      J.ctypes.data_as(lp), I.shape[0], _p(out), threads),
           "crmsd_pairs")
    return out


def crmsd_cross(a, b, threads: int = 0) -> np.ndarray:
    """Dense [Na, Nb] cRMSD between two sets of models of equal L."""
    a, b = _d(a), _d(b)
    out = np.zeros((a.shape[0], b.shape[0]))
    _check(_load().oracle_crmsd_cross(_p(a), a.shape[0], _p(b), b.shape[0], a.shape[1],
                                      _p(out), threads), "crmsd_cross")
    return out


def crmsd_grad_pair(a, b):
    """(rmsd, dRMSD/dA, dRMSD/dB) for one pair."""
    a, b = _d(a), _d(b)
    gA, gB = np.zeros_like(a), np.zeros_like(b)
    r = np.zeros(1)
    _check(_load().oracle_crmsd_grad_pair(_p(a), _p(b), a.shape[0], _p(gA), _p(gB), _p(r)),
           "crmsd_grad_pair")
    return float(r[0]), gA, gB


def crmsd_matrix_grad(x, g, threads: int = 0) -> np.ndarray:
    """d/dX of sum_{i<j} g[k(i,j)] cRMSD_ij, shape [N,L,3]."""
    x, g = _d(x), _d(g)
    N = x.shape[0]
    assert g.shape == (N * (N - 1) // 2,)
    out = np.zeros_like(x)
    _check(_load().oracle_crmsd_matrix_grad(_p(x), N, x.shape[1], _p(g), _p(out), threads),
           "crmsd_matrix_grad")
    return out


def crmsd_matrix_grad_rows(x, g, rows, threads: int = 0) -> np.ndarray:
    """Rows `rows` of crmsd_matrix_grad(x, g), shape [len(rows), L, 3]."""
    x, g = _d(x), _d(g)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros((rows.shape[0], x.shape[1], 3))
    lp = ctypes.POINTER(ctypes.c_int64)
    _check(_load().oracle_crmsd_matrix_grad_rows(_p(x), x.shape[0], x.shape[1], _p(g),
                                                 rows.ctypes.data_as(lp), rows.shape[0],
                                                 _p(out), threads), "crmsd_matrix_grad_rows")
    return out


def crmsd_cross_grad(a, b, g, threads: int = 0):
    """(d/dA, d/dB) of sum_{ia,ib} g[ia,ib] cRMSD(A_ia, B_ib)."""
    a, b, g = _d(a), _d(b), _d(g)
    assert g.shape == (a.shape[0], b.shape[0])
    gA, gB = np.zeros_like(a), np.zeros_like(b)
    _check(_load().oracle_crmsd_cross_grad(_p(a), a.shape[0], _p(b), b.shape[0], a.shape[1],
                                           _p(g), _p(gA), _p(gB), threads), "crmsd_cross_grad")
    return gA, gB


def drmsd(a, b) -> float:
    """Distance RMSD (Eq. 5) of two [L,3] models."""
    a, b = _d(a), _d(b)
    assert a.shape == b.shape and a.ndim == 2 and a.shape[1] == 3
    return float(_load().oracle_drmsd_pair(_p(a), _p(b), a.shape[0]))


def drmsd_matrix(x, threads: int = 0) -> np.ndarray:
    """Packed all-vs-all dRMSD of an [N,L,3] ensemble."""
    x = _d(x)
    N, L = x.shape[0], x.shape[1]
    out = np.zeros(N * (N - 1) // 2)
    _check(_load().oracle_drmsd_matrix(_p(x), N, L, _p(out), threads), "drmsd_matrix")
    return out


def drmsd_pairs(x, I, J, threads: int = 0) -> np.ndarray:
    """dRMSD of selected pairs (I[p], J[p]) of one ensemble."""
    x = _d(x)
    I = np.ascontiguousarray(I, dtype=np.int64)
    J = np.ascontiguousarray(J, dtype=np.int64)
    out = np.zeros(I.shape[0])
    lp = ctypes.POINTER(ctypes.c_int64)
    _check(_load().oracle_drmsd_pairs(_p(x), x.shape[0], x.shape[1], I.ctypes.data_as(lp),
                                      J.ctypes.data_as(lp), I.shape[0], _p(out), threads),
           "drmsd_pairs")
    return out


def cmo(A, B, cutoff: float) -> float:
    """Contact map overlap (Sorensen index, 0..100) of two models."""
    A, B = _d(A), _d(B)
    return float(_load().oracle_cmo_pair(_p(A), _p(B), A.shape[0], float(cutoff)))


def cmo_matrix(x, cutoff: float, threads: int = 0) -> np.ndarray:
    """Packed all-vs-all contact map overlap of an [N,L,3] ensemble."""
    x = _d(x)
    N, L = x.shape[0], x.shape[1]
    out = np.zeros(N * (N - 1) // 2)
    _check(_load().oracle_cmo_matrix(_p(x), N, L, float(cutoff), _p(out), threads), "cmo_matrix")
    return out


def cmo_pairs(x, I, J, cutoff: float, threads: int = 0) -> np.ndarray:
    """Contact map overlap of selected pairs (I[p], J[p]) of one ensemble."""
    x = _d(x)
    I = np.ascontiguousarray(I, dtype=np.int64)
    J = np.ascontiguousarray(J, dtype=np.int64)
    out = np.zeros(I.shape[0])
    lp = ctypes.POINTER(ctypes.c_int64)
    _check(_load().oracle_cmo_pairs(_p(x), x.shape[0], x.shape[1], float(cutoff),
                                    I.ctypes.data_as(lp), J.ctypes.data_as(lp), I.shape[0],
                                    _p(out), threads), "cmo_pairs")
    return out


def kmedoids(D, N: int, k: int, init, max_iter: int = 100) -> dict:
    """K-means over a packed float32 score matrix with members as centres
    (K-medoids, alternating assignment / update), plain FP64 sums of the
    scores, and the representative cluster by min <R>/f.  ``tie_margin`` is
    the smallest (second smallest - smallest in-cluster sum) / (n - 1) met by
    any update: how close the trajectory came to a tie, per summed score.
    See the clustering section of crmsd_oracle.c for the exact rules."""
    D = np.ascontiguousarray(D, dtype=np.float32)
    assert D.shape == (N * (N - 1) // 2,)
    init = np.ascontiguousarray(init, dtype=np.int32)
    label = np.zeros(N, np.int32)
    med = np.zeros(k, np.int32)
    size = np.zeros(k, np.int64)
    mean_r = np.zeros(k)
    info = np.zeros(3, np.int64)
    margin = np.zeros(1)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lp = ctypes.POINTER(ctypes.c_int64)
    rc = _load().oracle_kmedoids(D.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), N, k,
                                 init.ctypes.data_as(i32p), max_iter, label.ctypes.data_as(i32p),
                                 med.ctypes.data_as(i32p), size.ctypes.data_as(lp), _p(mean_r),
                                 info.ctypes.data_as(lp), _p(margin))
    _check(rc, "kmedoids")
    rep = int(info[0])
    return {"labels": label, "medoids": med, "sizes": size, "mean_r": mean_r,
            "rep_cluster": rep, "representative": int(med[rep]) if rep >= 0 else -1,
            "iterations": int(info[1]), "converged": bool(info[2]),
            "tie_margin": float(margin[0])}


def cmo_near_ties(x, cutoff: float, rel: float = 1e-12) -> np.ndarray:
    """Per model of an [N,L,3] ensemble, the number of atom pairs whose
    squared distance is within rel * cutoff^2 of cutoff^2 (where another
    rounding of the same squared distance could decide the contact the
    other way).  A comparison diagnostic, not part of the method."""
    x = _d(x)
    cnt = np.zeros(x.shape[0], np.int64)
    _check(_load().oracle_cmo_near_ties(_p(x), x.shape[0], x.shape[1], float(cutoff), float(rel),
                                        cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
           "cmo_near_ties")
    return cnt


def packed_index(i, j, N):
    """k(i,j) = i(2N-i-1)/2 + j-i-1 for i<j (int64)."""
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    return i * (2 * N - i - 1) // 2 + j - i - 1
