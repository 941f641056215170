"""ctypes wrapper of the oracle's compression and H-matrix product (hcore.c).

Oracle -- test infrastructure only (tests/, smoke(), bench.py's cpu_baseline).
The structure it returns (tree permutation, neighbour lists, near/far lists,
skeletons, interpolation matrices) is the CPU build of the hierarchical
approximation K~ = D + S + UV of Eq. (3); ``matvec`` is its float64 product.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from .build import build

_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        vp, i64, i32, f64 = C.c_void_p, C.c_int64, C.c_int, C.c_double
        L.orc_compress.restype = vp
        L.orc_compress.argtypes = [vp, i64, i32, i32, f64, i32, i32, i32, i32, f64, f64, C.c_uint64]
        L.orc_free.argtypes = [vp]
        L.orc_get_perm.argtypes = [vp, vp]
        L.orc_get_knn.argtypes = [vp, vp, vp]
        L.orc_near_nnz.restype = i64
        L.orc_near_nnz.argtypes = [vp]
        L.orc_far_nnz.restype = i64
        L.orc_far_nnz.argtypes = [vp]
        L.orc_get_near.argtypes = [vp, vp, vp]
        L.orc_get_far.argtypes = [vp, vp, vp]
        L.orc_get_ranks.argtypes = [vp, vp, vp, vp]
        L.orc_get_node.argtypes = [vp, i64, vp, vp, vp]
        L.orc_hmatvec.restype = i32
        L.orc_hmatvec.argtypes = [vp, vp, vp, i32]
        L.orc_hmatvec_abs.restype = i32
        L.orc_hmatvec_abs.argtypes = [vp, vp, vp, i32]
        L.orc_dense_kmatvec.argtypes = [vp, i64, i32, i32, f64, vp, i32, vp, i64, i64]
        L.orc_dense_sqdist.argtypes = [vp, i64, i32, i32, i64, i64, vp]
        L.orc_kernel.restype = f64
        L.orc_kernel.argtypes = [vp, i64, i32, i32, f64, i64, i64]
        L.orc_det_exp.restype = f64
        L.orc_det_exp.argtypes = [f64]
        L.orc_rand_u32.restype = C.c_uint32
        L.orc_rand_u32.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_build_tree.restype = i32
        L.orc_get_trace.restype = i32
        L.orc_get_trace.argtypes = [vp, i64, vp]
        L.orc_sample_positions.restype = i32
        L.orc_sample_positions.argtypes = [C.c_uint64, C.c_uint32, i64, i32, vp]
        L.orc_pivoted_id.restype = i32
        L.orc_pivoted_id.argtypes = [vp, i32, i32, i32, f64, vp, vp, vp, vp]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _points(X: np.ndarray):
    if X.dtype == np.uint8:
        return np.ascontiguousarray(X), 1
    return np.ascontiguousarray(X, dtype=np.float64), 0


def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def rand_u32(seed, purpose, a, b, i):
    return int(lib().orc_rand_u32(seed, purpose, a, b, i))


def det_exp(x: float) -> float:
    """The compression's exponential (Cody-Waite reduction, Taylor polynomial of
    degree 13), as the CPU build evaluates it."""
    return lib().orc_det_exp(float(x))


def sample_positions(seed, node, n, ns):
    """Floyd's sample of ns distinct positions of [0, n) for tree node ``node`` (ascending)."""
    out = np.zeros(max(ns, 1), np.int64)
    cnt = lib().orc_sample_positions(seed, node, n, ns, _ptr(out))
    return out[:cnt]


def pivoted_id(B, s, tau):
    """Oracle ID of one block: (rank, column order cp, P [rank x nc], trace [steps x 2])."""
    B = np.array(B, dtype=np.float64, order="C", copy=True)
    nr, nc = B.shape
    cp = np.zeros(max(nc, 1), np.int32)
    P = np.zeros(max(s * nc, 1), np.float64)
    kmax = min(nr, nc, s)
    trace = np.zeros(2 * (kmax + 1), np.float64)
    steps = C.c_int32(0)
    rk = lib().orc_pivoted_id(_ptr(B), nr, nc, s, float(tau), _ptr(cp), _ptr(P), _ptr(trace), C.byref(steps))
    return rk, cp[:nc], P[:rk * nc].reshape(rk, nc), trace[:2 * steps.value].reshape(-1, 2)


def tree_depth(n: int, m: int) -> int:
    d = 0
    while -(-n // (1 << d)) > m:
        d += 1
    return d


def tree_ranges(n: int, depth: int):
    """(start, size) per heap id; root 1, children 2h, 2h+1, left gets floor."""
    nn = 1 << (depth + 1)
    start = np.zeros(nn, np.int64)
    size = np.zeros(nn, np.int64)
    size[1] = n
    for h in range(1, 1 << depth):
        nl = size[h] // 2
        start[2 * h], size[2 * h] = start[h], nl
        start[2 * h + 1], size[2 * h + 1] = start[h] + nl, size[h] - nl
    return start, size


class HMatrix:
    """Oracle-side compressed operator.  All vectors in original point order."""

    def __init__(self, X, eps, m, s, tau, k, seed, knn_iters=10, budget=0.05, depth=None):
        self.X, self.is_u8 = _points(X)
        self.n, self.dim = self.X.shape
        self.eps, self.m, self.s, self.tau, self.k = float(eps), m, s, float(tau), k
        self.seed, self.knn_iters, self.budget = seed, knn_iters, float(budget)
        self.depth = tree_depth(self.n, m) if depth is None else depth
        if -(-self.n // (1 << self.depth)) // 2 < 1 or self.n // (1 << self.depth) <= k:
            raise ValueError("every leaf must hold more than k points")
        self.h = lib().orc_compress(_ptr(self.X), self.n, self.dim, self.is_u8, self.eps, self.depth, k,
                                    knn_iters, s, self.tau, self.budget, seed)
        if not self.h:
            raise RuntimeError("oracle compression failed")
        self.L = 1 << self.depth
        self.nnodes = 1 << (self.depth + 1)
        self.start, self.size = tree_ranges(self.n, self.depth)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_free(self.h)
            self.h = None

    # ---- structure -------------------------------------------------------
    def perm(self):
        p = np.zeros(self.n, np.int32)
        lib().orc_get_perm(self.h, _ptr(p))
        return p

    def knn(self):
        idx = np.zeros((self.n, self.k), np.int32)
        d2 = np.zeros((self.n, self.k), np.float64)
        lib().orc_get_knn(self.h, _ptr(idx), _ptr(d2))
        return idx, d2

    def near(self):
        nnz = lib().orc_near_nnz(self.h)
        off = np.zeros(self.L + 1, np.int32)
        idx = np.zeros(max(nnz, 1), np.int32)
        lib().orc_get_near(self.h, _ptr(off), _ptr(idx))
        return off, idx[:nnz]

    def far(self):
        nnz = lib().orc_far_nnz(self.h)
        off = np.zeros(self.nnodes + 1, np.int32)
        idx = np.zeros(max(nnz, 1), np.int32)
        lib().orc_get_far(self.h, _ptr(off), _ptr(idx))
        return off, idx[:nnz]

    def ranks(self):
        r = np.zeros(self.nnodes, np.int32)
        c = np.zeros(self.nnodes, np.int32)
        nr = np.zeros(self.nnodes, np.int32)
        lib().orc_get_ranks(self.h, _ptr(r), _ptr(c), _ptr(nr))
        return r, c, nr

    def node(self, h):
        """(skeleton indices, sampled row indices, P [rank x ncand]) of heap node h."""
        r, c, nr = self.ranks()
        skel = np.zeros(max(r[h], 1), np.int32)
        rows = np.zeros(max(nr[h], 1), np.int32)
        P = np.zeros(max(r[h] * c[h], 1), np.float64)
        lib().orc_get_node(self.h, h, _ptr(skel), _ptr(rows), _ptr(P))
        return skel[:r[h]], rows[:nr[h]], P[:r[h] * c[h]].reshape(r[h], c[h])

    def trace(self, h):
        """Pivot trace of heap node h's ID: per examined step the largest and the
        second largest remaining column norm (-1: no second column)."""
        tr = np.zeros(2 * (self.s + 1), np.float64)
        ns = lib().orc_get_trace(self.h, h, _ptr(tr))
        return tr[:2 * ns].reshape(-1, 2)

    def candidates(self, h):
        """Candidate columns of heap node h (points of a leaf, children's skeletons otherwise)."""
        if h >= self.L:
            p = self.perm()
            return p[self.start[h]:self.start[h] + self.size[h]].copy()
        return np.concatenate([self.node(2 * h)[0], self.node(2 * h + 1)[0]])

    # ---- products ----------------------------------------------------------
    def matvec(self, w):
        """u = K~ w in float64; w of shape (n,) or (n, nrhs)."""
        w = np.asarray(w, dtype=np.float64)
        vec = w.ndim == 1
        W = np.asfortranarray(w.reshape(self.n, -1))
        U = np.zeros_like(W, order="F")
        if lib().orc_hmatvec(self.h, _ptr(W), _ptr(U), W.shape[1]):
            raise RuntimeError("oracle hmatvec failed")
        return U[:, 0] if vec else U

    def matvec_abs(self, w):
        """|K~| |w| in float64 (every factor of the product by its magnitude)."""
        w = np.asarray(w, dtype=np.float64)
        vec = w.ndim == 1
        W = np.asfortranarray(w.reshape(self.n, -1))
        U = np.zeros_like(W, order="F")
        if lib().orc_hmatvec_abs(self.h, _ptr(W), _ptr(U), W.shape[1]):
            raise RuntimeError("oracle hmatvec failed")
        return U[:, 0] if vec else U

    def kernel(self, i, j):
        return lib().orc_kernel(_ptr(self.X), self.n, self.dim, self.is_u8, self.eps, int(i), int(j))


def dense_kmatvec(X, eps, w, rows=None):
    """Rows of u = K w for the exact Gaussian kernel of Eq. (2), evaluated on the fly.

    ``rows``: None for all rows, or (r0, r1).  w of shape (n,) or (n, nrhs).
    """
    Xc, is_u8 = _points(X)
    n, dim = Xc.shape
    w = np.asarray(w, dtype=np.float64)
    vec = w.ndim == 1
    W = np.asfortranarray(w.reshape(n, -1))
    r0, r1 = (0, n) if rows is None else rows
    U = np.zeros((r1 - r0, W.shape[1]), order="F")
    lib().orc_dense_kmatvec(_ptr(Xc), n, dim, is_u8, float(eps), _ptr(W), W.shape[1], _ptr(U), r0, r1)
    return U[:, 0] if vec else U


def dense_sqdist_rows(X, r0, r1):
    Xc, is_u8 = _points(X)
    n, dim = Xc.shape
    out = np.zeros((r1 - r0, n), np.float64)
    lib().orc_dense_sqdist(_ptr(Xc), n, dim, is_u8, r0, r1, _ptr(out))
    return out
