"""Comparison rules shared by the GPU parity tests (imported by tests only).

Skeletons (Sec. 2.1, the low-rank part UV of Eq. (3)).  The interpolative
decomposition takes its pivots from column norms and its rank from
|R_jj| > tau |R_11|.  The paper fixes no summation order for those norms and
inner products, so two correct implementations agree on a pivot unless the two
largest remaining column norms lie within their rounding error, and on the rank
unless |R_jj| lies within it of tau |R_11|.  The rounding error of step j of
Householder QR on an nr-row block is bounded by a multiple of nr (j + 1) u times
the largest column norm of the block, which is R_11 (backward stability of
Householder QR; Higham, Accuracy and Stability of Numerical Algorithms, 2nd ed.,
Thm. 19.4 with its constant taken as 8):

    delta_j = 8 nr (j + 1) u R_11,   u = 2^-53.

A node whose GPU skeleton differs from the oracle's is accepted only at such a
near tie (the oracle records the two largest norms of every step); its
ancestors then see other candidates and are not compared.  Where the pivots
agree, P must agree to 1e-10 relative to max(1, max |P|).

Products (Eq. (3)).  Every entry of u = K~ w is compared with the oracle's
float64 product against the row-wise magnitude product a = |K~| |w| (the
oracle's matvec_abs): each term of u_i enters with its magnitude, so a rounding
of relative size e anywhere in a term moves u_i by at most e a_i, and a sum of T
terms in any order adds at most gamma_T = T v / (1 - T v) times a_i (v the unit
roundoff of the accumulation; Higham, Lemma 3.1 and Sec. 4.2).
"""
from __future__ import annotations

import numpy as np

U64 = 2.0 ** -53
U32 = 2.0 ** -24

# unit roundoff of the tile formats (values scaled into (0, 1])
TILE_U = {"f64": U64, "f32": U32, "bf16": 2.0 ** -8, "f16": 2.0 ** -11}
# accumulation and vector unit roundoff of each path; the float16 path stages the
# vector as a power-of-two scale times a float16 hi + lo pair (about 22 bits)
VEC_U = {"f64": U64, "f32": U32, "bf16": U32, "f16": 2.0 ** -21}
# float16 tiles: entries below the normal range keep an absolute error of half
# the smallest subnormal (times the tile scale, at most 1)
TILE_ABS = {"f64": 0.0, "f32": 0.0, "bf16": 0.0, "f16": 2.0 ** -25}
# the interpolation matrices of two correct IDs differ by up to 1e-10 (relative),
# which moves a product by a few 1e-15 in practice; allowed per entry for float64
ID_ALLOWANCE = 1e-12


def id_delta(nr: int, j: int, r11: float) -> float:
    return 8.0 * nr * (j + 1) * U64 * r11


def check_skeletons(op, H, s: int, tau: float, p_tol: float = 1e-10):
    """Node-by-node comparison of ranks, sampled rows, skeletons and P, bottom-up.

    Returns (compared, near_ties, max_p_dev).  Raises AssertionError on any
    difference that the near-tie rule does not allow.
    """
    r_o, c_o, nr_o = H.ranks()
    r_g, c_g, nr_g = op.ranks()
    diverged = set()
    compared, ties, pmax = 0, 0, 0.0
    for lvl in range(H.depth, 0, -1):
        for h in range(1 << lvl, 2 << lvl):
            if lvl < H.depth and (2 * h in diverged or 2 * h + 1 in diverged):
                diverged.add(h)   # its candidates come from a legitimately different child
                continue
            assert c_g[h] == c_o[h] and nr_g[h] == nr_o[h], h
            gs, grows, gP = op.node(h)
            os_, orows, oP = H.node(h)
            assert np.array_equal(grows, orows), f"sampled rows of node {h}"
            compared += 1
            if r_g[h] == r_o[h] and np.array_equal(gs, os_):
                if oP.size:
                    dev = np.max(np.abs(gP - oP)) / max(1.0, np.max(np.abs(oP)))
                    pmax = max(pmax, dev)
                    assert dev <= p_tol, (h, dev)
                continue
            tr = H.trace(h)
            r11 = tr[0, 0]
            kmin = min(r_g[h], r_o[h])
            k = next((j for j in range(kmin) if gs[j] != os_[j]), kmin)
            d = id_delta(int(nr_o[h]), k, r11)
            if k < kmin:   # a different pivot at step k
                assert tr[k, 1] >= 0 and tr[k, 0] - tr[k, 1] <= d, (h, k, tr[k], d)
            else:          # a different rank: the stopping test at step k
                assert k < tr.shape[0] and abs(tr[k, 0] - tau * r11) <= d, (h, k, r_g[h], r_o[h])
            ties += 1
            diverged.add(h)
    return compared, ties, pmax


def product_terms(H, s: int) -> np.ndarray:
    """Per point, an upper bound on the number of terms its entry of K~ w sums:
    the points of its near leaves plus, along its path, the far columns and the
    interpolation columns (at most 2 s per node and direction)."""
    L = H.L
    off, idx = H.near()
    foff, fidx = H.far()
    r, c, _ = H.ranks()
    perm = H.perm()
    T = np.zeros(H.n, np.int64)
    for a in range(L):
        near_pts = int(sum(H.size[L + b] for b in idx[off[a]:off[a + 1]]))
        path = 0
        h = L + a
        while h >= 2:
            path += int(sum(r[g] for g in fidx[foff[h]:foff[h + 1]])) + 2 * int(c[h]) + 2 * s
            h //= 2
        T[perm[H.start[L + a]:H.start[L + a] + H.size[L + a]]] = near_pts + path
    return T


def product_bound(H, w: np.ndarray, prec: str, far_prec: str | None = None, s: int | None = None) -> np.ndarray:
    """Entry-wise bound on |u - K~ w| for a product in the given tile precision."""
    s = H.s if s is None else s
    far_prec = prec if far_prec is None else far_prec
    a = H.matvec_abs(w)
    T = product_terms(H, s).astype(np.float64)
    if a.ndim == 2:
        T = T[:, None]
    v = VEC_U[prec] if prec != "f64" else U64
    gamma = T * v / (1.0 - T * v)
    e = max(TILE_U[prec], TILE_U[far_prec]) + (2 * H.depth + 4) * v + gamma
    b = e * a
    if prec == "f64":
        b = b + ID_ALLOWANCE * a
    if TILE_ABS[prec] > 0.0:
        w1 = np.abs(w).sum(axis=0)
        b = b + TILE_ABS[prec] * w1
    return b


def check_product(u: np.ndarray, ref: np.ndarray, bound: np.ndarray, what: str = ""):
    """Assert |u_i - ref_i| <= bound_i for every entry; returns the largest ratio."""
    err = np.abs(u - ref)
    ratio = err / bound
    worst = float(np.max(ratio))
    i = np.unravel_index(int(np.argmax(ratio)), ratio.shape)
    assert worst <= 1.0, f"{what}: entry {i} off by {err[i]:.3e} > bound {bound[i]:.3e}"
    return worst


def structure_digests(op) -> dict:
    """SHA-256 of each structure array of an operator (oracle or GPU: anything with
    perm(), knn(), near(), far(), ranks() and node(h)), little-endian, in a fixed
    layout: the tree permutation, neighbour indices and squared distances, the near
    and far CSR lists, ranks | candidates | sampled rows per heap id from 2 on, and
    the skeletons of heap ids 2, 3, ... concatenated."""
    import hashlib

    def sha(*arrays):
        h = hashlib.sha256()
        for a in arrays:
            a = np.ascontiguousarray(a)
            h.update(a.astype(a.dtype.newbyteorder("<"), copy=False).tobytes())
        return h.hexdigest()

    idx, d2 = op.knn()
    r, c, nr = op.ranks()
    nn = len(r)
    return {
        "perm": sha(np.asarray(op.perm(), np.int32)),
        "knn_idx": sha(np.asarray(idx, np.int32)),
        "knn_d2": sha(np.asarray(d2, np.float64)),
        "near": sha(*[np.asarray(a, np.int32) for a in op.near()]),
        "far": sha(*[np.asarray(a, np.int32) for a in op.far()]),
        "ranks": sha(np.asarray(r[2:], np.int32), np.asarray(c[2:], np.int32), np.asarray(nr[2:], np.int32)),
        "skeletons": sha(*[np.asarray(op.node(h)[0], np.int32) for h in range(2, nn)]),
    }
