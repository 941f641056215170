"""Pins of the oracle's hierarchical approximation (Eq. (3)) and its compression steps.

Structural invariants, special cases that reduce to the dense product or to a
library routine, brute force on small inputs, and published known-answer values.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sl

import synth
from oracle import dense as D
from oracle import diffusion as DF


# ---------------------------------------------------------------- generator
@pytest.mark.parametrize("ctr,key,want", [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
])
def test_philox_known_answers(orc, ctr, key, want):
    # Known-answer vectors published with Random123 (Salmon et al., SC'11).
    assert tuple(int(x) for x in orc.philox4x32_10(ctr, key)) == want


# ---------------------------------------------------------------- fixtures
@pytest.fixture(scope="module")
def c1(orc):
    cfg = synth.get_config("scurve-2k")
    X, eps = synth.configs.make_inputs(cfg)
    H = orc.HMatrix(X, eps, cfg["m"], cfg["s"], cfg["tau"], cfg["k"], cfg["seed"])
    return X, eps, cfg, H


# ---------------------------------------------------------------- tree
def test_tree_is_a_balanced_bijection(c1):
    X, eps, cfg, H = c1
    perm = H.perm()
    assert np.array_equal(np.sort(perm), np.arange(H.n))
    for h in range(1, H.L):
        assert H.size[2 * h] == H.size[h] // 2
        assert H.size[2 * h + 1] == H.size[h] - H.size[h] // 2
    for h in range(H.L, 2 * H.L):  # leaves keep ascending original index
        seg = perm[H.start[h]:H.start[h] + H.size[h]]
        assert np.all(np.diff(seg) > 0)


def test_tree_on_a_line_cuts_intervals(orc):
    # On 1-D data the kernel-space ball split separates the points nearer one
    # end of the node from those nearer the other: every node is an interval.
    rng = np.random.default_rng(3)
    x = np.sort(rng.uniform(0, 1, 1000))[rng.permutation(1000)][:, None]
    eps = synth.median_sq_dist_eps(x, 0)
    H = orc.HMatrix(x, eps, 64, 8, 1e-3, 8, 7)
    perm = H.perm()
    rank_of = np.argsort(np.argsort(x[:, 0]))
    for h in range(2, 2 * H.L):
        r = np.sort(rank_of[perm[H.start[h]:H.start[h] + H.size[h]]])
        assert r[-1] - r[0] + 1 == r.size


# ---------------------------------------------------------------- kNN
def _brute_knn(X, k):
    Dm = D.sq_dists(X)
    n = X.shape[0]
    idx = np.zeros((n, k), np.int64)
    d2 = np.zeros((n, k))
    for i in range(n):
        cand = np.delete(np.arange(n), i)
        o = np.lexsort((cand, Dm[i, cand]))[:k]
        idx[i], d2[i] = cand[o], Dm[i, cand[o]]
    return idx, d2


def test_knn_single_leaf_is_exact(orc):
    # With one leaf (depth 0) every pair is compared: the lists equal brute force.
    X, _ = synth.s_curve(300, 21)
    H = orc.HMatrix(X, 1.0, 512, 8, 1e-3, 12, 1, depth=0)
    idx, d2 = H.knn()
    bi, bd = _brute_knn(X, 12)
    assert np.array_equal(idx, bi)
    assert np.array_equal(d2, bd)


def test_knn_single_leaf_exact_u8(orc):
    X, _ = synth.mnist_shaped(200, 22, dim=40)
    H = orc.HMatrix(X, 50.0, 512, 8, 1e-3, 10, 1, depth=0)
    idx, d2 = H.knn()
    bi, bd = _brute_knn(X, 10)
    assert np.array_equal(idx, bi)
    assert np.array_equal(d2, bd)


def test_knn_lists_are_valid_and_recall_high(c1):
    X, eps, cfg, H = c1
    idx, d2 = H.knn()
    Dm = D.sq_dists(X)
    rows = np.arange(H.n)[:, None]
    assert np.all(idx >= 0) and np.all(idx != rows)
    assert np.array_equal(d2, Dm[rows, idx])
    assert all(len(set(r)) == r.size for r in idx)
    assert np.all((np.diff(d2, axis=1) > 0) | ((np.diff(d2, axis=1) == 0) & (np.diff(idx, axis=1) > 0)))
    bi, _ = _brute_knn(X[:512], 1)  # cheap spot check on a subset's geometry
    assert bi.shape == (512, 1)
    exact = np.argsort(np.where(np.eye(H.n, dtype=bool), np.inf, Dm), axis=1, kind="stable")[:, :cfg["k"]]
    recall = np.mean([np.intersect1d(idx[i], exact[i]).size for i in range(H.n)]) / cfg["k"]
    assert recall >= 0.9


# ---------------------------------------------------------------- lists
def _covered_once(H):
    off, idx = H.near()
    foff, fidx = H.far()
    L = H.L
    cover = np.zeros((L, L), np.int64)
    for a in range(L):
        for b in idx[off[a]:off[a + 1]]:
            cover[a, b] += 1
    for h in range(1, H.nnodes):
        lvl = int(np.log2(h))
        sh = H.depth - lvl
        for g in fidx[foff[h]:foff[h + 1]]:
            cover[(h << sh) - L:((h + 1) << sh) - L, (g << sh) - L:((g + 1) << sh) - L] += 1
    return cover


def test_near_far_partition_every_leaf_pair(c1):
    X, eps, cfg, H = c1
    off, idx = H.near()
    L = H.L
    rel = np.zeros((L, L), bool)
    for a in range(L):
        rel[a, idx[off[a]:off[a + 1]]] = True
    assert rel.diagonal().all() and np.array_equal(rel, rel.T)
    assert np.all(_covered_once(H) == 1)


def test_hss_mode_far_is_sibling(orc):
    X, _ = synth.s_curve(1024, 2)
    H = orc.HMatrix(X, 4.0, 128, 32, 1e-5, 16, 1, budget=0.0)
    foff, fidx = H.far()
    for h in range(2, H.nnodes):
        assert list(fidx[foff[h]:foff[h + 1]]) == [h ^ 1]


# ---------------------------------------------------------------- ID
def test_interpolative_decomposition_against_lapack(c1):
    # The pivots of QR with column pivoting are those of LAPACK's GEQP3 and the
    # rank follows |R_jj| > tau |R_11|; P reproduces the skeleton columns exactly.
    X, eps, cfg, H = c1
    W = D.kernel_matrix(X, eps)
    ranks, ncand, nrows = H.ranks()
    for h in [2, 5, 9, H.L, H.L + 7, 2 * H.L - 1]:
        skel, rows, P = H.node(h)
        cand = H.candidates(h)
        B = W[np.ix_(rows, cand)]
        Q, R, piv = sl.qr(B, mode="economic", pivoting=True)
        dr = np.abs(np.diag(R))
        r = min(cfg["s"], int(np.sum(dr > cfg["tau"] * dr[0])))
        assert r == ranks[h]
        assert np.array_equal(skel, cand[piv[:r]])
        pos = {c: i for i, c in enumerate(cand)}
        sp = [pos[c] for c in skel]
        np.testing.assert_array_equal(P[:, sp], np.eye(r))
        res = np.linalg.norm(B - B[:, sp] @ P)
        bound = np.sqrt(max(B.shape[1] - r, 1)) * (dr[r] if r < dr.size else 0.0)
        assert res <= 1.0001 * bound + 1e-13 * np.linalg.norm(B)


# ---------------------------------------------------------------- products
def test_no_compression_is_exact(orc):
    # tau = 0 and s = n/2: every ID keeps all of its candidates, so K~ = K.
    X, _ = synth.s_curve(512, 4)
    eps = synth.median_sq_dist_eps(X, 4)
    H = orc.HMatrix(X, eps, 64, 256, 0.0, 16, 4)
    r, c, nr = H.ranks()
    assert np.array_equal(r[2:], c[2:])
    W = D.kernel_matrix(X, eps)
    w = np.random.default_rng(0).standard_normal((H.n, 2))
    np.testing.assert_allclose(H.matvec(w), W @ w, rtol=0, atol=1e-11 * np.abs(W @ w).max())


def test_all_near_is_exact(orc):
    # budget = 1: every leaf is near every leaf, the far field is empty.
    X, _ = synth.s_curve(1024, 5)
    eps = synth.median_sq_dist_eps(X, 5)
    H = orc.HMatrix(X, eps, 128, 16, 1e-3, 16, 5, budget=1.0)
    assert H.far()[0][-1] == 0
    W = D.kernel_matrix(X, eps)
    w = np.random.default_rng(1).standard_normal(H.n)
    np.testing.assert_allclose(H.matvec(w), W @ w, rtol=0, atol=1e-12 * np.abs(W @ w).max())


def test_hmatrix_is_symmetric(c1):
    X, eps, cfg, H = c1
    rng = np.random.default_rng(2)
    x, y = rng.standard_normal(H.n), rng.standard_normal(H.n)
    a, b = x @ H.matvec(y), y @ H.matvec(x)
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))


def test_compression_error_within_ten_tau(c1):
    # Eq. (1) with the 2-norm of K~ w - K w over three Gaussian w
    # (empirical: the paper states no bound for the compression).
    X, eps, cfg, H = c1
    W = D.kernel_matrix(X, eps)
    rng = np.random.default_rng(3)
    for _ in range(3):
        w = rng.standard_normal(H.n)
        u = W @ w
        assert np.linalg.norm(H.matvec(w) - u) / np.linalg.norm(u) <= 10 * cfg["tau"]


def test_normalised_hmatrix_top_eigenpair(c1):
    # Degrees taken from K~ itself: lambda_1(S~) = 1, phi_1 = sqrt(d~) / ||sqrt(d~)||.
    X, eps, cfg, H = c1
    th, ph, info = DF.eigs(H.matvec, H.n, 3, tol=1e-12)
    assert abs(th[0] - 1) < 1e-12
    want = np.sqrt(info["d"]) / np.linalg.norm(np.sqrt(info["d"]))
    assert np.linalg.norm(np.abs(ph[:, 0]) - want) < 1e-8


def test_dense_rows_match_numpy(orc, c1):
    X, eps, cfg, H = c1
    W = D.kernel_matrix(X, eps)
    w = np.random.default_rng(4).standard_normal(H.n)
    u = W @ w
    np.testing.assert_allclose(orc.dense_kmatvec(X, eps, w, (100, 300)), u[100:300], rtol=0,
                               atol=1e-13 * np.abs(u).max())


# ---------------------------------------------------------------- |K~| |w|
def test_abs_product_without_compression_is_kernel_times_abs(orc):
    # tau = 0, s = n/2: every P is a column selection (entries 0 and 1), so the
    # magnitude product through the tree is K |w|.
    X, _ = synth.s_curve(512, 4)
    eps = synth.median_sq_dist_eps(X, 4)
    H = orc.HMatrix(X, eps, 64, 256, 0.0, 16, 4)
    W = D.kernel_matrix(X, eps)
    w = np.random.default_rng(5).standard_normal(H.n)
    np.testing.assert_allclose(H.matvec_abs(w), W @ np.abs(w), rtol=1e-12)


def test_abs_product_bounds_every_row(orc, c1):
    # |(K~ w)_i| <= (|K~| |w|)_i for every w (triangle inequality), with equality
    # when w >= 0 and no P entry is negative on the row's paths; and |K~||w| >= K~|w|.
    X, eps, cfg, H = c1
    rng = np.random.default_rng(6)
    w = rng.standard_normal((H.n, 2))
    u, a = H.matvec(w), H.matvec_abs(w)
    assert np.all(np.abs(u) <= a * (1 + 1e-12))
    assert np.all(H.matvec(np.abs(w)) <= a * (1 + 1e-12))
    # the near blocks alone (budget 1) have no P: |K~||w| = K |w|
    Hn = orc.HMatrix(X, eps, cfg["m"], cfg["s"], cfg["tau"], cfg["k"], cfg["seed"], budget=1.0)
    Wk = D.kernel_matrix(X, eps)
    np.testing.assert_allclose(Hn.matvec_abs(w[:, 0]), Wk @ np.abs(w[:, 0]), rtol=1e-12)


# ---------------------------------------------------------------- sampling steps
def _floyd(orc, seed, node, n, ns):
    """Floyd's algorithm written out: for j = n - ns .. n - 1 draw t uniform in
    [0, j]; take t unless already taken, else j.  One Philox draw (purpose 1,
    counter (j, node, 0)) per step, mapped to [0, j] by multiply-shift."""
    chosen = []
    for j in range(n - ns, n):
        t = (orc.rand_u32(seed, 1, node, 0, j) * (j + 1)) >> 32
        chosen.append(j if t in chosen else t)
    return sorted(chosen)


@pytest.mark.parametrize("seed,node,n", [(0, 1, 2048), (3, 17, 65), (9, 5, 1000), (1, 2, 64)])
def test_sample_positions_is_floyd(orc, seed, node, n):
    ns = min(n, 64)
    got = orc.sample_positions(seed, node, n, ns)
    assert got.size == ns
    assert np.all((got >= 0) & (got < n)) and np.all(np.diff(got) > 0)
    assert list(got) == _floyd(orc, seed, node, n, ns)


def _near_brute(H):
    """Votes of leaf a for leaf b: neighbours of a's points that sit in b.  Each
    leaf keeps itself and the ceil(budget L) others with most votes (ties: lower
    leaf id); the relation is then made symmetric."""
    L = H.L
    perm = H.perm()
    iperm = np.empty_like(perm)
    iperm[perm] = np.arange(H.n)
    leaf_of_pos = np.searchsorted(H.start[L:2 * L], np.arange(H.n), side="right") - 1
    idx, _ = H.knn()
    votes = np.zeros((L, L), np.int64)
    for pos in range(H.n):
        for j in idx[perm[pos]]:
            if j >= 0:
                votes[leaf_of_pos[pos], leaf_of_pos[iperm[j]]] += 1
    extra = int(np.ceil(H.budget * L))
    rel = np.eye(L, dtype=bool)
    for a in range(L):
        others = [b for b in range(L) if b != a]
        others.sort(key=lambda b: (-votes[a, b], b))
        rel[a, others[:extra]] = True
    rel = rel | rel.T
    off = np.concatenate([[0], np.cumsum(rel.sum(axis=1))]).astype(np.int32)
    return off, np.nonzero(rel)[1].astype(np.int32)


@pytest.mark.parametrize("budget", [0.05, 0.2])
def test_near_lists_from_vote_matrix(orc, budget):
    X, _ = synth.s_curve(2048, 0)
    eps = synth.median_sq_dist_eps(X, 0)
    H = orc.HMatrix(X, eps, 64, 16, 1e-5, 16, 0, budget=budget)
    off, idx = H.near()
    boff, bidx = _near_brute(H)
    assert np.array_equal(off, boff)
    assert np.array_equal(idx, bidx)


def _rows_brute(orc, H, h):
    """Sampled rows of node h, written out: the candidates' neighbours outside h
    ranked by (votes desc, index asc), the first min(count, want // 2) kept, where
    want = min(n - |h|, 2 s); then every outside point in index order when
    want = n - |h|, else uniform Philox draws (purpose 3, counter (t, h, 0)) from
    outside h, skipping repeats, until want rows are taken."""
    perm = H.perm()
    iperm = np.empty_like(perm)
    iperm[perm] = np.arange(H.n)
    lo, hi = H.start[h], H.start[h] + H.size[h]
    inside = lambda i: lo <= iperm[i] < hi  # noqa: E731
    want = min(H.n - H.size[h], 2 * H.s)
    idx, _ = H.knn()
    votes = {}
    for c in H.candidates(h):
        for i in idx[c]:
            if i >= 0 and not inside(i):
                votes[i] = votes.get(i, 0) + 1
    ranked = sorted(votes, key=lambda i: (-votes[i], i))
    rows = ranked[:want // 2]
    taken = set(rows)
    if len(rows) < want:
        if want == H.n - H.size[h]:
            rows += [i for i in range(H.n) if not inside(i) and i not in taken][:want - len(rows)]
        else:
            t = 0
            while len(rows) < want:
                i = (orc.rand_u32(H.seed, 3, h, 0, t) * H.n) >> 32
                t += 1
                if inside(i) or i in taken:
                    continue
                rows.append(i)
                taken.add(i)
    return np.array(rows, np.int32)


@pytest.mark.parametrize("n,m,s", [(2048, 128, 64), (300, 64, 128)])
def test_sampled_rows_brute_force(orc, n, m, s):
    # (300, 64, 128): 2 s exceeds the points outside the upper nodes, so they take every outside point
    X, _ = synth.s_curve(n, 8)
    eps = synth.median_sq_dist_eps(X, 8)
    H = orc.HMatrix(X, eps, m, s, 1e-5, 16, 8)
    perm = H.perm()
    iperm = np.empty_like(perm)
    iperm[perm] = np.arange(H.n)
    for h in range(2, H.nnodes):
        rows = H.node(h)[1]
        assert rows.size == min(H.n - H.size[h], 2 * s)
        assert np.unique(rows).size == rows.size
        pos = iperm[rows]
        assert np.all((pos < H.start[h]) | (pos >= H.start[h] + H.size[h]))
        assert np.array_equal(rows, _rows_brute(orc, H, h)), h


def test_pivot_trace_matches_column_norms(orc, c1):
    # The first recorded pair is the largest and second largest column norm of B;
    # each recorded largest is |R_jj| of LAPACK's pivoted QR.
    X, eps, cfg, H = c1
    W = D.kernel_matrix(X, eps)
    for h in [3, H.L + 2]:
        skel, rows, P = H.node(h)
        B = W[np.ix_(rows, H.candidates(h))]
        tr = H.trace(h)
        cn = np.sort(np.linalg.norm(B, axis=0))[::-1]
        np.testing.assert_allclose(tr[0], cn[:2], rtol=1e-13)
        _, R, _ = sl.qr(B, mode="economic", pivoting=True)
        k = tr.shape[0]
        np.testing.assert_allclose(tr[:, 0], np.abs(np.diag(R))[:k], rtol=1e-9)
        # the block routine on the same B (numpy's exp may differ from the C
        # library's in the last bit, so the traces agree to rounding)
        rk, cp, P1, tr1 = orc.pivoted_id(B, cfg["s"], cfg["tau"])
        assert rk == P.shape[0]
        np.testing.assert_allclose(tr1, tr, rtol=1e-12, atol=1e-14 * tr[0, 0])


def test_deterministic_exponential_within_two_ulp(orc):
    """The compression's exponential (Cody-Waite reduction of x = n ln2 + r, Taylor
    polynomial of degree 13 on |r| <= ln2/2) against the C library's exp and, at a
    few points, against e^x to 60 digits: within 2 ulp over the arguments the kernel
    values take ([-745, 0]); exact at 0; 0 below the subnormal range; monotone."""
    from decimal import Decimal, getcontext
    rng = np.random.default_rng(5)
    xs = np.concatenate([-rng.exponential(3.0, 20000), -rng.uniform(0, 745, 20000),
                         -np.linspace(0, 1e-3, 2001), np.array([-708.4, -709.0, -720.0, -740.0, -745.0])])
    worst = 0.0
    for x in xs:
        got = orc.det_exp(x)
        ref = math.exp(x)
        ulp = math.ulp(ref) if ref > 0 else math.ulp(0.0)
        worst = max(worst, abs(got - ref) / ulp)
    assert worst <= 2.0, worst
    getcontext().prec = 60
    for x in (-0.3465, -1.0, -10.5, -100.25, -700.0):
        ref = float(Decimal(x).exp())
        assert abs(orc.det_exp(x) - ref) <= 2 * math.ulp(ref)
    assert orc.det_exp(0.0) == 1.0
    assert orc.det_exp(-745.3) == 0.0 and orc.det_exp(-1e6) == 0.0
    g = np.array([orc.det_exp(x) for x in np.linspace(-30.0, 0.0, 30001)])
    assert np.all(np.diff(g) >= 0.0)
