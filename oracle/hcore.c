/*
 * ORACLE -- test infrastructure only.  Only tests/, __graft_entry__.smoke() and
 * bench.py's cpu_baseline leg may load this code.  It shares nothing with the
 * HIP library: no headers, helpers, tables or generators.
 *
 * Plain, sequential, float64 CPU implementation of the hierarchical (H-matrix)
 * approximation K~ = D + S + UV of a Gaussian kernel matrix (Eq. (3), Sec. 2.1
 * "Hierarchical partitioning") and of its matrix-vector product, which the
 * Lanczos iteration calls once per step (Sec. 1.2: compressed once, evaluated in
 * every iteration; Sec. 3 integration through a matvec operator).
 *
 * The paper treats the compression (GOFMM) as a black box: geometry-oblivious,
 * O(N log N), a user tolerance (Eq. (1)) and the parameters leaf size, maximal
 * off-diagonal rank, tolerance and neighbour count (Sec. 4.2.3).  The concrete
 * steps below -- kernel-distance ball tree, randomized-tree nearest neighbours,
 * neighbour-voted near lists, dual-tree far lists, sampled-row interpolative
 * decomposition with nested skeletons -- are the readings written down in the
 * design notes; every decision is taken with a total order (value, index) so the
 * result is unique.
 *
 * Compile with -ffp-contract=off: every product and sum below is one IEEE
 * operation, evaluated in the order written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11).  */
/* ------------------------------------------------------------------------- */
static void philox_round(uint32_t c[4], const uint32_t k[2]) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0];
    const uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    memcpy(out, c, sizeof(c));
}

/* One 32-bit draw for (seed, purpose, a, b, i): counter (i, a, b, purpose),
 * key (low and high half of the seed); the first output word. */
uint32_t orc_rand_u32(uint64_t seed, uint32_t purpose, uint32_t a, uint32_t b, uint32_t i) {
    const uint32_t ctr[4] = {i, a, b, purpose};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[0];
}

/* integer in [0, bound) from one draw (multiply-shift) */
static uint32_t uniform_below(uint32_t r, uint32_t bound) {
    return (uint32_t)(((uint64_t)r * (uint64_t)bound) >> 32);
}

enum { PURPOSE_TREE = 1, PURPOSE_KNN = 2, PURPOSE_ROWS = 3, PURPOSE_LANCZOS = 4 };

/* ------------------------------------------------------------------------- */
/* Points, squared distances and the Gaussian kernel of Eq. (2).              */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t n;
    int dim;
    int is_u8;          /* 1: u8 codes k standing for k/255; 0: float64 */
    const double *xf;   /* n x dim row-major (is_u8 == 0) */
    const uint8_t *xu;  /* n x dim row-major (is_u8 == 1) */
    double eps;         /* sigma^2 in Eq. (2) */
} orc_points;

/* ||x_i - x_j||^2, summed over coordinates in increasing order */
static double sqd(const orc_points *P, int64_t i, int64_t j) {
    if (P->is_u8) {
        const uint8_t *a = P->xu + i * P->dim, *b = P->xu + j * P->dim;
        int64_t acc = 0;
        for (int d = 0; d < P->dim; ++d) {
            const int64_t t = (int64_t)a[d] - (int64_t)b[d];
            acc += t * t;
        }
        return (double)acc / 65025.0;
    }
    const double *a = P->xf + i * P->dim, *b = P->xf + j * P->dim;
    double acc = 0.0;
    for (int d = 0; d < P->dim; ++d) {
        const double t = a[d] - b[d];
        acc = acc + t * t;
    }
    return acc;
}

/* ------------------------------------------------------------------------- */
/* The exponential of the compression's kernel values.  The tree, neighbour    */
/* and skeleton decisions are taken on kernel values, so the CPU build and the  */
/* device evaluate e^x by the same sequence of IEEE operations (a library exp   */
/* is correctly rounded on neither side): Cody and Waite's argument reduction   */
/* x = n ln2 + r (Cody & Waite, Software Manual for the Elementary Functions,   */
/* 1980), n = floor(x / ln2 + 1/2), ln2 split in a high part of 32 significant  */
/* bits (n times it is exact) and the rest; e^r by the Taylor polynomial of     */
/* degree 13 (|r| <= ln2 / 2: the omitted terms are below 1e-17 relative),      */
/* Horner with fused multiply-adds; then times 2^n, in two exact powers of two  */
/* when the result is subnormal.  Arguments <= -745.2 give 0 (e^x is below half */
/* the smallest subnormal).  Within 2 ulp of e^x (tests/test_oracle_hmatrix.py).*/
/* The constants are the doubles nearest to ln2's high part, ln2 - high, 1/ln2  */
/* and 1/k!, written as hexadecimal floats.                                     */
/* ------------------------------------------------------------------------- */
static const double EXP_LN2_HI = 0x1.62e42fee00000p-1;
static const double EXP_LN2_LO = 0x1.a39ef35793c76p-33;
static const double EXP_INV_LN2 = 0x1.71547652b82fep+0;
static const double EXP_INV_FACT[14] = {  /* 1/k!, k = 0..13 */
    1.0, 1.0, 0x1.0000000000000p-1, 0x1.5555555555555p-3, 0x1.5555555555555p-5, 0x1.1111111111111p-7,
    0x1.6c16c16c16c17p-10, 0x1.a01a01a01a01ap-13, 0x1.a01a01a01a01ap-16, 0x1.71de3a556c734p-19,
    0x1.27e4fb7789f5cp-22, 0x1.ae64567f544e4p-26, 0x1.1eed8eff8d898p-29, 0x1.6124613a86d09p-33};

double orc_det_exp(double x) {
    if (!(x > -745.2)) return 0.0;
    const double n = floor(x * EXP_INV_LN2 + 0.5);
    const double r = (x - n * EXP_LN2_HI) - n * EXP_LN2_LO;
    double p = EXP_INV_FACT[13];
    for (int k = 12; k >= 0; --k) p = fma(p, r, EXP_INV_FACT[k]);
    const int e = (int)n;
    if (e >= -1021) return p * ldexp(1.0, e);
    return (p * ldexp(1.0, e + 600)) * ldexp(1.0, -600);
}

/* Eq. (2): W_ij = exp(-||x_i - x_j||^2 / sigma^2), sigma^2 = eps; the compression's
 * values through orc_det_exp, the dense definitions through the C library's exp */
static double kval(const orc_points *P, int64_t i, int64_t j) {
    return orc_det_exp(-(sqd(P, i, j) / P->eps));
}
static double kval_libm(const orc_points *P, int64_t i, int64_t j) {
    return exp(-(sqd(P, i, j) / P->eps));
}

/* ------------------------------------------------------------------------- */
/* Perfect binary tree: heap ids (root 1, children 2h, 2h+1), left child takes  */
/* floor(n/2) points.                                                          */
/* ------------------------------------------------------------------------- */
static void tree_ranges(int64_t n, int depth, int64_t *start, int64_t *size) {
    start[1] = 0;
    size[1] = n;
    for (int64_t h = 1; h < ((int64_t)1 << depth); ++h) {
        const int64_t nl = size[h] / 2;
        start[2 * h] = start[h];
        size[2 * h] = nl;
        start[2 * h + 1] = start[h] + nl;
        size[2 * h + 1] = size[h] - nl;
    }
}

typedef struct {
    double key;
    int32_t idx;
} keyed;

static int cmp_keyed(const void *a, const void *b) {
    const keyed *x = (const keyed *)a, *y = (const keyed *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* Split pts[0..n) (ascending original index) into the floor(n/2) points with
 * the smallest (key, index) and the rest; both halves keep ascending index. */
static void split_by_key(int32_t *pts, int64_t n, const double *key, keyed *scratch, int32_t *tmp,
                         unsigned char *left) {
    for (int64_t i = 0; i < n; ++i) {
        scratch[i].key = key[i];
        scratch[i].idx = pts[i];
    }
    qsort(scratch, (size_t)n, sizeof(keyed), cmp_keyed);
    const int64_t nl = n / 2;
    /* membership by original index: mark the first nl of the sorted order */
    for (int64_t i = 0; i < n; ++i) left[i] = 0;
    /* pts is ascending, so a binary search finds each member's position */
    for (int64_t t = 0; t < nl; ++t) {
        int64_t lo = 0, hi = n - 1;
        const int32_t v = scratch[t].idx;
        while (lo < hi) {
            const int64_t mid = (lo + hi) / 2;
            if (pts[mid] < v) lo = mid + 1; else hi = mid;
        }
        left[lo] = 1;
    }
    int64_t a = 0, b = nl;
    for (int64_t i = 0; i < n; ++i) {
        if (left[i]) tmp[a++] = pts[i]; else tmp[b++] = pts[i];
    }
    memcpy(pts, tmp, (size_t)n * sizeof(int32_t));
}

/* Floyd's sampling of ns distinct positions out of [0, n), sorted ascending. */
static int sample_positions(uint64_t seed, uint32_t node, int64_t n, int ns, int64_t *out) {
    int cnt = 0;
    for (int64_t j = n - ns; j < n; ++j) {
        const int64_t t = uniform_below(orc_rand_u32(seed, PURPOSE_TREE, node, 0, (uint32_t)j),
                                        (uint32_t)(j + 1));
        int present = 0;
        for (int q = 0; q < cnt; ++q)
            if (out[q] == t) { present = 1; break; }
        out[cnt++] = present ? j : t;
    }
    /* insertion sort, ascending */
    for (int a = 1; a < cnt; ++a) {
        const int64_t v = out[a];
        int b = a - 1;
        while (b >= 0 && out[b] > v) { out[b + 1] = out[b]; --b; }
        out[b + 1] = v;
    }
    return cnt;
}

#define ORC_TREE_SAMPLE 64

/* Geometry-oblivious ball tree in kernel space.  For each node: p is the point
 * farthest (in the feature space of the kernel) from the centroid of a sample,
 * i.e. the smallest sum of kernel values to the sample; q is the point farthest
 * from p, i.e. the largest squared distance to p; the key K_iq - K_ip orders
 * points from the p side to the q side and the node is cut at its median. */
int orc_build_tree(const orc_points *P, int depth, uint64_t seed, int32_t *perm) {
    const int64_t n = P->n;
    const int64_t nn = (int64_t)1 << (depth + 1);
    int64_t *start = malloc(sizeof(int64_t) * nn), *size = malloc(sizeof(int64_t) * nn);
    double *key = malloc(sizeof(double) * n);
    keyed *scr = malloc(sizeof(keyed) * n);
    int32_t *tmp = malloc(sizeof(int32_t) * n);
    unsigned char *left = malloc(n);
    if (!start || !size || !key || !scr || !tmp || !left) return -1;
    tree_ranges(n, depth, start, size);
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    for (int64_t h = 1; h < ((int64_t)1 << depth); ++h) {
        int32_t *pts = perm + start[h];
        const int64_t m = size[h];
        int64_t samp[ORC_TREE_SAMPLE];
        int ns;
        if (m <= ORC_TREE_SAMPLE) {
            ns = (int)m;
            for (int q = 0; q < ns; ++q) samp[q] = q;
        } else {
            ns = sample_positions(seed, (uint32_t)h, m, ORC_TREE_SAMPLE, samp);
        }
        /* p = argmin_i sum_{j in sample} K_ij */
        int64_t p = 0;
        double best = INFINITY;
        for (int64_t i = 0; i < m; ++i) {
            double acc = 0.0;
            for (int q = 0; q < ns; ++q) acc = acc + kval(P, pts[i], pts[samp[q]]);
            if (acc < best) { best = acc; p = i; }
        }
        /* q = argmax_i ||x_i - x_p||^2 */
        int64_t q = 0;
        double far = -1.0;
        for (int64_t i = 0; i < m; ++i) {
            const double d = sqd(P, pts[i], pts[p]);
            if (d > far) { far = d; q = i; }
        }
        const int32_t ip = pts[p], iq = pts[q];
        for (int64_t i = 0; i < m; ++i) key[i] = kval(P, pts[i], iq) - kval(P, pts[i], ip);
        split_by_key(pts, m, key, scr, tmp, left);
    }
    free(start); free(size); free(key); free(scr); free(tmp); free(left);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Randomized-tree k nearest neighbours.                                       */
/* ------------------------------------------------------------------------- */
/* insert (d, j) into the ascending (d, idx) list of length k, no duplicates */
static void knn_insert(int32_t *li, double *ld, int k, double d, int32_t j) {
    if (d > ld[k - 1] || (d == ld[k - 1] && j >= li[k - 1] && li[k - 1] >= 0)) return;
    for (int t = 0; t < k; ++t)
        if (li[t] == j) return;
    int pos = k - 1;
    while (pos > 0 && (ld[pos - 1] > d || (ld[pos - 1] == d && (li[pos - 1] > j || li[pos - 1] < 0)))) {
        ld[pos] = ld[pos - 1];
        li[pos] = li[pos - 1];
        --pos;
    }
    ld[pos] = d;
    li[pos] = j;
}

/* T random projection trees of the same shape as the ball tree: each node cuts
 * at the median of ||x - x_p||^2 - ||x - x_q||^2 for two random members p != q;
 * inside every leaf all pairs are compared and each point keeps its k nearest
 * other points by (squared distance, index). */
int orc_knn(const orc_points *P, int depth, int k, int iters, uint64_t seed, int32_t *idx, double *d2) {
    const int64_t n = P->n;
    const int64_t nn = (int64_t)1 << (depth + 1);
    int64_t *start = malloc(sizeof(int64_t) * nn), *size = malloc(sizeof(int64_t) * nn);
    int32_t *perm = malloc(sizeof(int32_t) * n), *tmp = malloc(sizeof(int32_t) * n);
    double *key = malloc(sizeof(double) * n);
    keyed *scr = malloc(sizeof(keyed) * n);
    unsigned char *left = malloc(n);
    if (!start || !size || !perm || !tmp || !key || !scr || !left) return -1;
    tree_ranges(n, depth, start, size);
    for (int64_t i = 0; i < n * k; ++i) { idx[i] = -1; d2[i] = INFINITY; }
    for (int it = 0; it < iters; ++it) {
        for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
        for (int64_t h = 1; h < ((int64_t)1 << depth); ++h) {
            int32_t *pts = perm + start[h];
            const int64_t m = size[h];
            const uint32_t a = uniform_below(orc_rand_u32(seed, PURPOSE_KNN, (uint32_t)h, (uint32_t)it, 0), (uint32_t)m);
            uint32_t b = uniform_below(orc_rand_u32(seed, PURPOSE_KNN, (uint32_t)h, (uint32_t)it, 1), (uint32_t)(m - 1));
            if (b >= a) ++b;
            const int32_t ip = pts[a], iq = pts[b];
            for (int64_t i = 0; i < m; ++i) key[i] = sqd(P, pts[i], ip) - sqd(P, pts[i], iq);
            split_by_key(pts, m, key, scr, tmp, left);
        }
        for (int64_t h = (int64_t)1 << depth; h < nn; ++h) {
            const int32_t *pts = perm + start[h];
            const int64_t m = size[h];
            for (int64_t a = 0; a < m; ++a) {
                const int32_t i = pts[a];
                for (int64_t b = 0; b < m; ++b) {
                    if (a == b) continue;
                    knn_insert(idx + (int64_t)i * k, d2 + (int64_t)i * k, k, sqd(P, i, pts[b]), pts[b]);
                }
            }
        }
    }
    free(start); free(size); free(perm); free(tmp); free(key); free(scr); free(left);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* The compressed operator.                                                    */
/* ------------------------------------------------------------------------- */
typedef struct {
    orc_points P;
    int depth, k, s;
    double tau, budget;
    uint64_t seed;
    int64_t nnodes;          /* 2^(depth+1) heap slots (slot 0 unused) */
    int64_t *start, *size;   /* per heap id */
    int32_t *perm, *iperm;   /* tree position -> original index and back */
    int32_t *knn_idx;        /* n x k original indices */
    double *knn_d2;
    int32_t *near_off, *near_idx; /* CSR over leaves 0..L-1 (leaf id = heap id - L) */
    int32_t *far_off, *far_idx;   /* CSR over heap ids 0..nnodes-1 (heap ids) */
    int32_t *rank;           /* per heap id (levels >= 1) */
    int32_t **skel;          /* per heap id: rank original indices */
    int32_t *ncand;          /* per heap id: number of candidate columns */
    double **pmat;           /* per heap id: rank x ncand row-major */
    int32_t *nrows;          /* per heap id: sampled rows */
    int32_t **rows;          /* per heap id: original indices of the sampled rows */
    int32_t *nsteps;         /* per heap id: pivot steps the ID examined */
    double **trace;          /* per heap id: 2 x nsteps (largest, second largest remaining norm) */
} orc_h;

static int leaf_of_pos(const orc_h *H, int64_t pos) {
    const int64_t L = (int64_t)1 << H->depth;
    int64_t lo = 0, hi = L - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (H->start[L + mid] <= pos) lo = mid; else hi = mid - 1;
    }
    return (int)lo;
}

typedef struct { int32_t votes; int32_t id; } vote_ent;
static int cmp_votes(const void *a, const void *b) {
    const vote_ent *x = (const vote_ent *)a, *y = (const vote_ent *)b;
    if (x->votes != y->votes) return (x->votes < y->votes) - (x->votes > y->votes); /* desc */
    return (x->id > y->id) - (x->id < y->id);
}

/* Near lists (the sparse part S of Eq. (3) plus the diagonal blocks D): leaf a
 * keeps itself and the ceil(budget * L) other leaves that receive most of its
 * points' neighbour votes (ties, including zero votes: lower leaf id), then the
 * relation is symmetrised.  budget = 1 makes every leaf pair near. */
static int build_near(orc_h *H) {
    const int64_t L = (int64_t)1 << H->depth;
    int32_t *votes = calloc((size_t)(L * L), sizeof(int32_t));
    unsigned char *rel = calloc((size_t)(L * L), 1);
    vote_ent *ent = malloc(sizeof(vote_ent) * L);
    if (!votes || !rel || !ent) return -1;
    for (int64_t pos = 0; pos < H->P.n; ++pos) {
        const int a = leaf_of_pos(H, pos);
        const int32_t i = H->perm[pos];
        for (int t = 0; t < H->k; ++t) {
            const int32_t j = H->knn_idx[(int64_t)i * H->k + t];
            if (j < 0) continue;
            votes[a * L + leaf_of_pos(H, H->iperm[j])] += 1;
        }
    }
    const int64_t extra = (int64_t)ceil(H->budget * (double)L);
    for (int64_t a = 0; a < L; ++a) {
        rel[a * L + a] = 1;
        int cnt = 0;
        for (int64_t b = 0; b < L; ++b) {
            if (b == a) continue;
            ent[cnt].votes = votes[a * L + b];
            ent[cnt].id = (int32_t)b;
            ++cnt;
        }
        qsort(ent, (size_t)cnt, sizeof(vote_ent), cmp_votes);
        for (int64_t t = 0; t < extra && t < cnt; ++t) rel[a * L + ent[t].id] = 1;
    }
    for (int64_t a = 0; a < L; ++a)
        for (int64_t b = 0; b < L; ++b)
            if (rel[a * L + b]) rel[b * L + a] = 1;
    H->near_off = malloc(sizeof(int32_t) * (L + 1));
    int64_t tot = 0;
    for (int64_t a = 0; a < L * L; ++a) tot += rel[a];
    H->near_idx = malloc(sizeof(int32_t) * (tot > 0 ? tot : 1));
    int64_t c = 0;
    for (int64_t a = 0; a < L; ++a) {
        H->near_off[a] = (int32_t)c;
        for (int64_t b = 0; b < L; ++b)
            if (rel[a * L + b]) H->near_idx[c++] = (int32_t)b;
    }
    H->near_off[L] = (int32_t)c;
    free(votes); free(rel); free(ent);
    return 0;
}

/* does any leaf below heap node x have a near leaf below heap node y? */
static int near_related(const orc_h *H, int64_t x, int64_t y, int lvl) {
    const int64_t L = (int64_t)1 << H->depth;
    const int sh = H->depth - lvl;
    const int64_t xl = (x << sh) - L, xh = xl + ((int64_t)1 << sh);
    const int64_t yl = (y << sh) - L, yh = yl + ((int64_t)1 << sh);
    for (int64_t a = xl; a < xh; ++a)
        for (int32_t t = H->near_off[a]; t < H->near_off[a + 1]; ++t)
            if (H->near_idx[t] >= yl && H->near_idx[t] < yh) return 1;
    return 0;
}

typedef struct { int64_t *a, *b; int64_t n, cap; } pair_list;
static int push_pair(pair_list *pl, int64_t a, int64_t b) {
    if (pl->n == pl->cap) {
        pl->cap = pl->cap ? 2 * pl->cap : 1024;
        pl->a = realloc(pl->a, sizeof(int64_t) * pl->cap);
        pl->b = realloc(pl->b, sizeof(int64_t) * pl->cap);
        if (!pl->a || !pl->b) return -1;
    }
    pl->a[pl->n] = a;
    pl->b[pl->n] = b;
    ++pl->n;
    return 0;
}

/* Far lists (the low-rank part UV of Eq. (3)): a dual traversal from
 * (root, root); a pair of same-level nodes with no near leaf pair between them
 * is admitted as far, otherwise its four child pairs are visited. */
static int far_visit(orc_h *H, pair_list *pl, int64_t x, int64_t y, int lvl) {
    if (!near_related(H, x, y, lvl)) return push_pair(pl, x, y);
    if (lvl == H->depth) return 0;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            if (far_visit(H, pl, 2 * x + i, 2 * y + j, lvl + 1)) return -1;
    return 0;
}

static int build_far(orc_h *H) {
    pair_list pl = {0};
    if (far_visit(H, &pl, 1, 1, 0)) return -1;
    H->far_off = calloc((size_t)(H->nnodes + 1), sizeof(int32_t));
    H->far_idx = malloc(sizeof(int32_t) * (pl.n > 0 ? pl.n : 1));
    for (int64_t t = 0; t < pl.n; ++t) H->far_off[pl.a[t] + 1] += 1;
    for (int64_t h = 0; h < H->nnodes; ++h) H->far_off[h + 1] += H->far_off[h];
    int32_t *fill = calloc((size_t)(H->nnodes > 0 ? H->nnodes : 1), sizeof(int32_t));
    /* traversal order is not sorted by target: insert, then sort each row */
    for (int64_t t = 0; t < pl.n; ++t) {
        const int64_t a = pl.a[t];
        H->far_idx[H->far_off[a] + fill[a]++] = (int32_t)pl.b[t];
    }
    for (int64_t h = 0; h < H->nnodes; ++h) {
        int32_t *row = H->far_idx + H->far_off[h];
        const int32_t cnt = H->far_off[h + 1] - H->far_off[h];
        for (int32_t a = 1; a < cnt; ++a) {
            const int32_t v = row[a];
            int32_t b = a - 1;
            while (b >= 0 && row[b] > v) { row[b + 1] = row[b]; --b; }
            row[b + 1] = v;
        }
    }
    free(fill); free(pl.a); free(pl.b);
    return 0;
}

/* Rows that represent the rest of the matrix for node h: up to half of the
 * min(n - |node|, 2s) rows are neighbours (outside the node) of its candidate
 * columns, most-voted first (ties: lower index); uniform draws from outside the
 * node fill the rest.  Neighbour rows alone would only see the near side. */
static int sample_rows(orc_h *H, int64_t h, const int32_t *cand, int32_t nc, int32_t *cnt, unsigned char *mark,
                       vote_ent *ent, int32_t *rows_out) {
    const int64_t n = H->P.n, lo = H->start[h], hi = H->start[h] + H->size[h];
    int64_t want = n - H->size[h];
    if (want > 2 * (int64_t)H->s) want = 2 * (int64_t)H->s;
    int32_t ne = 0;
    for (int32_t c = 0; c < nc; ++c) {
        const int32_t j = cand[c];
        for (int t = 0; t < H->k; ++t) {
            const int32_t i = H->knn_idx[(int64_t)j * H->k + t];
            if (i < 0) continue;
            const int64_t pi = H->iperm[i];
            if (pi >= lo && pi < hi) continue;
            if (cnt[i] == 0) { ent[ne].id = i; ++ne; }
            cnt[i] += 1;
        }
    }
    for (int32_t e = 0; e < ne; ++e) ent[e].votes = cnt[ent[e].id];
    qsort(ent, (size_t)ne, sizeof(vote_ent), cmp_votes);
    int32_t nr = 0;
    const int64_t want_nb = want / 2;
    for (int32_t e = 0; e < ne; ++e) {
        cnt[ent[e].id] = 0;
        if (nr < want_nb) { rows_out[nr++] = ent[e].id; mark[ent[e].id] = 1; }
    }
    if (nr < want) {
        if (want == n - H->size[h]) {
            for (int64_t i = 0; i < n && nr < want; ++i) {
                const int64_t pi = H->iperm[i];
                if (pi >= lo && pi < hi) continue;
                if (!mark[i]) { rows_out[nr++] = (int32_t)i; mark[i] = 1; }
            }
        } else {
            uint32_t t = 0;
            const uint64_t cap = 64ull * (uint64_t)n + 1024ull;
            while (nr < want) {
                if ((uint64_t)t > cap) return -1;
                const int32_t i = (int32_t)uniform_below(orc_rand_u32(H->seed, PURPOSE_ROWS, (uint32_t)h, 0, t), (uint32_t)n);
                ++t;
                const int64_t pi = H->iperm[i];
                if (pi >= lo && pi < hi) continue;
                if (mark[i]) continue;
                rows_out[nr++] = i;
                mark[i] = 1;
            }
        }
    }
    for (int32_t r = 0; r < nr; ++r) mark[rows_out[r]] = 0;
    return nr;
}

/* Interpolative decomposition of B (nr x nc, row-major, overwritten) by
 * Householder QR with column pivoting: the pivot is the column of largest
 * remaining 2-norm (ties: lowest current column); the rank is the number of
 * pivots whose norm exceeds tau times the first, at most s.  Returns the rank;
 * cp[0..nc) receives the column order; P (rank x nc) satisfies
 * B[:, cp[j]] = I for j < rank and B ~ B[:, skel] P.  Every norm and inner
 * product is a plain sequential sum over increasing row index.
 *
 * trace (2 (kmax + 1) doubles, or NULL) records, for every pivot step j that
 * was examined, the largest remaining column norm (|R_jj|) and the second
 * largest (-1 when only one column remains); *nsteps receives the number of
 * examined steps.  Another implementation that sums in another order may pick
 * another pivot only where these two are within its rounding error. */
static int32_t pivoted_id(double *B, int32_t nr, int32_t nc, int32_t s, double tau, int32_t *cp, double *P,
                          double *v, double *trace, int32_t *nsteps) {
    for (int32_t c = 0; c < nc; ++c) cp[c] = c;
    int32_t kmax = nr < nc ? nr : nc;
    if (kmax > s) kmax = s;
    double r11 = 0.0;
    int32_t rank = 0, steps = 0;
    for (int32_t j = 0; j < kmax; ++j) {
        int32_t best = j;
        double bestv = -1.0, second = -1.0;
        for (int32_t c = j; c < nc; ++c) {
            double acc = 0.0;
            for (int32_t i = j; i < nr; ++i) acc = acc + B[(int64_t)i * nc + c] * B[(int64_t)i * nc + c];
            const double nrm = sqrt(acc);
            if (nrm > bestv) { second = bestv; bestv = nrm; best = c; }
            else if (nrm > second) second = nrm;
        }
        if (trace) { trace[2 * j] = bestv; trace[2 * j + 1] = second; }
        steps = j + 1;
        if (best != j) {
            for (int32_t i = 0; i < nr; ++i) {
                const double t = B[(int64_t)i * nc + j];
                B[(int64_t)i * nc + j] = B[(int64_t)i * nc + best];
                B[(int64_t)i * nc + best] = t;
            }
            const int32_t t = cp[j]; cp[j] = cp[best]; cp[best] = t;
        }
        if (j == 0) r11 = bestv;
        if (!(bestv > tau * r11)) break;
        const double x0 = B[(int64_t)j * nc + j];
        const double alpha = x0 >= 0.0 ? -bestv : bestv;
        v[j] = x0 - alpha;
        for (int32_t i = j + 1; i < nr; ++i) v[i] = B[(int64_t)i * nc + j];
        double vtv = 0.0;
        for (int32_t i = j; i < nr; ++i) vtv = vtv + v[i] * v[i];
        for (int32_t c = j + 1; c < nc; ++c) {
            double dot = 0.0;
            for (int32_t i = j; i < nr; ++i) dot = dot + v[i] * B[(int64_t)i * nc + c];
            const double f = (2.0 * dot) / vtv;
            for (int32_t i = j; i < nr; ++i) B[(int64_t)i * nc + c] = B[(int64_t)i * nc + c] - f * v[i];
        }
        B[(int64_t)j * nc + j] = alpha;
        for (int32_t i = j + 1; i < nr; ++i) B[(int64_t)i * nc + j] = 0.0;
        rank = j + 1;
    }
    if (nsteps) *nsteps = steps;
    /* P[:, cp[j]] = e_j (j < rank); P[:, cp[rank + c]] = R11^{-1} R12[:, c] */
    for (int64_t t = 0; t < (int64_t)rank * nc; ++t) P[t] = 0.0;
    for (int32_t j = 0; j < rank; ++j) P[(int64_t)j * nc + cp[j]] = 1.0;
    for (int32_t c = rank; c < nc; ++c) {
        for (int32_t i = rank - 1; i >= 0; --i) {
            double acc = B[(int64_t)i * nc + c];
            for (int32_t q = i + 1; q < rank; ++q) acc = acc - B[(int64_t)i * nc + q] * P[(int64_t)q * nc + cp[c]];
            P[(int64_t)i * nc + cp[c]] = acc / B[(int64_t)i * nc + i];
        }
    }
    return rank;
}

/* bottom-up skeletonisation: leaves offer their points as candidates, inner
 * nodes the skeletons of their two children (left first) */
static int skeletonize(orc_h *H) {
    const int64_t n = H->P.n;
    int32_t *cnt = calloc((size_t)n, sizeof(int32_t));
    unsigned char *mark = calloc((size_t)n, 1);
    int64_t maxc = 2 * (int64_t)H->s;
    const int64_t L = (int64_t)1 << H->depth;
    for (int64_t h = L; h < 2 * L; ++h)
        if (H->size[h] > maxc) maxc = H->size[h];
    vote_ent *ent = malloc(sizeof(vote_ent) * (size_t)(maxc * H->k + 1));
    int32_t *cand = malloc(sizeof(int32_t) * maxc);
    int32_t *cp = malloc(sizeof(int32_t) * maxc);
    double *v = malloc(sizeof(double) * (2 * H->s + 1));
    double *B = malloc(sizeof(double) * (size_t)(2 * H->s) * (size_t)maxc + 8);
    if (!cnt || !mark || !ent || !cand || !cp || !v || !B) return -1;
    for (int lvl = H->depth; lvl >= 1; --lvl) {
        for (int64_t h = (int64_t)1 << lvl; h < ((int64_t)1 << (lvl + 1)); ++h) {
            int32_t nc = 0;
            if (lvl == H->depth) {
                for (int64_t t = 0; t < H->size[h]; ++t) cand[nc++] = H->perm[H->start[h] + t];
            } else {
                for (int32_t t = 0; t < H->rank[2 * h]; ++t) cand[nc++] = H->skel[2 * h][t];
                for (int32_t t = 0; t < H->rank[2 * h + 1]; ++t) cand[nc++] = H->skel[2 * h + 1][t];
            }
            H->ncand[h] = nc;
            H->rows[h] = malloc(sizeof(int32_t) * (2 * H->s + 1));
            const int nr = sample_rows(H, h, cand, nc, cnt, mark, ent, H->rows[h]);
            if (nr < 0) return -1;
            H->nrows[h] = nr;
            for (int32_t r = 0; r < nr; ++r)
                for (int32_t c = 0; c < nc; ++c) B[(int64_t)r * nc + c] = kval(&H->P, H->rows[h][r], cand[c]);
            double *Pm = malloc(sizeof(double) * (size_t)(H->s) * (size_t)(nc > 0 ? nc : 1));
            H->trace[h] = malloc(sizeof(double) * 2 * ((size_t)H->s + 1));
            const int32_t rk = pivoted_id(B, nr, nc, H->s, H->tau, cp, Pm, v, H->trace[h], &H->nsteps[h]);
            H->rank[h] = rk;
            H->pmat[h] = Pm;
            H->skel[h] = malloc(sizeof(int32_t) * (rk > 0 ? rk : 1));
            for (int32_t t = 0; t < rk; ++t) H->skel[h][t] = cand[cp[t]];
        }
    }
    free(cnt); free(mark); free(ent); free(cand); free(cp); free(v); free(B);
    return 0;
}

void orc_free(orc_h *H) {
    if (!H) return;
    for (int64_t h = 0; h < H->nnodes; ++h) {
        if (H->skel) free(H->skel[h]);
        if (H->pmat) free(H->pmat[h]);
        if (H->rows) free(H->rows[h]);
        if (H->trace) free(H->trace[h]);
    }
    free(H->skel); free(H->pmat); free(H->rows); free(H->trace); free(H->nsteps); free(H->nrows); free(H->ncand); free(H->rank);
    free(H->start); free(H->size); free(H->perm); free(H->iperm); free(H->knn_idx); free(H->knn_d2);
    free(H->near_off); free(H->near_idx); free(H->far_off); free(H->far_idx);
    free(H);
}

/* Compress: tree, neighbours, near and far lists, nested skeletons.
 * x points to n x dim float64 (is_u8 = 0) or u8 codes (is_u8 = 1). */
orc_h *orc_compress(const void *x, int64_t n, int dim, int is_u8, double eps, int depth, int k, int knn_iters,
                    int s, double tau, double budget, uint64_t seed) {
    orc_h *H = calloc(1, sizeof(orc_h));
    if (!H) return NULL;
    H->P.n = n;
    H->P.dim = dim;
    H->P.is_u8 = is_u8;
    H->P.xf = is_u8 ? NULL : (const double *)x;
    H->P.xu = is_u8 ? (const uint8_t *)x : NULL;
    H->P.eps = eps;
    H->depth = depth;
    H->k = k;
    H->s = s;
    H->tau = tau;
    H->budget = budget;
    H->seed = seed;
    H->nnodes = (int64_t)1 << (depth + 1);
    H->start = malloc(sizeof(int64_t) * H->nnodes);
    H->size = malloc(sizeof(int64_t) * H->nnodes);
    H->perm = malloc(sizeof(int32_t) * n);
    H->iperm = malloc(sizeof(int32_t) * n);
    H->knn_idx = malloc(sizeof(int32_t) * n * k);
    H->knn_d2 = malloc(sizeof(double) * n * k);
    H->rank = calloc((size_t)H->nnodes, sizeof(int32_t));
    H->ncand = calloc((size_t)H->nnodes, sizeof(int32_t));
    H->nrows = calloc((size_t)H->nnodes, sizeof(int32_t));
    H->skel = calloc((size_t)H->nnodes, sizeof(int32_t *));
    H->pmat = calloc((size_t)H->nnodes, sizeof(double *));
    H->rows = calloc((size_t)H->nnodes, sizeof(int32_t *));
    H->trace = calloc((size_t)H->nnodes, sizeof(double *));
    H->nsteps = calloc((size_t)H->nnodes, sizeof(int32_t));
    if (!H->trace || !H->nsteps) { orc_free(H); return NULL; }
    if (!H->start || !H->size || !H->perm || !H->iperm || !H->knn_idx || !H->knn_d2 || !H->rank || !H->ncand ||
        !H->nrows || !H->skel || !H->pmat || !H->rows) { orc_free(H); return NULL; }
    tree_ranges(n, depth, H->start, H->size);
    if (orc_build_tree(&H->P, depth, seed, H->perm)) { orc_free(H); return NULL; }
    for (int64_t t = 0; t < n; ++t) H->iperm[H->perm[t]] = (int32_t)t;
    if (orc_knn(&H->P, depth, k, knn_iters, seed, H->knn_idx, H->knn_d2)) { orc_free(H); return NULL; }
    if (build_near(H) || build_far(H) || skeletonize(H)) { orc_free(H); return NULL; }
    return H;
}

/* ------------------------------------------------------------------------- */
/* Accessors                                                                   */
/* ------------------------------------------------------------------------- */
void orc_get_perm(const orc_h *H, int32_t *perm) { memcpy(perm, H->perm, sizeof(int32_t) * H->P.n); }
void orc_get_knn(const orc_h *H, int32_t *idx, double *d2) {
    memcpy(idx, H->knn_idx, sizeof(int32_t) * H->P.n * H->k);
    memcpy(d2, H->knn_d2, sizeof(double) * H->P.n * H->k);
}
int64_t orc_near_nnz(const orc_h *H) { return H->near_off[(int64_t)1 << H->depth]; }
void orc_get_near(const orc_h *H, int32_t *off, int32_t *idx) {
    const int64_t L = (int64_t)1 << H->depth;
    memcpy(off, H->near_off, sizeof(int32_t) * (L + 1));
    memcpy(idx, H->near_idx, sizeof(int32_t) * H->near_off[L]);
}
int64_t orc_far_nnz(const orc_h *H) { return H->far_off[H->nnodes]; }
void orc_get_far(const orc_h *H, int32_t *off, int32_t *idx) {
    memcpy(off, H->far_off, sizeof(int32_t) * (H->nnodes + 1));
    memcpy(idx, H->far_idx, sizeof(int32_t) * H->far_off[H->nnodes]);
}
void orc_get_ranks(const orc_h *H, int32_t *rank, int32_t *ncand, int32_t *nrows) {
    memcpy(rank, H->rank, sizeof(int32_t) * H->nnodes);
    memcpy(ncand, H->ncand, sizeof(int32_t) * H->nnodes);
    memcpy(nrows, H->nrows, sizeof(int32_t) * H->nnodes);
}
/* skeleton (rank), rows (nrows) and P (rank x ncand) of one heap node */
void orc_get_node(const orc_h *H, int64_t h, int32_t *skel, int32_t *rows, double *P) {
    if (H->rank[h] > 0) {
        memcpy(skel, H->skel[h], sizeof(int32_t) * H->rank[h]);
        memcpy(P, H->pmat[h], sizeof(double) * (size_t)H->rank[h] * (size_t)H->ncand[h]);
    }
    if (H->nrows[h] > 0) memcpy(rows, H->rows[h], sizeof(int32_t) * H->nrows[h]);
}

/* pivot trace of the ID of heap node h: returns the number of examined steps;
 * trace receives 2 per step (largest, second largest remaining column norm) */
int32_t orc_get_trace(const orc_h *H, int64_t h, double *trace) {
    const int32_t ns = H->nsteps[h];
    if (trace && ns > 0 && H->trace[h]) memcpy(trace, H->trace[h], sizeof(double) * 2 * (size_t)ns);
    return ns;
}

/* Floyd's sample of ns distinct positions of [0, n) for tree node `node`,
 * ascending (the ball tree's centroid sample; exported for its pin) */
int orc_sample_positions(uint64_t seed, uint32_t node, int64_t n, int ns, int64_t *out) {
    return sample_positions(seed, node, n, ns, out);
}

/* ID of one block (tests): B nr x nc row-major (overwritten), P rank x nc,
 * cp nc entries, trace 2 (min(nr, nc, s) + 1) doubles; returns the rank */
int32_t orc_pivoted_id(double *B, int32_t nr, int32_t nc, int32_t s, double tau, int32_t *cp, double *P,
                       double *trace, int32_t *nsteps) {
    double *v = malloc(sizeof(double) * (size_t)(nr > 0 ? nr : 1));
    if (!v) return -1;
    const int32_t rk = pivoted_id(B, nr, nc, s, tau, cp, P, v, trace, nsteps);
    free(v);
    return rk;
}

/* ------------------------------------------------------------------------- */
/* u = K~ w (float64), w and u n x nrhs column-major in original point order.  */
/* Upward pass (skeleton weights), far products between skeletons, downward     */
/* pass (skeleton potentials back to points) and the exact near blocks.         */
/* ------------------------------------------------------------------------- */
/* The same loops with every factor replaced by its magnitude (abs_mode = 1):
 * u = |K~| |w|, the row-wise scale that bounds the rounding error of any
 * evaluation of K~ w (each term of (K~ w)_i enters with its magnitude). */
static int hmatvec_impl(const orc_h *H, const double *w, double *u, int nrhs, int abs_mode) {
    const int64_t n = H->P.n, L = (int64_t)1 << H->depth;
    double **wt = calloc((size_t)H->nnodes, sizeof(double *));
    double **ut = calloc((size_t)H->nnodes, sizeof(double *));
    if (!wt || !ut) return -1;
    for (int64_t h = 2; h < H->nnodes; ++h) {
        wt[h] = calloc((size_t)(H->rank[h] > 0 ? H->rank[h] : 1) * nrhs, sizeof(double));
        ut[h] = calloc((size_t)(H->rank[h] > 0 ? H->rank[h] : 1) * nrhs, sizeof(double));
    }
    for (int64_t t = 0; t < n * nrhs; ++t) u[t] = 0.0;
    /* upward: w~_h = P_h [w_h] (leaf) or P_h [w~_left; w~_right] */
    for (int lvl = H->depth; lvl >= 1; --lvl) {
        for (int64_t h = (int64_t)1 << lvl; h < ((int64_t)1 << (lvl + 1)); ++h) {
            const int32_t rk = H->rank[h], nc = H->ncand[h];
            const double *Pm = H->pmat[h];
            for (int c = 0; c < nrhs; ++c) {
                for (int32_t i = 0; i < rk; ++i) {
                    double acc = 0.0;
                    for (int32_t j = 0; j < nc; ++j) {
                        double xj;
                        if (lvl == H->depth) {
                            xj = w[(int64_t)c * n + H->perm[H->start[h] + j]];
                            if (abs_mode) xj = fabs(xj);
                        } else {
                            const int32_t rl = H->rank[2 * h];
                            xj = j < rl ? wt[2 * h][(int64_t)c * rl + j]
                                        : wt[2 * h + 1][(int64_t)c * H->rank[2 * h + 1] + (j - rl)];
                        }
                        acc = acc + (abs_mode ? fabs(Pm[(int64_t)i * nc + j]) : Pm[(int64_t)i * nc + j]) * xj;
                    }
                    wt[h][(int64_t)c * rk + i] = acc;
                }
            }
        }
    }
    /* far: u~_h += K(skel_h, skel_g) w~_g for g in Far(h) */
    for (int64_t h = 2; h < H->nnodes; ++h) {
        for (int32_t t = H->far_off[h]; t < H->far_off[h + 1]; ++t) {
            const int32_t g = H->far_idx[t];
            for (int32_t i = 0; i < H->rank[h]; ++i)
                for (int32_t j = 0; j < H->rank[g]; ++j) {
                    const double kij = kval(&H->P, H->skel[h][i], H->skel[g][j]);
                    for (int c = 0; c < nrhs; ++c)
                        ut[h][(int64_t)c * H->rank[h] + i] += kij * wt[g][(int64_t)c * H->rank[g] + j];
                }
        }
    }
    /* downward: [u~_left; u~_right] += P_h^T u~_h; leaves: u_h += P_h^T u~_h */
    for (int lvl = 1; lvl <= H->depth; ++lvl) {
        for (int64_t h = (int64_t)1 << lvl; h < ((int64_t)1 << (lvl + 1)); ++h) {
            const int32_t rk = H->rank[h], nc = H->ncand[h];
            const double *Pm = H->pmat[h];
            for (int c = 0; c < nrhs; ++c) {
                for (int32_t j = 0; j < nc; ++j) {
                    double acc = 0.0;
                    for (int32_t i = 0; i < rk; ++i)
                        acc = acc + (abs_mode ? fabs(Pm[(int64_t)i * nc + j]) : Pm[(int64_t)i * nc + j]) * ut[h][(int64_t)c * rk + i];
                    if (lvl == H->depth) {
                        u[(int64_t)c * n + H->perm[H->start[h] + j]] += acc;
                    } else {
                        const int32_t rl = H->rank[2 * h];
                        if (j < rl) ut[2 * h][(int64_t)c * rl + j] += acc;
                        else ut[2 * h + 1][(int64_t)c * H->rank[2 * h + 1] + (j - rl)] += acc;
                    }
                }
            }
        }
    }
    /* near: u_a += K(a, b) w_b for b in Near(a), exact kernel values */
    for (int64_t a = 0; a < L; ++a) {
        const int64_t ha = L + a;
        for (int32_t t = H->near_off[a]; t < H->near_off[a + 1]; ++t) {
            const int64_t hb = L + H->near_idx[t];
            for (int64_t i = 0; i < H->size[ha]; ++i) {
                const int32_t pi = H->perm[H->start[ha] + i];
                for (int c = 0; c < nrhs; ++c) {
                    double acc = 0.0;
                    for (int64_t j = 0; j < H->size[hb]; ++j) {
                        const int32_t pj = H->perm[H->start[hb] + j];
                        const double wj = w[(int64_t)c * n + pj];
                        acc = acc + kval(&H->P, pi, pj) * (abs_mode ? fabs(wj) : wj);
                    }
                    u[(int64_t)c * n + pi] += acc;
                }
            }
        }
    }
    for (int64_t h = 2; h < H->nnodes; ++h) { free(wt[h]); free(ut[h]); }
    free(wt); free(ut);
    return 0;
}

int orc_hmatvec(const orc_h *H, const double *w, double *u, int nrhs) { return hmatvec_impl(H, w, u, nrhs, 0); }

/* u = |K~| |w| (see hmatvec_impl) */
int orc_hmatvec_abs(const orc_h *H, const double *w, double *u, int nrhs) { return hmatvec_impl(H, w, u, nrhs, 1); }

/* ------------------------------------------------------------------------- */
/* Dense definitions (Eq. (2)): rows [r0, r1) of u = K w, K evaluated on the  */
/* fly; OpenMP over rows.                                                       */
/* ------------------------------------------------------------------------- */
void orc_dense_kmatvec(const void *x, int64_t n, int dim, int is_u8, double eps, const double *w, int nrhs,
                       double *u, int64_t r0, int64_t r1) {
    orc_points P = {n, dim, is_u8, is_u8 ? NULL : (const double *)x, is_u8 ? (const uint8_t *)x : NULL, eps};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = r0; i < r1; ++i) {
        for (int c = 0; c < nrhs; ++c) {
            double acc = 0.0;
            for (int64_t j = 0; j < n; ++j) acc = acc + kval_libm(&P, i, j) * w[(int64_t)c * n + j];
            u[(int64_t)c * (r1 - r0) + (i - r0)] = acc;
        }
    }
}

/* rows [r0, r1) of the squared-distance matrix (for brute-force neighbours) */
void orc_dense_sqdist(const void *x, int64_t n, int dim, int is_u8, int64_t r0, int64_t r1, double *out) {
    orc_points P = {n, dim, is_u8, is_u8 ? NULL : (const double *)x, is_u8 ? (const uint8_t *)x : NULL, 1.0};
#pragma omp parallel for schedule(static)
    for (int64_t i = r0; i < r1; ++i)
        for (int64_t j = 0; j < n; ++j) out[(i - r0) * n + j] = sqd(&P, i, j);
}

/* kernel value between two points (test helper) */
double orc_kernel(const void *x, int64_t n, int dim, int is_u8, double eps, int64_t i, int64_t j) {
    orc_points P = {n, dim, is_u8, is_u8 ? NULL : (const double *)x, is_u8 ? (const uint8_t *)x : NULL, eps};
    return kval(&P, i, j);
}
