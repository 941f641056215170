// Lanczos iteration with full float64 reorthogonalisation (Sec. 2.2: the
// symmetric case of the Arnoldi factorisation of Alg. 2 / Eq. (5), whose
// projected matrix H is tridiagonal).  Every step: z = S~ x_j (one hierarchical
// product), classical Gram-Schmidt against the whole basis applied twice,
// alpha_j and beta_j = ||r_j||.  Every few steps the tridiagonal matrix is
// solved on the GPU for its leading Ritz values theta_i and the last entries of
// their eigenvectors; the pair is accepted when |beta_j y_{j,i}| <= tol |theta_i|
// (a Ritz pair is exact when the residual vanishes, Sec. 2.2).
#include <chrono>
#include <cmath>
#include <cstring>
#include <initializer_list>

#include "op.hpp"

namespace hdm {

namespace {

constexpr int kBlock = 256;
constexpr int kRows = 1024;   // rows per workgroup in the basis products

__global__ void k_start(double* v, int64_t n, uint64_t seed, uint32_t col) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    const uint32_t r = philox_draw(seed, kLanczosStart, col, 0, static_cast<uint32_t>(i));
    v[i] = (static_cast<double>(r) + 0.5) / 4294967296.0 - 0.5;
}

__device__ inline double block_sum(double v, double* sm) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane == 0) sm[wv] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < static_cast<int>(blockDim.x / 64); ++w) r += sm[w];
    __syncthreads();
    return r;
}

// Values passed between workgroups of one launch go through device-scope
// atomic stores and loads (coherent across the chip's L2 slices without
// flushing them).
__device__ inline void put_shared(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double get_shared(const double* p) {
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// h[c] = sum over the nb partial rows of column c (c in the 64-column group g):
// four quarters of the rows, eight interleaved partial sums each, combined in a
// fixed order.  Needs 256 threads.
template <bool kShared>
__device__ inline void reduce_cols_group(const double* partial, int nb, int ldp, int ncols, double* h, int g,
                                         double (*qs)[64]) {
    auto ld = [&](int64_t e) { return kShared ? get_shared(partial + e) : partial[e]; };
    const int cl = threadIdx.x % 64, qt = threadIdx.x / 64;
    const int c = g * 64 + cl;
    const int per = (nb + 3) / 4;
    const int b0 = min(nb, qt * per), b1 = min(nb, b0 + per);
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (c < ncols) {
        int b = b0;
        for (; b + 8 <= b1; b += 8) {
            double x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = ld(static_cast<int64_t>(b + u) * ldp + c);
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[u] += x[u];
        }
        for (; b < b1; ++b) acc[0] += ld(static_cast<int64_t>(b) * ldp + c);
    }
    qs[qt][cl] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    __syncthreads();
    if (qt == 0 && c < ncols) h[c] = ((qs[0][cl] + qs[1][cl]) + qs[2][cl]) + qs[3][cl];
    __syncthreads();
}

__global__ void __launch_bounds__(256) k_reduce_cols(const double* partial, int nb, int ldp, int ncols, double* h) {
    __shared__ double qs[4][64];
    reduce_cols_group<false>(partial, nb, ldp, ncols, h, blockIdx.x, qs);
}


// true in the one workgroup that finishes last.  Every thread's put_shared
// stores are ordered before thread 0's arrival by the barrier, and the arrival
// is a release at device scope; the last workgroup's arrival is also an
// acquire, and the barrier after it orders its threads' get_shared loads after
// it: the loads see every workgroup's stores (happens-before through the
// counter, under the HIP/HSA scoped memory model).  The counter is left at
// zero for the next launch.  Every thread of the workgroup must call it.
__device__ inline bool last_workgroup(unsigned* counter, bool* flag) {
    __syncthreads();
    if (threadIdx.x == 0)
        *flag = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
    __syncthreads();
    if (!*flag) return false;
    if (threadIdx.x == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// partial[b][c] = sum over the block's rows of V[row, c] * y[row], c < ncols.
// Each wave takes whole columns (lanes over rows, y held in registers) and
// reduces with a butterfly: no workgroup barriers per column.
__global__ void __launch_bounds__(kBlock) k_gemvt(const double* V, int64_t ldv, int ncols, const double* y, int64_t n,
                                                  double* partial, int ldp) {
    constexpr int kPer = kRows / 64;   // rows per lane
    const int64_t r0 = blockIdx.x * static_cast<int64_t>(kRows);
    const int wv = threadIdx.x / 64, lane = threadIdx.x % 64, nw = blockDim.x / 64;
    double yr[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int64_t row = r0 + u * 64 + lane;
        yr[u] = row < n ? y[row] : 0.0;
    }
    for (int c = wv; c < ncols; c += nw) {
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t row = r0 + u * 64 + lane;
            acc += (row < n ? V[c * ldv + row] : 0.0) * yr[u];
        }
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0) partial[static_cast<int64_t>(blockIdx.x) * ldp + c] = acc;
    }
}

// k_gemvt, then the last workgroup reduces the partial rows into h
__global__ void __launch_bounds__(kBlock) k_gemvt_h(const double* V, int64_t ldv, int ncols, const double* y, int64_t n,
                                                    double* partial, int ldp, double* h, unsigned* counter) {
    constexpr int kPer = kRows / 64;   // rows per lane
    const int64_t r0 = blockIdx.x * static_cast<int64_t>(kRows);
    const int wv = threadIdx.x / 64, lane = threadIdx.x % 64, nw = blockDim.x / 64;
    double yr[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int64_t row = r0 + u * 64 + lane;
        yr[u] = row < n ? y[row] : 0.0;
    }
    for (int c = wv; c < ncols; c += nw) {
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t row = r0 + u * 64 + lane;
            acc += (row < n ? V[c * ldv + row] : 0.0) * yr[u];
        }
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0) put_shared(partial + static_cast<int64_t>(blockIdx.x) * ldp + c, acc);
    }
    // the last workgroup sums the partial rows into h (the k_reduce_cols order)
    __shared__ bool last;
    __shared__ double qs[4][64];
    if (!last_workgroup(counter, &last)) return;
    for (int g = 0; g * 64 < ncols; ++g) reduce_cols_group<true>(partial, gridDim.x, ldp, ncols, h, g, qs);
}

// y -= V h (c < ncols); partial norms of the result when np != nullptr
__global__ void k_gemvn(const double* V, int64_t ldv, int ncols, const double* h, double* y, int64_t n, double* np) {
    __shared__ double sm[kBlock / 64];
    __shared__ double hs[1024];
    for (int c = threadIdx.x; c < ncols && c < 1024; c += blockDim.x) hs[c] = h[c];
    __syncthreads();
    const int64_t r0 = blockIdx.x * static_cast<int64_t>(kRows);
    double nrm = 0.0;
    for (int u = 0; u < kRows / kBlock; ++u) {
        const int64_t row = r0 + u * kBlock + threadIdx.x;
        if (row >= n) continue;
        double acc = 0.0;
        for (int c = 0; c < ncols; ++c) acc += V[c * ldv + row] * (c < 1024 ? hs[c] : h[c]);
        const double v = y[row] - acc;
        y[row] = v;
        nrm += v * v;
    }
    if (np) {
        const double t = block_sum(nrm, sm);
        if (threadIdx.x == 0) np[blockIdx.x] = t;
    }
}

// y -= V h (the k_gemvn rows and order), then the block's rows of the result
// (staged in shared memory) against V as in k_gemvt_h, whose last workgroup
// reduces the partial rows into h_out: the second Gram-Schmidt projection read
// with the first update, one pass over V instead of two
__global__ void __launch_bounds__(kBlock) k_gemvn_t_h(const double* V, int64_t ldv, int ncols, const double* h,
                                                      double* y, int64_t n, double* partial, int ldp, double* h_out,
                                                      unsigned* counter) {
    __shared__ double hs[1024];
    __shared__ double ys[kRows];
    for (int c = threadIdx.x; c < ncols && c < 1024; c += blockDim.x) hs[c] = h[c];
    __syncthreads();
    const int64_t r0 = blockIdx.x * static_cast<int64_t>(kRows);
    for (int u = 0; u < kRows / kBlock; ++u) {
        const int64_t row = r0 + u * kBlock + threadIdx.x;
        double v = 0.0;
        if (row < n) {
            double acc = 0.0;
            for (int c = 0; c < ncols; ++c) acc += V[c * ldv + row] * (c < 1024 ? hs[c] : h[c]);
            v = y[row] - acc;
            y[row] = v;
        }
        ys[u * kBlock + threadIdx.x] = v;
    }
    __syncthreads();
    constexpr int kPer = kRows / 64;   // rows per lane
    const int wv = threadIdx.x / 64, lane = threadIdx.x % 64, nw = blockDim.x / 64;
    double yr[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) yr[u] = ys[u * 64 + lane];
    for (int c = wv; c < ncols; c += nw) {
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t row = r0 + u * 64 + lane;
            acc += (row < n ? V[c * ldv + row] : 0.0) * yr[u];
        }
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0) put_shared(partial + static_cast<int64_t>(blockIdx.x) * ldp + c, acc);
    }
    __shared__ bool last;
    __shared__ double qs[4][64];
    if (!last_workgroup(counter, &last)) return;
    for (int g = 0; g * 64 < ncols; ++g) reduce_cols_group<true>(partial, gridDim.x, ldp, ncols, h_out, g, qs);
}

// k_gemvn with the partial norms, then the last workgroup forms alpha_j = h1[j] + h2[j]
// and beta_j = sqrt(sum of the partial norms) (the k_alpha_beta order)
__global__ void k_gemvn_ab(const double* V, int64_t ldv, int ncols, const double* h, double* y, int64_t n, double* np,
                           const double* h1, int j, double* alpha, double* beta, unsigned* counter) {
    __shared__ double sm[kBlock / 64];
    __shared__ double hs[1024];
    for (int c = threadIdx.x; c < ncols && c < 1024; c += blockDim.x) hs[c] = h[c];
    __syncthreads();
    const int64_t r0 = blockIdx.x * static_cast<int64_t>(kRows);
    double nrm = 0.0;
    for (int u = 0; u < kRows / kBlock; ++u) {
        const int64_t row = r0 + u * kBlock + threadIdx.x;
        if (row >= n) continue;
        double acc = 0.0;
        for (int c = 0; c < ncols; ++c) acc += V[c * ldv + row] * (c < 1024 ? hs[c] : h[c]);
        const double v = y[row] - acc;
        y[row] = v;
        nrm += v * v;
    }
    const double t = block_sum(nrm, sm);
    if (threadIdx.x == 0) put_shared(np + blockIdx.x, t);
    __shared__ bool last;
    if (!last_workgroup(counter, &last)) return;
    if (threadIdx.x == 0) {
        alpha[j] = h1[j] + h[j];
        double s2 = 0.0;
        for (int b = 0; b < static_cast<int>(gridDim.x); ++b) s2 += get_shared(np + b);
        beta[j] = sqrt(s2);
    }
}

// alpha_j = h1[j] + h2[j]; beta_j = sqrt(sum of partial norms)
__global__ void k_alpha_beta(const double* h1, const double* h2, int j, const double* np, int nb, double* alpha,
                             double* beta) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    alpha[j] = h1[j] + h2[j];
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += np[b];
    beta[j] = sqrt(s);
}

// x_{j+1} = r_j / beta_j
__global__ void k_next(const double* y, const double* beta, int j, double* vout, int64_t n) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    const double b = beta[j];
    vout[i] = b > 0.0 ? y[i] / b : 0.0;
}

__global__ void k_norm_partial(const double* v, int64_t n, double* np) {
    __shared__ double sm[kBlock / 64];
    const int64_t r0 = blockIdx.x * static_cast<int64_t>(kRows);
    double acc = 0.0;
    for (int u = 0; u < kRows / kBlock; ++u) {
        const int64_t row = r0 + u * kBlock + threadIdx.x;
        if (row < n) acc += v[row] * v[row];
    }
    const double t = block_sum(acc, sm);
    if (threadIdx.x == 0) np[blockIdx.x] = t;
}

__global__ void k_scale_by_norm(double* v, int64_t n, const double* np, int nb) {
    __shared__ double inv;
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += np[b];
        inv = 1.0 / sqrt(s);
    }
    __syncthreads();
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        v[i] *= inv;
}

// ---------------------------------------------------------------------------
// symmetric tridiagonal eigenproblem T (diag a[0..m), off-diag b[0..m-1))
// ---------------------------------------------------------------------------
// number of eigenvalues of T strictly below x (Sturm sequence of the LDL^T
// factorisation of T - x I; a zero pivot is nudged to a tiny negative value)
__device__ inline int sturm_below(const double* a, const double* b2, int m, double x, double tiny) {
    int cnt = 0;
    double q = a[0] - x;
    if (q == 0.0) q = -tiny;
    cnt += q < 0.0;
    for (int i = 1; i < m; ++i) {
        q = (a[i] - x) - b2[i - 1] / q;
        if (q == 0.0) q = -tiny;
        cnt += q < 0.0;
    }
    return cnt;
}

// One 64-lane workgroup per requested eigenvalue (k-th largest, k < r):
// multisection of the Gershgorin interval with 64 Sturm counts per round, then
// inverse iteration (three solves with one Gaussian elimination with partial
// pivoting of T - theta I) for the eigenvector.  T, the factors and the
// iterate live in shared memory (tridiag_shmem(m) bytes); the sequential
// passes of the elimination run on lane 0 in chunks of kTriChunk rows whose
// operands are loaded together, so one shared-memory round trip serves a
// chunk.  Outputs theta[k], Y[:, k] (m entries, unit norm) and the residual
// bound |beta_last * Y[m-1, k]|.
constexpr int kTriChunk = 8;

inline size_t tridiag_shmem(int m) {
    const size_t slots = static_cast<size_t>(m) + kTriChunk + 2;
    return slots * (8 * sizeof(double) + 1);
}

__global__ void __launch_bounds__(64) k_tridiag(const double* alpha, const double* beta, int m, int r,
                                                double* theta, double* Y, double* bound) {
    extern __shared__ double tsh[];
    const int ms = m + kTriChunk + 2;   // slots per array: chunk loads may run past m
    double* a = tsh;
    double* b2 = a + ms;
    double* bb = b2 + ms;
    double* u0 = bb + ms;   // U diagonal
    double* u1 = u0 + ms;
    double* u2 = u1 + ms;
    double* lmul = u2 + ms;
    double* x = lmul + ms;
    unsigned char* swp = reinterpret_cast<unsigned char*>(x + ms);   // 1: rows i, i+1 exchanged
    const int lane = threadIdx.x;
    const int k = blockIdx.x;
    for (int i = lane; i < ms; i += 64) {
        const bool in = i < m, off = i + 1 < m;
        a[i] = in ? alpha[i] : 0.0;
        bb[i] = off ? beta[i] : 0.0;
        b2[i] = off ? beta[i] * beta[i] : 0.0;
        x[i] = in ? 1.0 : 0.0;
        u0[i] = u1[i] = u2[i] = lmul[i] = 0.0;
        swp[i] = 0;
    }
    __syncthreads();
    // Gershgorin bounds: each lane over a strided share of the rows, then the
    // wave's min / max (exact, so the order does not matter)
    double lo = INFINITY, hi = -INFINITY, amax = 0.0;
    for (int i = lane; i < m; i += 64) {
        const double rad = (i > 0 ? fabs(bb[i - 1]) : 0.0) + fabs(bb[i]);
        lo = fmin(lo, a[i] - rad);
        hi = fmax(hi, a[i] + rad);
        amax = fmax(amax, fabs(a[i]) + rad);
    }
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
        amax = fmax(amax, __shfl_xor(amax, off, 64));
    }
    const double tiny = 1e-300 + amax * 1e-300;
    const int target = m - 1 - k;   // index in ascending order
    double l = lo - 1e-12 * (fabs(lo) + 1.0), h = hi + 1e-12 * (fabs(hi) + 1.0);
    for (int round = 0; round < 12; ++round) {
        const double xs = l + (h - l) * (lane + 1) / 65.0;
        const int c = sturm_below(a, b2, m, xs, tiny);
        // largest x with count <= target, smallest with count > target
        const unsigned long long le = __ballot(c <= target);
        const int nle = __popcll(le);   // counts are monotone in x: lanes 0..nle-1 satisfy it
        const double nl = nle > 0 ? l + (h - l) * nle / 65.0 : l;
        const double nh = nle < 64 ? l + (h - l) * (nle + 1) / 65.0 : h;
        l = nl;
        h = nh;
        if (h - l <= 2.0 * 2.220446049250313e-16 * fmax(fabs(l), fabs(h))) break;
    }
    const double th = 0.5 * (l + h);
    const double shift_eps = 2.220446049250313e-16 * fmax(amax, 1e-300);
    if (lane == 0) {
        // LU with partial pivoting of T - th I, rows i and i+1; the carried
        // (d, e) is the pending row i
        double d = a[0] - th, e = bb[0];
        for (int i0 = 0; i0 < m - 1; i0 += kTriChunk) {
            double ac[kTriChunk], bc[kTriChunk + 1];
#pragma unroll
            for (int u = 0; u < kTriChunk; ++u) { ac[u] = a[i0 + 1 + u]; bc[u] = bb[i0 + u]; }
            bc[kTriChunk] = bb[i0 + kTriChunk];
#pragma unroll
            for (int u = 0; u < kTriChunk; ++u) {
                const int i = i0 + u;
                if (i >= m - 1) break;
                const double sub = bc[u];
                const double dn = ac[u] - th, en = (i + 2 < m) ? bc[u + 1] : 0.0;
                if (fabs(d) >= fabs(sub)) {
                    const double piv_v = d == 0.0 ? shift_eps : d;
                    const double mult = sub / piv_v;
                    u0[i] = piv_v; u1[i] = e; u2[i] = 0.0;
                    lmul[i] = mult;
                    d = dn - mult * e;
                    e = en;
                    swp[i] = 0;
                } else {
                    const double mult = d / sub;
                    u0[i] = sub; u1[i] = dn; u2[i] = en;
                    lmul[i] = mult;
                    d = e - mult * dn;
                    e = 0.0 - mult * en;
                    swp[i] = 1;
                }
            }
        }
        u0[m - 1] = d == 0.0 ? shift_eps : d;
    }
    for (int iter = 0; iter < 3; ++iter) {
        if (lane == 0) {
            // forward elimination of the right-hand side; c is the current x[i]
            double c = x[0];
            for (int i0 = 0; i0 < m - 1; i0 += kTriChunk) {
                double lm[kTriChunk], nx[kTriChunk];
                unsigned char sw[kTriChunk];
#pragma unroll
                for (int u = 0; u < kTriChunk; ++u) { lm[u] = lmul[i0 + u]; nx[u] = x[i0 + 1 + u]; sw[u] = swp[i0 + u]; }
#pragma unroll
                for (int u = 0; u < kTriChunk; ++u) {
                    const int i = i0 + u;
                    if (i >= m - 1) break;
                    const double xi = sw[u] ? nx[u] : c, xn = sw[u] ? c : nx[u];
                    x[i] = xi;
                    c = xn - lm[u] * xi;
                }
            }
            x[m - 1] = c;
            // back substitution with U (bandwidth 2); x1, x2 are x[i+1], x[i+2]
            double x1 = 0.0, x2 = 0.0;
            for (int top = m - 1; top >= 0; top -= kTriChunk) {
                double xv[kTriChunk], d0[kTriChunk], d1[kTriChunk], d2[kTriChunk];
#pragma unroll
                for (int u = 0; u < kTriChunk; ++u) {
                    const int i = top - u < 0 ? 0 : top - u;
                    xv[u] = x[i]; d0[u] = u0[i]; d1[u] = u1[i]; d2[u] = u2[i];
                }
#pragma unroll
                for (int u = 0; u < kTriChunk; ++u) {
                    const int i = top - u;
                    if (i < 0) break;
                    double v = xv[u];
                    if (i + 1 < m) v -= d1[u] * x1;
                    if (i + 2 < m) v -= d2[u] * x2;
                    const double xi = v / d0[u];
                    x[i] = xi;
                    x2 = x1;
                    x1 = xi;
                }
            }
        }
        __syncthreads();
        double ss = 0.0;
        for (int i = lane; i < m; i += 64) ss += x[i] * x[i];
        for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
        const double nrm = sqrt(ss);
        for (int i = lane; i < m; i += 64) x[i] /= nrm;
        __syncthreads();
    }
    double* y = Y + static_cast<int64_t>(k) * m;
    for (int i = lane; i < m; i += 64) y[i] = x[i];
    if (lane == 0) {
        theta[k] = th;
        bound[k] = fabs(beta[m - 1] * x[m - 1]);
    }
}

// one workgroup per eigenvalue, shared memory set for the basis size
static void launch_tridiag(const double* alpha, const double* beta, int m, int r, double* theta, double* Y,
                           double* bound, hipStream_t s, hipEvent_t start = nullptr, hipEvent_t stop = nullptr) {
    const size_t shmem = tridiag_shmem(m);
    if (shmem > 65536)
        HDM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tridiag),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(shmem)));
    hipExtLaunchKernelGGL(k_tridiag, dim3(r), dim3(64), shmem, s, start, stop, 0, alpha, beta, m, r, theta, Y, bound);
}

// Phi[:, k] = V Y[:, k] for k < r (rows per thread); with perm, row p of V is
// point perm[p] of Phi (a basis kept in the tree's order)
__global__ void k_ritz(const double* V, int64_t ldv, int m, const double* Y, int r, double* Phi, int64_t n,
                       const int32_t* perm) {
    __shared__ double ys[4096];
    const int tot = m * r;
    for (int e = threadIdx.x; e < tot && e < 4096; e += blockDim.x) ys[e] = Y[e];
    __syncthreads();
    const int64_t row = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (row >= n) return;
    // sixteen vectors per pass over the basis (each V element loaded once per
    // pass); every output sums over the basis columns in increasing order
    constexpr int KB = 16;
    for (int k0 = 0; k0 < r; k0 += KB) {
        double acc[KB];
#pragma unroll
        for (int t = 0; t < KB; ++t) acc[t] = 0.0;
        for (int c = 0; c < m; ++c) {
            const double v = V[c * ldv + row];
#pragma unroll
            for (int t = 0; t < KB; ++t) {
                const int e = min(k0 + t, r - 1) * m + c;
                acc[t] += v * (e < 4096 ? ys[e] : Y[e]);
            }
        }
        const int64_t dst = perm ? perm[row] : row;
#pragma unroll
        for (int t = 0; t < KB; ++t)
            if (k0 + t < r) Phi[(k0 + t) * n + dst] = acc[t];
    }
}

// per column: 2-norm and index of the largest |entry| (first on ties)
// per column k: the scale that makes it unit-norm with its largest-magnitude entry
// (first index on ties) positive; computed before any entry is rescaled
__global__ void k_col_stats(const double* Phi, int64_t n, double* scale) {
    __shared__ double sv[kBlock];
    __shared__ int64_t si[kBlock];
    __shared__ double sn[kBlock];
    const int k = blockIdx.x;
    double best = -1.0, ss = 0.0;
    int64_t bi = INT64_MAX;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double v = Phi[k * n + i];
        ss += v * v;
        if (fabs(v) > best) { best = fabs(v); bi = i; }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    sn[threadIdx.x] = ss;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const double ov = sv[threadIdx.x + w];
            const int64_t oi = si[threadIdx.x + w];
            if (ov > sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi < si[threadIdx.x])) {
                sv[threadIdx.x] = ov;
                si[threadIdx.x] = oi;
            }
            sn[threadIdx.x] += sn[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t a = si[0];
        const double sgn = (a >= 0 && a < n && Phi[k * n + a] < 0.0) ? -1.0 : 1.0;
        scale[k] = sgn / sqrt(sn[0]);
    }
}

// Phi[:, k] *= scale[k]; the scale is fixed before this launch (workgroups of one
// launch rescale entries in place, so none of them may read an entry to decide it)
__global__ void k_col_fix(double* Phi, int64_t n, const double* scale) {
    const int k = blockIdx.y;
    const double sc = scale[k];
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        Phi[k * n + i] *= sc;
}

// ---------------------------------------------------------------------------
// block Lanczos (b right-hand sides per product): basis products, the block QR
// of the residual, the banded projected matrix and its Rayleigh-Ritz solve
// ---------------------------------------------------------------------------
constexpr int kMaxBlockBasis = 512;

// the start block: column c of V takes the start-vector draws of column c (the
// draw of point i, which sits at row p with perm[p] = i when V is in tree order)
__global__ void k_start_block(double* V, int64_t n, int b, uint64_t seed, const int32_t* perm) {
    const int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (e >= n * b) return;
    const uint32_t c = static_cast<uint32_t>(e / n), p = static_cast<uint32_t>(e % n);
    const uint32_t i = perm ? static_cast<uint32_t>(perm[p]) : p;
    const uint32_t r = philox_draw(seed, kLanczosStart, c, 0, i);
    V[e] = (static_cast<double>(r) + 0.5) / 4294967296.0 - 0.5;
}

// partial[blk][c * b + q] = sum over the block's rows of X[c][row] * Y[q][row]
// (c < ncols, q < b <= 16) on the float64 matrix cores.  One workgroup per
// (block of kGramRows rows, group of up to kGramTiles 16-column tiles of X); its
// four waves take a quarter of the rows each, 16 at a time: lane (m, k) loads
// rows 4k .. 4k + 3 of column m of X (for every tile) and of Y, and the four
// 16 x 16 x 4 instructions of a step take row 4k + s as their k-th term
// (s < 4).  The waves' sums meet in shared memory and are added in wave
// order.  Columns past ncols or b read the last column and rows past n read
// zeros; neither is stored.
typedef double d4_t __attribute__((ext_vector_type(4)));
constexpr int kGramRows = 256;
constexpr int kGramTiles = 8;
__global__ void __launch_bounds__(kBlock) k_gram_mma(const double* X, int64_t ldx, int ncols, const double* Y,
                                                     int64_t ldy, int b, int64_t n, double* partial, int64_t ldp) {
    __shared__ d4_t red[3][kGramTiles][64];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, m = lane % 16, k = lane / 16;
    const int t0 = blockIdx.y * kGramTiles;
    const int nt = min(kGramTiles, (ncols + 15) / 16 - t0);
    const int64_t r0 = blockIdx.x * static_cast<int64_t>(kGramRows) + wave * (kGramRows / 4);
    const int64_t r1 = min(n, r0 + kGramRows / 4);
    const double* yp = Y + static_cast<int64_t>(min(m, b - 1)) * ldy;
    const double* xp[kGramTiles];
#pragma unroll
    for (int t = 0; t < kGramTiles; ++t)
        xp[t] = X + static_cast<int64_t>(min(16 * (t0 + min(t, nt - 1)) + m, ncols - 1)) * ldx;
    d4_t acc[kGramTiles];
#pragma unroll
    for (int t = 0; t < kGramTiles; ++t) acc[t] = d4_t{0.0, 0.0, 0.0, 0.0};
    for (int64_t r = r0; r < r1; r += 16) {
        const int64_t row = r + 4 * k;
        double y[4], x[kGramTiles][4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const bool in = row + s < r1;
            const int64_t rr = in ? row + s : r0;
            y[s] = in ? yp[rr] : 0.0;
#pragma unroll
            for (int t = 0; t < kGramTiles; ++t) x[t][s] = t < nt ? xp[t][rr] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < kGramTiles; ++t)
            if (t < nt) {
#pragma unroll
                for (int s = 0; s < 4; ++s) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[t][s], y[s], acc[t], 0, 0, 0);
            }
    }
    if (wave > 0) {
#pragma unroll
        for (int t = 0; t < kGramTiles; ++t)
            if (t < nt) red[wave - 1][t][lane] = acc[t];
    }
    __syncthreads();
    if (wave > 0) return;
    // lane (m, k) holds entries (k + 4v, m) of every tile (the float64 instruction's
    // result layout): column 16 t + k + 4v of X against column m of Y
#pragma unroll
    for (int t = 0; t < kGramTiles; ++t) {
        if (t >= nt) break;
        const d4_t g = ((acc[t] + red[0][t][lane]) + red[1][t][lane]) + red[2][t][lane];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int c = 16 * (t0 + t) + k + 4 * v;
            if (c < ncols && m < b) partial[static_cast<int64_t>(blockIdx.x) * ldp + c * b + m] = g[v];
        }
    }
}

// Y[q][row] -= sum_c V[c][row] * H[c * b + q]
__global__ void __launch_bounds__(kBlock) k_gemmn(const double* V, int64_t ldv, int ncols, const double* H, double* Y,
                                                  int64_t ldy, int b, int64_t n) {
    __shared__ double hs[kMaxBlockBasis * kMaxRhs];
    for (int e = threadIdx.x; e < ncols * b; e += blockDim.x) hs[e] = H[e];
    __syncthreads();
    const int64_t row = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (row >= n) return;
    double acc[kMaxRhs];
#pragma unroll
    for (int q = 0; q < kMaxRhs; ++q) acc[q] = 0.0;
    for (int c = 0; c < ncols; ++c) {
        const double v = V[c * ldv + row];
#pragma unroll
        for (int q = 0; q < kMaxRhs; ++q) acc[q] += v * hs[c * b + min(q, b - 1)];
    }
    double yv[kMaxRhs];
#pragma unroll
    for (int q = 0; q < kMaxRhs; ++q) yv[q] = Y[min(q, b - 1) * ldy + row];
#pragma unroll
    for (int q = 0; q < kMaxRhs; ++q)
        if (q < b) Y[q * ldy + row] = yv[q] - acc[q];
}

__global__ void k_add(double* a, const double* b, int cnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) a[i] += b[i];
}

// Cholesky G + s I = R^T R (R upper, s = shift_coef * trace G), R^-1 and
// R_tot <- R R_tot, by one workgroup of 256 threads (one per element of a
// 16 x 16 block).  status = 1 when a pivot is not positive.
__global__ void __launch_bounds__(256) k_chol(const double* G, int b, double shift_coef, double* Rinv, double* Rtot,
                                              int* status) {
    __shared__ double A[kMaxRhs * kMaxRhs], R[kMaxRhs * kMaxRhs], W[kMaxRhs * kMaxRhs];
    __shared__ double sh;
    __shared__ int bad;
    const int t = threadIdx.x, i = t / kMaxRhs, k = t % kMaxRhs;
    const bool in = i < b && k < b;
    if (t == 0) {
        double tr = 0.0;
        for (int q = 0; q < b; ++q) tr += G[q * b + q];
        sh = shift_coef * tr;
        bad = 0;
    }
    __syncthreads();
    if (in) {
        A[i * b + k] = G[i * b + k] + (i == k ? sh : 0.0);
        R[i * b + k] = 0.0;
    }
    __syncthreads();
    // right-looking: row j of R, then the trailing update
    for (int j = 0; j < b; ++j) {
        if (t == 0) {
            const double dj = A[j * b + j];
            if (!(dj > 0.0)) bad = 1;
            R[j * b + j] = dj > 0.0 ? sqrt(dj) : 1.0;
        }
        __syncthreads();
        if (t > j && t < b) R[j * b + t] = A[j * b + t] / R[j * b + j];
        __syncthreads();
        if (in && i > j && k >= i) {
            A[i * b + k] -= R[j * b + i] * R[j * b + k];
            if (k > i) A[k * b + i] = A[i * b + k];
        }
        __syncthreads();
    }
    if (bad) {
        if (t == 0) *status = 1;
        return;
    }
    // R^-1: column c by back substitution (thread c)
    if (t < b) {
        const int c = t;
        for (int r = b - 1; r >= 0; --r) {
            double v = (r == c) ? 1.0 : 0.0;
            for (int q = r + 1; q < b; ++q) v -= R[r * b + q] * W[q * b + c];
            W[r * b + c] = r <= c ? v / R[r * b + r] : 0.0;
        }
    }
    __syncthreads();
    double rt = 0.0;
    if (in) {
        Rinv[i * b + k] = W[i * b + k];
        for (int q = i; q <= k; ++q) rt += R[i * b + q] * Rtot[q * b + k];
    }
    __syncthreads();
    if (in) Rtot[i * b + k] = k >= i ? rt : 0.0;
}

__global__ void k_eye(double* R, int b) {
    const int e = threadIdx.x;
    if (e < b * b) R[e] = (e / b == e % b) ? 1.0 : 0.0;
}

// rows of Y times R^-1 (upper), in place
__global__ void __launch_bounds__(kBlock) k_trsm(double* Y, int64_t ldy, int b, int64_t n, const double* Rinv) {
    __shared__ double ri[kMaxRhs * kMaxRhs];
    for (int e = threadIdx.x; e < b * b; e += blockDim.x) ri[e] = Rinv[e];
    __syncthreads();
    const int64_t row = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (row >= n) return;
    double y[kMaxRhs];
#pragma unroll
    for (int q = 0; q < kMaxRhs; ++q) y[q] = Y[min(q, b - 1) * ldy + row];
#pragma unroll
    for (int q = 0; q < kMaxRhs; ++q) {
        if (q >= b) break;
        double t = 0.0;
#pragma unroll
        for (int p = 0; p <= q; ++p) t += y[p] * ri[p * b + q];
        Y[q * ldy + row] = t;
    }
}

// block j of the banded projected matrix: T_jj = sym(A_j), T_{j+1,j} = B_j, T_{j,j+1} = B_j^T
__global__ void k_put_T(double* T, int ldt, int j, int b, const double* H, const double* Rtot) {
    const int e = threadIdx.x;
    if (e >= b * b) return;
    const int p = e / b, q = e % b;
    const int64_t o = static_cast<int64_t>(j) * b;
    T[(o + p) * ldt + o + q] = 0.5 * (H[(o + p) * b + q] + H[(o + q) * b + p]);
    T[(o + b + p) * ldt + o + q] = Rtot[p * b + q];
    T[(o + q) * ldt + o + b + p] = Rtot[p * b + q];
}

// sum over a workgroup of any size (multiple of 64), result in every thread
__device__ inline double wg_sum(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int wv = threadIdx.x / 64, lane = threadIdx.x % 64, nw = blockDim.x / 64;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += red[w];
    return t;
}

// Householder tridiagonalisation (one workgroup) of the leading m x m block of
// the symmetric T: d, e (e[m-1] = 0), the reflectors below the subdiagonal of
// A's columns and tau, so that T = Q tridiag(d, e) Q^T, Q = H_0 ... H_{m-3}.
__global__ void __launch_bounds__(1024) k_sytrd(const double* T, int ldt, int m, double* A, int lda, double* d,
                                                 double* e, double* tau) {
    __shared__ double v[kMaxBlockBasis], w[kMaxBlockBasis], red[16];
    __shared__ double s_tau;
    for (int64_t x = threadIdx.x; x < static_cast<int64_t>(m) * m; x += blockDim.x) {
        const int i = static_cast<int>(x / m), j = static_cast<int>(x % m);
        A[static_cast<int64_t>(i) * lda + j] = T[static_cast<int64_t>(i) * ldt + j];
    }
    __syncthreads();
    for (int k = 0; k + 1 < m; ++k) {
        const int len = m - k - 1;
        const int i = threadIdx.x;
        // x = column k below the diagonal, read as row k
        const double xi = i < len ? A[static_cast<int64_t>(k) * lda + k + 1 + i] : 0.0;
        const double sigma = wg_sum(i >= 1 && i < len ? xi * xi : 0.0, red);
        const double alpha = A[static_cast<int64_t>(k) * lda + k + 1];
        if (threadIdx.x == 0) d[k] = A[static_cast<int64_t>(k) * lda + k];
        if (len == 1 || sigma == 0.0) {
            if (threadIdx.x == 0) {
                e[k] = alpha;
                tau[k] = 0.0;
            }
            __syncthreads();
            continue;
        }
        const double mu = sqrt(alpha * alpha + sigma);
        const double beta = alpha <= 0.0 ? mu : -mu;
        const double t = (beta - alpha) / beta;
        const double inv = 1.0 / (alpha - beta);
        if (i < len) v[i] = i == 0 ? 1.0 : xi * inv;
        if (threadIdx.x == 0) {
            e[k] = beta;
            tau[k] = t;
            s_tau = t;
        }
        __syncthreads();
        // p = tau A22 v (A22 symmetric: element (j, i) read along rows, coalesced in i)
        double pi = 0.0;
        if (i < len) {
            const double* col = A + static_cast<int64_t>(k + 1) * lda + k + 1 + i;
            for (int j = 0; j < len; ++j) pi += col[static_cast<int64_t>(j) * lda] * v[j];
            pi *= s_tau;
        }
        const double K = 0.5 * s_tau * wg_sum(i < len ? pi * v[i] : 0.0, red);
        if (i < len) w[i] = pi - K * v[i];
        __syncthreads();
        // A22 -= v w^T + w v^T
        for (int64_t x = threadIdx.x; x < static_cast<int64_t>(len) * len; x += blockDim.x) {
            const int jj = static_cast<int>(x / len), ii = static_cast<int>(x % len);
            A[static_cast<int64_t>(k + 1 + jj) * lda + k + 1 + ii] -= v[ii] * w[jj] + w[ii] * v[jj];
        }
        // keep the reflector in column k (rows k+2 .., never read again)
        if (i >= 1 && i < len) A[static_cast<int64_t>(k + 1 + i) * lda + k] = v[i];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        d[m - 1] = A[static_cast<int64_t>(m - 1) * lda + m - 1];
        e[m - 1] = 0.0;
    }
}

// The same reduction with the matrix in shared memory (m <= kSytrdLds, leading
// dimension m + 1 against bank conflicts) and the product p = tau A22 v taken by
// eight threads per row (columns j = t mod 8, then combined across the eight in
// a fixed order), so that a step is a few barriers rather than len dependent
// global loads per thread.  The reflectors go to A's columns in global memory
// as they are formed (k_ormtr reads them there).
constexpr int kSytrdLds = 128;
__global__ void __launch_bounds__(1024) k_sytrd_lds(const double* T, int ldt, int m, double* A, int lda, double* d,
                                                     double* e, double* tau) {
    extern __shared__ double M[];
    __shared__ double v[kSytrdLds], w[kSytrdLds], red[16];
    __shared__ double s_tau;
    const int ldm = m + 1;
    for (int x = threadIdx.x; x < m * m; x += blockDim.x) {
        const int i = x / m, j = x % m;
        M[i * ldm + j] = T[static_cast<int64_t>(i) * ldt + j];
    }
    __syncthreads();
    const int row = threadIdx.x / 8, t8 = threadIdx.x % 8;
    for (int k = 0; k + 1 < m; ++k) {
        const int len = m - k - 1;
        const int i = threadIdx.x;
        const double xi = i < len ? M[k * ldm + k + 1 + i] : 0.0;
        const double sigma = wg_sum(i >= 1 && i < len ? xi * xi : 0.0, red);
        const double alpha = M[k * ldm + k + 1];
        if (threadIdx.x == 0) d[k] = M[k * ldm + k];
        if (len == 1 || sigma == 0.0) {
            if (threadIdx.x == 0) {
                e[k] = alpha;
                tau[k] = 0.0;
            }
            __syncthreads();
            continue;
        }
        const double mu = sqrt(alpha * alpha + sigma);
        const double beta = alpha <= 0.0 ? mu : -mu;
        const double tk = (beta - alpha) / beta;
        const double inv = 1.0 / (alpha - beta);
        if (i < len) {
            v[i] = i == 0 ? 1.0 : xi * inv;
            if (i >= 1) A[static_cast<int64_t>(k + 1 + i) * lda + k] = xi * inv;   // the reflector, below the subdiagonal
        }
        if (threadIdx.x == 0) {
            e[k] = beta;
            tau[k] = tk;
            s_tau = tk;
        }
        __syncthreads();
        // p_row = tau sum_j A22[row][j] v[j]: eight partial sums (j = t8 mod 8), combined in a fixed order
        double part = 0.0;
        if (row < len) {
            const double* r = M + (k + 1 + row) * ldm + k + 1;
            for (int j = t8; j < len; j += 8) part += r[j] * v[j];
        }
        part += __shfl_xor(part, 1, 8);
        part += __shfl_xor(part, 2, 8);
        part += __shfl_xor(part, 4, 8);
        const double pi = part * s_tau;
        const double K = 0.5 * s_tau * wg_sum(row < len && t8 == 0 ? pi * v[row] : 0.0, red);
        if (row < len && t8 == 0) w[row] = pi - K * v[row];
        __syncthreads();
        // A22 -= v w^T + w v^T
        for (int x = threadIdx.x; x < len * len; x += blockDim.x) {
            const int jj = x / len, ii = x % len;
            M[(k + 1 + jj) * ldm + k + 1 + ii] -= v[ii] * w[jj] + w[ii] * v[jj];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        d[m - 1] = M[(m - 1) * ldm + m - 1];
        e[m - 1] = 0.0;
    }
}

// the reduction of the leading m x m block of T: in shared memory up to
// kSytrdLds, else in global memory (A)
static void launch_sytrd(const double* T, int ldt, int m, double* A, int lda, double* d, double* e, double* tau,
                         hipStream_t s, hipEvent_t start = nullptr, hipEvent_t stop = nullptr) {
    if (m <= kSytrdLds) {
        const size_t shmem = static_cast<size_t>(m) * (m + 1) * sizeof(double);
        if (shmem > 65536)
            HDM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sytrd_lds),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(shmem)));
        hipExtLaunchKernelGGL(k_sytrd_lds, dim3(1), dim3(1024), shmem, s, start, stop, 0, T, ldt, m, A, lda, d, e, tau);
    } else {
        hipExtLaunchKernelGGL(k_sytrd, dim3(1), dim3(1024), 0, s, start, stop, 0, T, ldt, m, A, lda, d, e, tau);
    }
}

// Z[k] <- Q Z[k] for the r eigenvectors of the tridiagonal matrix (one wave per vector)
__global__ void __launch_bounds__(1024) k_ormtr(const double* A, int lda, const double* tau, int m, double* Z, int r) {
    __shared__ double zs[16][kMaxBlockBasis];
    const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int k = wv; k < r; k += 16) {
        double* z = zs[wv];
        for (int i = lane; i < m; i += 64) z[i] = Z[static_cast<int64_t>(k) * m + i];
        for (int kk = m - 3; kk >= 0; --kk) {
            const double t = tau[kk];
            if (t == 0.0) continue;
            const int len = m - kk - 1;   // rows kk+1 .. m-1, v[kk+1] = 1
            double dot = 0.0;
            for (int i = lane; i < len; i += 64) {
                const double vi = i == 0 ? 1.0 : A[static_cast<int64_t>(kk + 1 + i) * lda + kk];
                dot += vi * z[kk + 1 + i];
            }
            for (int off = 32; off > 0; off >>= 1) dot += __shfl_xor(dot, off, 64);
            for (int i = lane; i < len; i += 64) {
                const double vi = i == 0 ? 1.0 : A[static_cast<int64_t>(kk + 1 + i) * lda + kk];
                z[kk + 1 + i] -= t * dot * vi;
            }
        }
        for (int i = lane; i < m; i += 64) Z[static_cast<int64_t>(k) * m + i] = z[i];
    }
}

// The same back-transformation with the reflectors and tau staged in shared
// memory first (m <= kSytrdLds): each vector's m - 2 dependent steps then read
// no global memory.  Same sums in the same order as k_ormtr.
__global__ void __launch_bounds__(1024) k_ormtr_lds(const double* A, int lda, const double* tau, int m, double* Z,
                                                     int r) {
    extern __shared__ double sh[];
    double* refl = sh;               // reflector kk in row kk: entry i at refl[kk m + i] (v_0 = 1)
    double* ts = sh + m * m;         // tau
    double* zs = ts + m;             // one vector per wave
    for (int x = threadIdx.x; x < m * m; x += blockDim.x) {
        const int kk = x / m, i = x % m, len = m - kk - 1;
        refl[x] = i == 0 ? 1.0 : (i < len ? A[static_cast<int64_t>(kk + 1 + i) * lda + kk] : 0.0);
    }
    for (int x = threadIdx.x; x < m; x += blockDim.x) ts[x] = tau[x];
    __syncthreads();
    const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int k = wv; k < r; k += 16) {
        double* z = zs + wv * m;
        for (int i = lane; i < m; i += 64) z[i] = Z[static_cast<int64_t>(k) * m + i];
        for (int kk = m - 3; kk >= 0; --kk) {
            const double t = ts[kk];
            if (t == 0.0) continue;
            const int len = m - kk - 1;
            const double* v = refl + kk * m;
            double dot = 0.0;
            for (int i = lane; i < len; i += 64) dot += v[i] * z[kk + 1 + i];
            for (int off = 32; off > 0; off >>= 1) dot += __shfl_xor(dot, off, 64);
            for (int i = lane; i < len; i += 64) z[kk + 1 + i] -= t * dot * v[i];
        }
        for (int i = lane; i < m; i += 64) Z[static_cast<int64_t>(k) * m + i] = z[i];
    }
}

static void launch_ormtr(const double* A, int lda, const double* tau, int m, double* Z, int r, hipStream_t s) {
    if (m <= kSytrdLds) {
        const size_t shmem = (static_cast<size_t>(m) * m + m + 16 * static_cast<size_t>(m)) * sizeof(double);
        if (shmem > 65536)
            HDM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_ormtr_lds),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(shmem)));
        hipLaunchKernelGGL(k_ormtr_lds, dim3(1), dim3(1024), shmem, s, A, lda, tau, m, Z, r);
    } else {
        hipLaunchKernelGGL(k_ormtr, dim3(1), dim3(1024), 0, s, A, lda, tau, m, Z, r);
    }
}

// ---- thick restart of the single-vector iteration ---------------------------------
// The projected matrix T = V^T S~ V after a restart with k kept Ritz pairs is the
// diagonal of their Ritz values, coupled to the first new Lanczos vector by
// s_i = beta_m y_i[m - 1] (row and column k), followed by the tridiagonal of the
// steps since (Wu and Simon, thick-restart Lanczos, 2000; the exact-shift case of
// the implicitly restarted Lanczos method).
__global__ void k_thick_head(double* T, int ldt, int keep, int m_old, const double* theta, const double* Y,
                             const double* beta, int jlast) {
    // T is cleared by the caller; one thread per kept pair
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= keep) return;
    const double s = beta[jlast] * Y[static_cast<int64_t>(i) * m_old + (m_old - 1)];
    T[static_cast<int64_t>(i) * ldt + i] = theta[i];
    T[static_cast<int64_t>(i) * ldt + keep] = s;
    T[static_cast<int64_t>(keep) * ldt + i] = s;
}

// the tridiagonal tail of T from the Lanczos coefficients of steps k .. m - 1
__global__ void k_thick_tail(double* T, int ldt, int k, int m, const double* alpha, const double* beta) {
    const int i = k + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    T[static_cast<int64_t>(i) * ldt + i] = alpha[i];
    if (i + 1 < m) {
        T[static_cast<int64_t>(i) * ldt + i + 1] = beta[i];
        T[static_cast<int64_t>(i + 1) * ldt + i] = beta[i];
    }
}

// residual bound of Ritz pair i of T (eigenvector row i of Y, m entries): |beta_{m-1} y_i[m - 1]|
__global__ void k_thick_bounds(const double* Y, int m, const double* beta, int jlast, int r, double* bound) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= r) return;
    bound[i] = fabs(beta[jlast] * Y[static_cast<int64_t>(i) * m + (m - 1)]);
}

__global__ void k_fill0(double* p, int64_t n) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// residual bound of Ritz pair k: || B_j Z[k][m-b .. m) ||
__global__ void k_block_bounds(const double* Z, int m, int b, const double* Bj, int r, double* bound) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= r) return;
    const double* y = Z + static_cast<int64_t>(k) * m + (m - b);
    double s = 0.0;
    for (int p = 0; p < b; ++p) {
        double t = 0.0;
        for (int q = 0; q < b; ++q) t += Bj[p * b + q] * y[q];
        s += t * t;
    }
    bound[k] = sqrt(s);
}

}  // namespace

// Small results of a convergence check to the host with one wait: through pinned
// staging inside a pool scope (the copies queue without a host round trip each;
// pageable copies wait one by one), else directly.
struct HostPart {
    void* host;
    const void* dev;
    size_t bytes;
};
static void download_parts(std::initializer_list<HostPart> parts, hipStream_t s) {
    size_t total = 0;
    for (const HostPart& q : parts) total += (q.bytes + 15) / 16 * 16;
    char* h = static_cast<char*>(host_stage(total));
    size_t off = 0;
    for (const HostPart& q : parts) {
        if (!q.bytes) continue;
        HDM_HIP(hipMemcpyAsync(h ? h + off : q.host, q.dev, q.bytes, hipMemcpyDeviceToHost, s));
        off += (q.bytes + 15) / 16 * 16;
    }
    HDM_HIP(hipStreamSynchronize(s));
    if (!h) return;
    off = 0;
    for (const HostPart& q : parts) {
        if (q.bytes) std::memcpy(q.host, h + off, q.bytes);
        off += (q.bytes + 15) / 16 * 16;
    }
}

// restarts of one single-vector solve before it ends with HDM_ENOCONV (the
// standalone solve and the serving loop alike, so their results agree)
constexpr int kMaxRestarts = 100;

void LanczosRun::start(Op& o, int r_, double tol_, int max_basis_, uint64_t seed_, hipStream_t s) {
    op = &o;
    n = o.n;
    HDM_CHECK(r_ >= 1 && r_ <= 64 && r_ <= n, HDM_EINVAL, "r must be in [1, min(64, n)]");
    int mb = max_basis_ <= 0 ? static_cast<int>(std::min<int64_t>(n, 300)) : max_basis_;
    mb = static_cast<int>(std::min<int64_t>(mb, n));
    HDM_CHECK(mb >= r_ && mb <= 1000, HDM_EINVAL, "max_basis must be in [r, 1000]");
    r = r_;
    tol = tol_;
    max_basis = mb;
    seed = seed_;
    nb = ceil_div(n, kRows);
    ldp = max_basis + 1;
    V.alloc(static_cast<size_t>(n) * (max_basis + 1));
    y.alloc(n);
    part.alloc(static_cast<size_t>(nb) * ldp);
    h1.alloc(ldp);
    h2.alloc(ldp);
    np.alloc(nb);
    alpha.alloc(max_basis);
    beta.alloc(max_basis);
    theta.alloc(max_basis);
    bound.alloc(max_basis);
    Y.alloc(static_cast<size_t>(max_basis) * max_basis);
    restarts = keep = 0;
    max_restarts = kMaxRestarts;
    restarted = false;
    counters.alloc(2);
    HDM_HIP(hipMemsetAsync(counters.get(), 0, counters.bytes(), s));
    h_theta.assign(r, 0.0);
    h_bound.assign(r, 0.0);
    j = m = matvecs = 0;
    converged = finished = false;
    t0 = std::chrono::steady_clock::now();
    const int gN = ceil_div(n, kBlock);
    hipLaunchKernelGGL(k_start, dim3(gN), dim3(kBlock), 0, s, V.get(), n, seed, 0u);
    hipLaunchKernelGGL(k_norm_partial, dim3(nb), dim3(kBlock), 0, s, V.get(), n, np.get());
    hipLaunchKernelGGL(k_scale_by_norm, dim3(std::min(gN, 1024)), dim3(kBlock), 0, s, V.get(), n, np.get(), nb);
    check_launch("lanczos start");
}

size_t LanczosRun::bytes() const {
    return V.bytes() + y.bytes() + part.bytes() + h1.bytes() + h2.bytes() + np.bytes() + alpha.bytes() +
           beta.bytes() + theta.bytes() + bound.bytes() + Y.bytes();
}

bool LanczosRun::after_product(hipStream_t s) {
    ++matvecs;
    const int nc = j + 1;
    {   // CGS2 against the whole basis, alpha_j, beta_j
        PhaseScope ph(op->ctx, HDM_PHASE_ORTHO, s);
        unsigned* cnt = counters.get();
        hipLaunchKernelGGL(k_gemvt_h, dim3(nb), dim3(kBlock), 0, s, V.get(), n, nc, y.get(), n, part.get(), ldp,
                           h1.get(), cnt);
        hipLaunchKernelGGL(k_gemvn_t_h, dim3(nb), dim3(kBlock), 0, s, V.get(), n, nc, h1.get(), y.get(), n,
                           part.get(), ldp, h2.get(), cnt);
        hipLaunchKernelGGL(k_gemvn_ab, dim3(nb), dim3(kBlock), 0, s, V.get(), n, nc, h2.get(), y.get(), n, np.get(),
                           h1.get(), j, alpha.get(), beta.get(), cnt + 1);
    }
    check_launch("lanczos step");
    m = j + 1;
    const bool last = (j == max_basis - 1);
    // Each check costs a tridiagonal eigensolve and a host synchronisation; r
    // pairs rarely meet the tolerance before 2r steps, so checking starts there.
    if ((m >= 2 * r && (m % check_every) == 0) || (last && m >= r)) {
        if (restarted) {
            solve_projected(r, s);
        } else {
            KernelEvents ev(op->ctx, HDM_PHASE_TRIDIAG);
            launch_tridiag(alpha.get(), beta.get(), m, r, theta.get(), Y.get(), bound.get(), s, ev.start, ev.stop);
        }
        check_launch("tridiagonal eigensolve");
        download_parts({{h_theta.data(), theta.get(), r * sizeof(double)}, {h_bound.data(), bound.get(), r * sizeof(double)}},
                       s);
        bool ok = true;
        for (int i = 0; i < r; ++i) ok = ok && (h_bound[i] <= tol * std::fabs(h_theta[i]));
        if (ok) {
            converged = finished = true;
            return true;
        }
    }
    hipLaunchKernelGGL(k_next, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, y.get(), beta.get(), j,
                       V.get() + static_cast<int64_t>(j + 1) * n, n);
    if (last) {
        if (restarts >= max_restarts || max_basis > kMaxBlockBasis || max_basis < r + 2) {
            finished = true;
            return true;
        }
        restart(s);
        return false;
    }
    ++j;
    return false;
}

// Ritz pairs of the (restarted) projected matrix: its tail from the latest
// Lanczos coefficients, Householder tridiagonalisation, the tridiagonal
// eigensolve for the nvec largest, back-transformation, residual bounds
void LanczosRun::solve_projected(int nvec, hipStream_t s) {
    const int ldt = max_basis + 1;
    hipLaunchKernelGGL(k_thick_tail, dim3(ceil_div(m - keep, kBlock)), dim3(kBlock), 0, s, T.get(), ldt, keep, m,
                       alpha.get(), beta.get());
    KernelEvents ev(op->ctx, HDM_PHASE_TRIDIAG);
    launch_sytrd(T.get(), ldt, m, A.get(), ldt, dd.get(), ee.get(), tau.get(), s);
    launch_tridiag(dd.get(), ee.get(), m, nvec, theta.get(), Y.get(), bound.get(), s, ev.start, nullptr);
    launch_ormtr(A.get(), ldt, tau.get(), m, Y.get(), nvec, s);
    hipExtLaunchKernelGGL(k_thick_bounds, dim3(ceil_div(nvec, 64)), dim3(64), 0, s, nullptr, ev.stop, 0, Y.get(), m,
                          beta.get(), m - 1, nvec, bound.get());
}

// Thick restart at a full basis of m = max_basis vectors: keep the leading
// `keep` Ritz vectors V Y_keep and the next Lanczos vector v_{m+1} (already
// formed in column m), and restart the projected matrix from their Ritz values
// and couplings.  The iteration then continues from column keep.
void LanczosRun::restart(hipStream_t s) {
    const int ldt = max_basis + 1;
    if (!restarted) {
        T.alloc(static_cast<size_t>(ldt) * ldt);
        A.alloc(static_cast<size_t>(ldt) * ldt);
        dd.alloc(ldt);
        ee.alloc(ldt);
        tau.alloc(ldt);
        // the basis so far is plain Lanczos: its projected matrix is the tridiagonal
        hipLaunchKernelGGL(k_fill0, dim3(ceil_div(int64_t(ldt) * ldt, kBlock)), dim3(kBlock), 0, s, T.get(),
                           int64_t(ldt) * ldt);
        keep = 0;
    }
    // keep about half of the free space beyond the r wanted pairs, at most max_basis - 2
    const int kp = std::min(max_basis - 2, std::max(r + 1, (max_basis + r) / 2));
    solve_projected(kp, s);
    tmp.alloc(static_cast<size_t>(n) * kp);
    hipLaunchKernelGGL(k_ritz, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, V.get(), n, m, Y.get(), kp, tmp.get(), n,
                       nullptr);
    HDM_HIP(hipMemcpyAsync(V.get(), tmp.get(), sizeof(double) * n * kp, hipMemcpyDeviceToDevice, s));
    HDM_HIP(hipMemcpyAsync(V.get() + static_cast<int64_t>(kp) * n, V.get() + static_cast<int64_t>(m) * n,
                           sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_fill0, dim3(ceil_div(int64_t(ldt) * ldt, kBlock)), dim3(kBlock), 0, s, T.get(),
                       int64_t(ldt) * ldt);
    hipLaunchKernelGGL(k_thick_head, dim3(ceil_div(kp, 64)), dim3(64), 0, s, T.get(), ldt, kp, m, theta.get(), Y.get(),
                       beta.get(), m - 1);
    check_launch("thick restart");
    keep = kp;
    restarted = true;
    ++restarts;
    j = kp;
    m = kp;
}

hdm_status LanczosRun::result(double* evals, double* evecs, hdm_eig_info_t* info, hipStream_t s) {
    // Ritz values are descending by construction (k-th largest)
    if (evals)
        for (int i = 0; i < r; ++i) evals[i] = h_theta[i];
    double worst = 0.0;
    for (int i = 0; i < r; ++i) worst = std::max(worst, h_bound[i] / std::max(std::fabs(h_theta[i]), 1e-300));
    if (evecs) {
        const int gN = ceil_div(n, kBlock);
        hipLaunchKernelGGL(k_ritz, dim3(gN), dim3(kBlock), 0, s, V.get(), n, m, Y.get(), r, evecs, n, nullptr);
        DevBuf<double> scale(r);
        hipLaunchKernelGGL(k_col_stats, dim3(r), dim3(kBlock), 0, s, evecs, n, scale.get());
        hipLaunchKernelGGL(k_col_fix, dim3(std::min(gN, 256), r), dim3(kBlock), 0, s, evecs, n, scale.get());
        check_launch("ritz vectors");
        HDM_HIP(hipStreamSynchronize(s));
    }
    if (info) {
        info->iters = matvecs;   // steps taken, restarts included
        info->matvecs = matvecs;
        info->converged = converged ? 1 : 0;
        info->max_rel_resid = worst;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return converged ? HDM_OK : HDM_ENOCONV;
}

// Block Lanczos with b vectors per step (Sec. 2.2 with a block Krylov space):
// each step applies S~ to the b newest basis vectors at once (one product with
// b right-hand sides), reorthogonalises against the whole basis by classical
// Gram-Schmidt twice, and orthonormalises the block by shifted Cholesky QR
// three times (Fukaya et al., 2020), whose R is the next off-diagonal block
// B_j of the banded projected matrix T.  Every second step T is reduced to
// tridiagonal form by Householder reflections and solved like the
// single-vector case; Ritz pair i is accepted when ||B_j y_i[last b]|| <=
// tol |theta_i|.
static hdm_status block_lanczos_eigs(Op& op, int r, double tol, int b, int max_basis, uint64_t seed, double* evals,
                                     double* evecs, hdm_eig_info_t* info, hipStream_t s) {
    const int64_t n = op.n;
    HDM_CHECK(b >= 2 && b <= kMaxRhs && b <= n, HDM_EINVAL, "block must be in [2, min(16, n)]");
    HDM_CHECK(r >= 1 && r <= 64 && r <= n, HDM_EINVAL, "r must be in [1, min(64, n)]");
    int mb = max_basis <= 0 ? static_cast<int>(std::min<int64_t>(n, kMaxBlockBasis)) : max_basis;
    mb = static_cast<int>(std::min<int64_t>(mb, n));
    mb = mb / b * b;
    HDM_CHECK(mb >= r && mb >= b && mb <= kMaxBlockBasis, HDM_EINVAL,
              "max_basis must be in [max(r, block), 512] (rounded down to a multiple of block)");
    const auto t0 = std::chrono::steady_clock::now();
    const int ldt = mb + b;
    const int nbk = ceil_div(n, kGramRows);
    const int64_t ldp = static_cast<int64_t>(mb + b) * b;
    DevBuf<double> V(static_cast<size_t>(n) * (mb + b)), Y(static_cast<size_t>(n) * b), part(static_cast<size_t>(nbk) * ldp),
        H1(ldp), H2(ldp), G(b * b), Rinv(b * b), Rtot(b * b), T(static_cast<size_t>(ldt) * ldt),
        A(static_cast<size_t>(mb) * mb), dd(mb), ee(mb), tau(mb), theta(r), Z(static_cast<size_t>(r) * mb), bound(r);
    DevBuf<int> status(1);
    HDM_HIP(hipMemsetAsync(status.get(), 0, sizeof(int), s));
    HDM_HIP(hipMemsetAsync(T.get(), 0, T.bytes(), s));
    const int gN = ceil_div(n, kBlock);
    // Gram products X^T Y (ncols x b) over the basis or the block itself
    auto gram = [&](const double* X, int ncols, const double* Yp, double* out) {
        hipLaunchKernelGGL(k_gram_mma, dim3(nbk, ceil_div(ceil_div(ncols, 16), kGramTiles)), dim3(kBlock), 0, s, X, n,
                           ncols, Yp, n, b, n, part.get(), ldp);
        hipLaunchKernelGGL(k_reduce_cols, dim3(ceil_div(int64_t(ncols) * b, 64)), dim3(256), 0, s, part.get(), nbk,
                           static_cast<int>(ldp), ncols * b, out);
    };
    // shifted Cholesky QR three times, in place; Rtot = R3 R2 R1
    const double shift = 11.0 * (static_cast<double>(n) * b + static_cast<double>(b) * (b + 1)) * 1.1102230246251565e-16;
    auto block_qr = [&](double* X) {
        hipLaunchKernelGGL(k_eye, dim3(1), dim3(256), 0, s, Rtot.get(), b);
        for (int pass = 0; pass < 3; ++pass) {
            gram(X, b, X, G.get());
            hipLaunchKernelGGL(k_chol, dim3(1), dim3(256), 0, s, G.get(), b, pass == 0 ? shift : 0.0, Rinv.get(),
                               Rtot.get(), status.get());
            hipLaunchKernelGGL(k_trsm, dim3(gN), dim3(kBlock), 0, s, X, n, b, n, Rinv.get());
        }
    };
    // the basis lives in the tree's point order: the products neither gather nor
    // scatter, and the Ritz vectors are written back in the caller's order
    const int32_t* perm = op.perm.get();
    hipLaunchKernelGGL(k_start_block, dim3(ceil_div(n * b, kBlock)), dim3(kBlock), 0, s, V.get(), n, b, seed, perm);
    block_qr(V.get());
    check_launch("block lanczos start");
    std::vector<double> h_theta(r), h_bound(r);
    int m = 0, j = 0, since = 0, matvecs = 0;
    bool converged = false;
    for (;; ++j) {
        const double* Q = V.get() + static_cast<int64_t>(j) * b * n;
        apply(op, 1, false, Q, Y.get(), b, s, false, true);
        matvecs += b;
        const int nc = (j + 1) * b;
        {
            PhaseScope ph(op.ctx, HDM_PHASE_ORTHO, s);
            gram(V.get(), nc, Y.get(), H1.get());
            hipLaunchKernelGGL(k_gemmn, dim3(gN), dim3(kBlock), 0, s, V.get(), n, nc, H1.get(), Y.get(), n, b, n);
            gram(V.get(), nc, Y.get(), H2.get());
            hipLaunchKernelGGL(k_gemmn, dim3(gN), dim3(kBlock), 0, s, V.get(), n, nc, H2.get(), Y.get(), n, b, n);
            hipLaunchKernelGGL(k_add, dim3(ceil_div(int64_t(nc) * b, 256)), dim3(256), 0, s, H1.get(), H2.get(), nc * b);
            block_qr(Y.get());
            HDM_HIP(hipMemcpyAsync(V.get() + static_cast<int64_t>(j + 1) * b * n, Y.get(), sizeof(double) * n * b,
                                   hipMemcpyDeviceToDevice, s));
            hipLaunchKernelGGL(k_put_T, dim3(1), dim3(256), 0, s, T.get(), ldt, j, b, H1.get(), Rtot.get());
        }
        check_launch("block lanczos step");
        m = (j + 1) * b;
        ++since;
        const bool last = m + b > mb;
        // a check costs a dense reduction of the projected matrix and a host wait:
        // every second block step once the basis holds 2 r vectors (r Ritz pairs
        // rarely meet the tolerance sooner; at N = 100000, r = 20, b = 16 this skips
        // the check at m = 32), and whenever the basis is full
        if ((m >= 2 * r && since >= 2 && (m / b) % 2 == 0) || (last && m >= r)) {
            since = 0;
            {
                KernelEvents ev(op.ctx, HDM_PHASE_TRIDIAG);
                launch_sytrd(T.get(), ldt, m, A.get(), mb, dd.get(), ee.get(), tau.get(), s, ev.start, ev.stop);
            }
            launch_tridiag(dd.get(), ee.get(), m, r, theta.get(), Z.get(), bound.get(), s);
            launch_ormtr(A.get(), mb, tau.get(), m, Z.get(), r, s);
            hipLaunchKernelGGL(k_block_bounds, dim3(1), dim3(64), 0, s, Z.get(), m, b, Rtot.get(), r, bound.get());
            check_launch("block rayleigh-ritz");
            int st = 0;
            download_parts({{&st, status.get(), sizeof(int)},
                            {h_theta.data(), theta.get(), r * sizeof(double)},
                            {h_bound.data(), bound.get(), r * sizeof(double)}},
                           s);
            HDM_CHECK(st == 0, HDM_ENUMERIC, "block Lanczos: the residual block lost rank (Cholesky QR failed)");
            bool ok = true;
            for (int i = 0; i < r; ++i) ok = ok && (h_bound[i] <= tol * std::fabs(h_theta[i]));
            if (ok) {
                converged = true;
                break;
            }
        }
        if (last) break;
    }
    if (m < r || h_theta.empty()) fail(HDM_EINTERNAL, "block Lanczos ended before a Rayleigh-Ritz step");
    for (int i = 0; i < r; ++i) evals[i] = h_theta[i];
    double worst = 0.0;
    for (int i = 0; i < r; ++i) worst = std::max(worst, h_bound[i] / std::max(std::fabs(h_theta[i]), 1e-300));
    if (evecs) {
        hipLaunchKernelGGL(k_ritz, dim3(gN), dim3(kBlock), 0, s, V.get(), n, m, Z.get(), r, evecs, n, perm);
        DevBuf<double> scale(r);
        hipLaunchKernelGGL(k_col_stats, dim3(r), dim3(kBlock), 0, s, evecs, n, scale.get());
        hipLaunchKernelGGL(k_col_fix, dim3(std::min(gN, 256), r), dim3(kBlock), 0, s, evecs, n, scale.get());
        check_launch("ritz vectors");
    }
    HDM_HIP(hipStreamSynchronize(s));
    if (info) {
        info->iters = m;
        info->matvecs = matvecs;
        info->converged = converged ? 1 : 0;
        info->max_rel_resid = worst;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return converged ? HDM_OK : HDM_ENOCONV;
}

hdm_status lanczos_eigs(Op& op, int r, double tol, int block, int max_basis, uint64_t seed, double* evals,
                        double* evecs, hdm_eig_info_t* info, hipStream_t s) {
    HDM_CHECK(block >= 1, HDM_EINVAL, "block must be >= 1");
    if (block > 1) return block_lanczos_eigs(op, r, tol, block, max_basis, seed, evals, evecs, info, s);
    LanczosRun run;
    run.start(op, r, tol, max_basis, seed, s);
    while (!run.finished) {
        apply(op, 1, false, run.current(), run.output(), 1, s);
        run.after_product(s);
    }
    return run.result(evals, evecs, info, s);
}

// ---- diffusion-map outputs (Alg. 1, last steps) ---------------------------------
// psi_k = phi_k / sqrt(d) (right eigenvectors of the Markov matrix from the
// eigenvectors of its symmetric conjugate) and the coordinates lambda_k^t psi_k,
// one thread per point (tree position p, original index perm[p])
struct PowT {
    double v[64];
};
__global__ void k_diffusion_coords(const double* phi, const double* d_tree, const int32_t* perm, int64_t n, int r,
                                   PowT lt, double* psi, double* coords) {
    const int64_t p = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (p >= n) return;
    const int64_t i = perm[p];
    const double s = 1.0 / sqrt(d_tree[p]);
    for (int k = 0; k < r; ++k) {
        const double v = phi[k * n + i] * s;
        if (psi) psi[k * n + i] = v;
        if (coords) coords[k * n + i] = lt.v[k] * v;
    }
}

hdm_status diffusion_map(Op& op, int r, const double* evals, const double* phi, int t, double delta, double* psi,
                         double* coords, double* evals_t, int32_t* dim_t, hipStream_t s) {
    HDM_CHECK(r >= 1 && r <= 64 && r <= op.n, HDM_EINVAL, "r must be in [1, min(64, n)]");
    HDM_CHECK(t >= 0, HDM_EINVAL, "t (random-walk steps) must be >= 0");
    HDM_CHECK(delta >= 0.0 && std::isfinite(delta), HDM_EINVAL, "delta must be finite and >= 0");
    HDM_CHECK((psi || coords) ? phi != nullptr : true, HDM_EINVAL, "phi is needed for psi or the coordinates");
    PowT lt{};
    for (int k = 0; k < r; ++k) {
        HDM_CHECK(std::isfinite(evals[k]), HDM_EINVAL, "eigenvalues must be finite");
        double p = 1.0;
        for (int j = 0; j < t; ++j) p *= evals[k];   // lambda^t of P^t, t steps of the walk
        lt.v[k] = p;
    }
    if (evals_t)
        for (int k = 0; k < r; ++k) evals_t[k] = lt.v[k];
    if (dim_t) {
        // max{l : |lambda_l|^t > delta |lambda_1|^t}, l counted from 1 (0 when none)
        int best = 0;
        for (int k = 0; k < r; ++k)
            if (std::fabs(lt.v[k]) > delta * std::fabs(lt.v[0])) best = k + 1;
        *dim_t = best;
    }
    if (psi || coords) {
        hipLaunchKernelGGL(k_diffusion_coords, dim3(ceil_div(op.n, kBlock)), dim3(kBlock), 0, s, phi, op.d.get(),
                           op.perm.get(), op.n, r, lt, psi, coords);
        check_launch("diffusion coordinates");
        HDM_HIP(hipStreamSynchronize(s));
    }
    return HDM_OK;
}

}  // namespace hdm
