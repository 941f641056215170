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

// partial[b][c] = sum over the block's rows of V[row, c] * y[row], c < ncols
__global__ void k_gemvt(const double* V, int64_t ldv, int ncols, const double* y, int64_t n, double* partial,
                        int ldp) {
    __shared__ double sm[kBlock / 64];
    const int64_t r0 = blockIdx.x * static_cast<int64_t>(kRows);
    double yr[kRows / kBlock];
#pragma unroll
    for (int u = 0; u < kRows / kBlock; ++u) {
        const int64_t row = r0 + u * kBlock + threadIdx.x;
        yr[u] = row < n ? y[row] : 0.0;
    }
    for (int c = 0; c < ncols; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < kRows / kBlock; ++u) {
            const int64_t row = r0 + u * kBlock + threadIdx.x;
            if (row < n) acc += V[c * ldv + row] * yr[u];
        }
        const double t = block_sum(acc, sm);
        if (threadIdx.x == 0) partial[static_cast<int64_t>(blockIdx.x) * ldp + c] = t;
    }
}

// h[c] = sum_b partial[b][c] (fixed order)
__global__ void k_reduce_cols(const double* partial, int nb, int ldp, int ncols, double* h) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncols) return;
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) acc += partial[static_cast<int64_t>(b) * ldp + c];
    h[c] = acc;
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

// One wave per requested eigenvalue (k-th largest, k < r): multisection of the
// Gershgorin interval with 64 Sturm counts per round, then inverse iteration
// (two steps, Gaussian elimination with partial pivoting of T - theta I) for
// the eigenvector.  Outputs theta[k], Y[:, k] (m entries, unit norm) and the
// residual bound |beta_last * Y[m-1, k]|.
__global__ void k_tridiag(const double* alpha, const double* beta, int m, int r, double* theta, double* Y,
                          double* bound, double* work) {
    __shared__ double a[1024], b2[1024], bb[1024];
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        a[i] = alpha[i];
        if (i + 1 < m) { b2[i] = beta[i] * beta[i]; bb[i] = beta[i]; }
    }
    __syncthreads();
    const int wv = threadIdx.x / 64, lane = threadIdx.x % 64, nw = blockDim.x / 64;
    // Gershgorin bounds
    double lo = INFINITY, hi = -INFINITY, amax = 0.0;
    for (int i = 0; i < m; ++i) {
        const double rad = (i > 0 ? fabs(bb[i - 1]) : 0.0) + (i + 1 < m ? fabs(bb[i]) : 0.0);
        lo = fmin(lo, a[i] - rad);
        hi = fmax(hi, a[i] + rad);
        amax = fmax(amax, fabs(a[i]) + rad);
    }
    const double tiny = 1e-300 + amax * 1e-300;
    for (int k = blockIdx.x * nw + wv; k < r; k += gridDim.x * nw) {
        const int target = m - 1 - k;   // index in ascending order
        double l = lo - 1e-12 * (fabs(lo) + 1.0), h = hi + 1e-12 * (fabs(hi) + 1.0);
        for (int round = 0; round < 12; ++round) {
            const double x = l + (h - l) * (lane + 1) / 65.0;
            const int c = sturm_below(a, b2, m, x, tiny);
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
        // inverse iteration on lane 0 (sequential tridiagonal elimination)
        if (lane == 0) {
            double* swp = work + static_cast<int64_t>(k) * 5 * m;   // 1: rows i, i+1 exchanged
            double* u0 = swp + m;   // U diagonal
            double* u1 = swp + 2 * m;
            double* u2 = swp + 3 * m;
            double* lmul = swp + 4 * m;
            const double shift_eps = 2.220446049250313e-16 * fmax(amax, 1e-300);
            // LU with partial pivoting of T - th I, rows i and i+1
            double d = a[0] - th, e = m > 1 ? bb[0] : 0.0, f = 0.0;
            for (int i = 0; i < m - 1; ++i) {
                const double sub = bb[i];
                const double dn = a[i + 1] - th, en = (i + 2 < m) ? bb[i + 1] : 0.0;
                if (fabs(d) >= fabs(sub)) {
                    const double piv_v = d == 0.0 ? shift_eps : d;
                    const double mult = sub / piv_v;
                    u0[i] = piv_v; u1[i] = e; u2[i] = f;
                    lmul[i] = mult;
                    d = dn - mult * e;
                    e = en - mult * 0.0;
                    f = 0.0;
                    swp[i] = 0.0;
                } else {
                    const double mult = d / sub;
                    u0[i] = sub; u1[i] = dn; u2[i] = en;
                    lmul[i] = mult;
                    d = e - mult * dn;
                    e = 0.0 - mult * en;
                    f = 0.0;
                    swp[i] = 1.0;
                }
            }
            u0[m - 1] = d == 0.0 ? shift_eps : d;
            // two solves with the same factors; start from the all-ones vector
            double* x = Y + static_cast<int64_t>(k) * m;
            for (int i = 0; i < m; ++i) x[i] = 1.0;
            for (int iter = 0; iter < 3; ++iter) {
                // forward elimination of the right-hand side
                for (int i = 0; i < m - 1; ++i) {
                    if (swp[i] != 0.0) { const double t = x[i]; x[i] = x[i + 1]; x[i + 1] = t; }
                    x[i + 1] -= lmul[i] * x[i];
                }
                // back substitution with U (bandwidth 2)
                for (int i = m - 1; i >= 0; --i) {
                    double v = x[i];
                    if (i + 1 < m) v -= u1[i] * x[i + 1];
                    if (i + 2 < m) v -= u2[i] * x[i + 2];
                    x[i] = v / u0[i];
                }
                double nrm = 0.0;
                for (int i = 0; i < m; ++i) nrm += x[i] * x[i];
                nrm = sqrt(nrm);
                for (int i = 0; i < m; ++i) x[i] /= nrm;
            }
            theta[k] = th;
            bound[k] = fabs(beta[m - 1] * x[m - 1]);
        }
    }
}

// Phi[:, k] = V Y[:, k] for k < r (rows per thread)
__global__ void k_ritz(const double* V, int64_t ldv, int m, const double* Y, int r, double* Phi, int64_t n) {
    __shared__ double ys[4096];
    const int tot = m * r;
    for (int e = threadIdx.x; e < tot && e < 4096; e += blockDim.x) ys[e] = Y[e];
    __syncthreads();
    const int64_t row = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (row >= n) return;
    for (int k = 0; k < r; ++k) {
        double acc = 0.0;
        for (int c = 0; c < m; ++c) acc += V[c * ldv + row] * (k * m + c < 4096 ? ys[k * m + c] : Y[k * m + c]);
        Phi[k * n + row] = acc;
    }
}

// per column: 2-norm and index of the largest |entry| (first on ties)
__global__ void k_col_stats(const double* Phi, int64_t n, double* nrm, int64_t* arg) {
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
        nrm[k] = sqrt(sn[0]);
        arg[k] = si[0];
    }
}

__global__ void k_col_fix(double* Phi, int64_t n, const double* nrm, const int64_t* arg) {
    const int k = blockIdx.y;
    const int64_t a = arg[k];
    const double sgn = (a >= 0 && a < n && Phi[k * n + a] < 0.0) ? -1.0 : 1.0;
    const double sc = sgn / nrm[k];
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        Phi[k * n + i] *= sc;
}

}  // namespace

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
    theta.alloc(r);
    bound.alloc(r);
    Y.alloc(static_cast<size_t>(r) * max_basis);
    work.alloc(static_cast<size_t>(r) * 5 * max_basis);
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
           beta.bytes() + theta.bytes() + bound.bytes() + Y.bytes() + work.bytes();
}

bool LanczosRun::after_product(hipStream_t s) {
    ++matvecs;
    const int nc = j + 1;
    {   // CGS2 against the whole basis, alpha_j, beta_j
        PhaseScope ph(op->ctx, HDM_PHASE_ORTHO, s);
        hipLaunchKernelGGL(k_gemvt, dim3(nb), dim3(kBlock), 0, s, V.get(), n, nc, y.get(), n, part.get(), ldp);
        hipLaunchKernelGGL(k_reduce_cols, dim3(ceil_div(nc, 64)), dim3(64), 0, s, part.get(), nb, ldp, nc, h1.get());
        hipLaunchKernelGGL(k_gemvn, dim3(nb), dim3(kBlock), 0, s, V.get(), n, nc, h1.get(), y.get(), n, nullptr);
        hipLaunchKernelGGL(k_gemvt, dim3(nb), dim3(kBlock), 0, s, V.get(), n, nc, y.get(), n, part.get(), ldp);
        hipLaunchKernelGGL(k_reduce_cols, dim3(ceil_div(nc, 64)), dim3(64), 0, s, part.get(), nb, ldp, nc, h2.get());
        hipLaunchKernelGGL(k_gemvn, dim3(nb), dim3(kBlock), 0, s, V.get(), n, nc, h2.get(), y.get(), n, np.get());
        hipLaunchKernelGGL(k_alpha_beta, dim3(1), dim3(1), 0, s, h1.get(), h2.get(), j, np.get(), nb, alpha.get(),
                           beta.get());
    }
    check_launch("lanczos step");
    m = j + 1;
    const bool last = (j == max_basis - 1);
    if (m >= r && ((m % check_every) == 0 || last)) {
        {
            KernelEvents ev(op->ctx, HDM_PHASE_TRIDIAG);
            hipExtLaunchKernelGGL(k_tridiag, dim3(ceil_div(r, 4)), dim3(kBlock), 0, s, ev.start, ev.stop, 0,
                                  alpha.get(), beta.get(), m, r, theta.get(), Y.get(), bound.get(), work.get());
        }
        check_launch("tridiagonal eigensolve");
        theta.download(h_theta.data(), r, s);
        bound.download(h_bound.data(), r, s);
        HDM_HIP(hipStreamSynchronize(s));
        bool ok = true;
        for (int i = 0; i < r; ++i) ok = ok && (h_bound[i] <= tol * std::fabs(h_theta[i]));
        if (ok) {
            converged = finished = true;
            return true;
        }
    }
    if (last) {
        finished = true;
        return true;
    }
    hipLaunchKernelGGL(k_next, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, y.get(), beta.get(), j,
                       V.get() + static_cast<int64_t>(j + 1) * n, n);
    ++j;
    return false;
}

hdm_status LanczosRun::result(double* evals, double* evecs, hdm_eig_info_t* info, hipStream_t s) {
    // Ritz values are descending by construction (k-th largest)
    if (evals)
        for (int i = 0; i < r; ++i) evals[i] = h_theta[i];
    double worst = 0.0;
    for (int i = 0; i < r; ++i) worst = std::max(worst, h_bound[i] / std::max(std::fabs(h_theta[i]), 1e-300));
    if (evecs) {
        const int gN = ceil_div(n, kBlock);
        hipLaunchKernelGGL(k_ritz, dim3(gN), dim3(kBlock), 0, s, V.get(), n, m, Y.get(), r, evecs, n);
        DevBuf<double> nrm(r);
        DevBuf<int64_t> arg(r);
        hipLaunchKernelGGL(k_col_stats, dim3(r), dim3(kBlock), 0, s, evecs, n, nrm.get(), arg.get());
        hipLaunchKernelGGL(k_col_fix, dim3(std::min(gN, 256), r), dim3(kBlock), 0, s, evecs, n, nrm.get(), arg.get());
        check_launch("ritz vectors");
        HDM_HIP(hipStreamSynchronize(s));
    }
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
    HDM_CHECK(block == 1, HDM_EINVAL, "only block = 1 is supported by this build");
    LanczosRun run;
    run.start(op, r, tol, max_basis, seed, s);
    while (!run.finished) {
        apply(op, 1, false, run.current(), run.output(), 1, s);
        run.after_product(s);
    }
    return run.result(evals, evecs, info, s);
}

}  // namespace hdm
