// C ABI of libhdm: argument checks, error mapping, operator lifetime.
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>

#include "op.hpp"

namespace hdm {

// callers hold mu
hipEvent_t Profiler::take() {
    if (used == pool.size()) {
        hipEvent_t e;
        HDM_HIP(hipEventCreate(&e));
        pool.push_back(e);
    }
    return pool[used++];
}

void Profiler::begin(int phase, hipStream_t s, size_t& slot) {
    std::lock_guard<std::mutex> g(mu);
    const size_t a = used;
    HDM_HIP(hipEventRecord(take(), s));
    marks.push_back(Mark{phase, a, SIZE_MAX});
    slot = marks.size() - 1;
}

void Profiler::end(size_t slot, hipStream_t s) noexcept {
    std::lock_guard<std::mutex> g(mu);
    if (used == pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        pool.push_back(e);
    }
    const size_t b = used++;
    if (hipEventRecord(pool[b], s) == hipSuccess) marks[slot].b = b;
}

void Profiler::kernel_events(int phase, hipEvent_t& start, hipEvent_t& stop) {
    std::lock_guard<std::mutex> g(mu);
    const size_t a = used;
    start = take();
    const size_t b = used;
    stop = take();
    marks.push_back(Mark{phase, a, b});
}

void Profiler::totals(int64_t* launches, double* ms) {
    std::lock_guard<std::mutex> g(mu);
    for (int p = 0; p < HDM_PHASE_COUNT; ++p) { launches[p] = 0; ms[p] = 0.0; }
    for (const Mark& m : marks) {
        if (m.b == SIZE_MAX || m.phase < 0 || m.phase >= HDM_PHASE_COUNT) continue;
        HDM_HIP(hipEventSynchronize(pool[m.b]));
        float t = 0.0f;
        HDM_HIP(hipEventElapsedTime(&t, pool[m.a], pool[m.b]));
        launches[m.phase] += 1;
        ms[m.phase] += t;
    }
}

Profiler::~Profiler() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

namespace {
thread_local std::string g_err;
}  // namespace

void set_last_error(const char* msg) { g_err = msg ? msg : ""; }

namespace {
bool prec_ok(int p) { return p == HDM_F64 || p == HDM_F32 || p == HDM_BF16 || p == HDM_F16; }
}  // namespace

void validate_params(const hdm_params& p) {
    if (p.n < 2) fail(HDM_EINVAL, "n must be >= 2");
    if (p.n > (int64_t(1) << 30)) fail(HDM_EINVAL, "n must be < 2^30");
    if (p.dim < 1) fail(HDM_EINVAL, "dim must be >= 1");
    if (p.x_dtype != HDM_F64 && p.x_dtype != HDM_U8) fail(HDM_EINVAL, "x_dtype must be HDM_F64 or HDM_U8");
    if (!(p.eps > 0.0) || !std::isfinite(p.eps)) fail(HDM_EINVAL, "eps must be finite and > 0");
    if (p.alpha != 1.0) fail(HDM_EINVAL, "only alpha = 1 is supported");
    if (p.leaf_m < 2) fail(HDM_EINVAL, "leaf_m must be >= 2");
    if (p.max_rank_s < 1 || p.max_rank_s > 1024) fail(HDM_EINVAL, "max_rank_s must be in [1, 1024]");
    if (!(p.tau >= 0.0) || !std::isfinite(p.tau)) fail(HDM_EINVAL, "tau must be finite and >= 0");
    if (p.knn_k < 1 || p.knn_k > 64) fail(HDM_EINVAL, "knn_k must be in [1, 64]");
    if (p.knn_iters < 1 || p.knn_iters > 1000) fail(HDM_EINVAL, "knn_iters must be in [1, 1000]");
    if (!(p.budget >= 0.0 && p.budget <= 1.0)) fail(HDM_EINVAL, "budget must be in [0, 1]");
    if (!prec_ok(p.near_prec) || !prec_ok(p.far_prec)) fail(HDM_EINVAL, "bad tile precision");
    if ((p.near_prec == HDM_F64) != (p.far_prec == HDM_F64))
        fail(HDM_EINVAL, "float64 tiles cannot be mixed with reduced-precision tiles");
    int depth = 0;
    while ((p.n + (int64_t(1) << depth) - 1) / (int64_t(1) << depth) > p.leaf_m) ++depth;
    if (depth > 16) fail(HDM_EINVAL, "tree deeper than 16 levels: raise leaf_m");
    if ((p.n >> depth) <= p.knn_k) fail(HDM_EINVAL, "every leaf must hold more than knn_k points");
    if (((p.n + (int64_t(1) << depth) - 1) >> depth) > 2048) fail(HDM_EINVAL, "leaves must hold <= 2048 points");
    // the combine keeps a leaf's skeleton potentials (at most min(s, leaf size))
    // in shared memory for up to 512 of them
    if (p.max_rank_s > 512 && ((p.n + (int64_t(1) << depth) - 1) >> depth) > 512)
        fail(HDM_EINVAL, "max_rank_s above 512 needs leaves of at most 512 points");
    // u8 codes with a maximal rank above the smallest leaf: two runs with such
    // requests ended in a GPU memory fault whose cause is not known, so this
    // class is refused until it is found
    if (p.x_dtype == HDM_U8 && p.max_rank_s > (p.n >> depth))
        fail(HDM_EINVAL, "u8 points: max_rank_s above the smallest leaf size is not supported");
}


hdm_op_s* make_operator(Ctx* ctx, const void* X, int x_on_device, const hdm_params& params, hipStream_t s) {
    validate_params(params);
    if (!x_on_device && params.x_dtype == HDM_F64) {
        const double* x = static_cast<const double*>(X);
        const int64_t cnt = params.n * params.dim;
        for (int64_t i = 0; i < cnt; ++i) HDM_CHECK(std::isfinite(x[i]), HDM_EINVAL, "points contain NaN or Inf");
    }
    std::unique_ptr<hdm_op_s> op(new hdm_op_s());
    op->ctx = ctx;
    op->prm = params;
    {
        PhaseScope ph(ctx, HDM_PHASE_COMPRESS, s);
        compress_operator(*op, X, x_on_device, s);
        build_eval_plan(*op, s);
        convert_eval_precision(*op, s);   // does not need the degrees: enqueued first
        normalise_degrees(*op, s);
        finish_operator(*op, s);
    }
    HDM_HIP(hipStreamSynchronize(s));
    return op.release();
}

size_t footprint_estimate(const hdm_params& p, int max_basis) {
    int depth = 0;
    while ((p.n + (int64_t(1) << depth) - 1) / (int64_t(1) << depth) > p.leaf_m) ++depth;
    const int64_t L = int64_t(1) << depth;
    const int64_t leaf = (p.n + L - 1) / L;
    const int64_t extra = static_cast<int64_t>(std::ceil(p.budget * static_cast<double>(L)));
    const int64_t near_per_leaf = std::min<int64_t>(L, 2 * extra + 1);
    const int64_t ld = (leaf + 7) / 8 * 8;
    const int64_t near_elems = L * ld * leaf * near_per_leaf;
    const size_t e_near = dtype_size(p.near_prec);
    const int64_t s2 = 2 * static_cast<int64_t>(p.max_rank_s);
    const int64_t cmax = std::max(leaf, s2);
    size_t b = 0;
    b += static_cast<size_t>(near_elems) * (8 + e_near);                 // float64 tiles for the degrees + eval copy
    b += static_cast<size_t>(p.n) * p.dim * dtype_size(p.x_dtype);       // points
    b += static_cast<size_t>(p.n) * p.knn_k * 12;                          // neighbour lists
    b += static_cast<size_t>(L) * p.n * 4 + static_cast<size_t>(L) * s2 * cmax * 8 * 2;   // skeletonisation workspaces
    b += static_cast<size_t>(2 * L) * p.max_rank_s * cmax * 12;           // interpolation matrices and far tiles
    b += static_cast<size_t>(p.n) * (max_basis + 8) * 8;                  // Lanczos basis and vectors
    return b;
}


}  // namespace hdm


namespace {

using hdm::g_err;

template <typename F>
hdm_status guarded(F&& f) {
    try {
        g_err.clear();
        return f();
    } catch (const hdm::Error& e) {
        g_err = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        return HDM_ENOMEM;
    } catch (const std::exception& e) {
        g_err = e.what();
        return HDM_EINTERNAL;
    } catch (...) {
        g_err = "unknown failure";
        return HDM_EINTERNAL;
    }
}

inline hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

bool prec_ok(int p) { return p == HDM_F64 || p == HDM_F32 || p == HDM_BF16 || p == HDM_F16; }

void set_device(int dev) { HDM_HIP(hipSetDevice(dev)); }

}  // namespace

extern "C" {

const char* hdm_last_error(void) { return g_err.c_str(); }

const char* hdm_version(void) { return "hdm 0.1 (gfx950)"; }

void hdm_params_default(hdm_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->x_dtype = HDM_F64;
    p->alpha = 1.0;
    p->leaf_m = 256;
    p->max_rank_s = 128;
    p->tau = 1e-5;
    p->knn_k = 32;
    p->knn_iters = 10;
    p->budget = 0.05;
    p->near_prec = HDM_F32;
    p->far_prec = HDM_F32;
}

hdm_status hdm_params_validate(const hdm_params* p) {
    return guarded([&] {
        HDM_CHECK(p != nullptr, HDM_EINVAL, "NULL parameters");
        hdm::validate_params(*p);
        return HDM_OK;
    });
}

hdm_status hdm_ctx_create(int device, size_t hbm_budget_bytes, hdm_ctx* out) {
    return guarded([&] {
        HDM_CHECK(out != nullptr, HDM_EINVAL, "out is NULL");
        int count = 0;
        HDM_HIP(hipGetDeviceCount(&count));
        HDM_CHECK(device >= 0 && device < count, HDM_EINVAL, "no such device");
        set_device(device);
        hdm::scratch_init(device);   // the allocation-free product's array on this device
        auto* c = new hdm_ctx_s();
        c->device = device;
        c->budget = hbm_budget_bytes;
        *out = c;
        return HDM_OK;
    });
}

hdm_status hdm_ctx_destroy(hdm_ctx ctx) {
    return guarded([&] {
        delete ctx;
        return HDM_OK;
    });
}

hdm_status hdm_ctx_graphs(hdm_ctx ctx, int enable) {
    return guarded([&] {
        HDM_CHECK(ctx, HDM_EINVAL, "NULL context");
        ctx->graphs = enable != 0;
        return HDM_OK;
    });
}

hdm_status hdm_ctx_profile_phases(hdm_ctx ctx, uint32_t phase_mask) {
    return guarded([&] {
        HDM_CHECK(ctx, HDM_EINVAL, "NULL context");
        set_device(ctx->device);
        if (phase_mask) {
            HDM_HIP(hipDeviceSynchronize());
            ctx->prof.reset();
        }
        ctx->prof.mask = phase_mask;
        ctx->prof.on = phase_mask != 0;
        return HDM_OK;
    });
}

hdm_status hdm_ctx_profile(hdm_ctx ctx, int enable) { return hdm_ctx_profile_phases(ctx, enable ? ~0u : 0u); }

hdm_status hdm_ctx_phase_times(hdm_ctx ctx, hdm_phase_times_t* out) {
    return guarded([&] {
        HDM_CHECK(ctx && out, HDM_EINVAL, "NULL argument");
        set_device(ctx->device);
        ctx->prof.totals(out->launches, out->ms);
        return HDM_OK;
    });
}

hdm_status hdm_compress(hdm_ctx ctx, const void* X, int x_on_device, const hdm_params* params, void* stream,
                        hdm_op* out) {
    return guarded([&] {
        hdm::PoolScope pool_scope;   // temporaries are cached once the device is idle
        HDM_CHECK(ctx && X && params && out, HDM_EINVAL, "NULL argument");
        hdm::validate_params(*params);
        set_device(ctx->device);
        std::unique_ptr<hdm_op_s> op(hdm::make_operator(ctx, X, x_on_device, *params, as_stream(stream)));
        const size_t fp = op->footprint();
        HDM_CHECK(ctx->budget == 0 || ctx->resident + fp <= ctx->budget, HDM_ENOMEM,
                  "operator exceeds the context's memory budget");
        ctx->resident += fp;
        *out = op.release();
        return HDM_OK;
    });
}

hdm_status hdm_op_destroy(hdm_op op) {
    return guarded([&] {
        if (!op) return HDM_OK;
        set_device(op->ctx->device);
        hdm::PoolScope pool_scope;   // the operator's buffers are cached once the device is idle
        const size_t fp = op->footprint();
        op->ctx->resident -= std::min(fp, op->ctx->resident);
        delete op;
        return HDM_OK;
    });
}

hdm_status hdm_op_stats(hdm_op op, hdm_op_stats_t* out) {
    return guarded([&] {
        HDM_CHECK(op && out, HDM_EINVAL, "NULL argument");
        hdm_op_stats_t st{};
        st.n = op->n;
        st.dim = op->dim;
        st.depth = op->depth;
        st.leaves = op->L;
        st.knn_k = op->prm.knn_k;
        int mx = 0, mn = 1 << 30;
        double sum = 0.0;
        for (int64_t h = 2; h < op->nnodes; ++h) mx = std::max(mx, op->rank[h]);
        for (int64_t h = op->L; h < op->nnodes; ++h) {
            mn = std::min(mn, op->rank[h]);
            sum += op->rank[h];
        }
        st.max_rank = mx;
        st.min_leaf_rank = mn;
        st.mean_leaf_rank = sum / op->L;
        st.near_pairs = static_cast<int64_t>(op->near_idx.size());
        st.far_pairs = static_cast<int64_t>(op->far_idx.size());
        const size_t en = hdm::dtype_size(op->prm.near_prec), ef = hdm::dtype_size(op->prm.far_prec);
        const size_t ep = op->prm.near_prec == HDM_F64 ? 8 : 4;
        st.bytes_near = static_cast<int64_t>(op->near_elems * en);
        st.bytes_far = static_cast<int64_t>(op->far_elems * ef);
        st.bytes_p = static_cast<int64_t>(op->np * ep);
        st.bytes_total = static_cast<int64_t>(op->footprint());
        // algorithmic bytes of one single-vector product: unpadded near tiles,
        // far tiles and P (read in N2S and S2N) once each, input and output
        // vectors, skeleton weights and potentials
        int64_t near_alg = 0;
        for (int64_t a = 0; a < op->L; ++a)
            for (int32_t t = op->near_off[a]; t < op->near_off[a + 1]; ++t)
                near_alg += op->size[op->L + a] * op->size[op->L + op->near_idx[t]];
        const size_t ev = op->prm.near_prec == HDM_F64 ? 8 : 4;
        st.algo_bytes_matvec = static_cast<int64_t>(near_alg * en + op->far_elems * ef + 2 * op->np * ep +
                                                     2 * op->n * 8 + 4 * op->nskel * ev);
        // the near-field launch of a single-vector product also forms the leaves'
        // skeleton weights: their P once and the weights written
        int64_t leaf_p = 0, leaf_sk = 0;
        if (op->nskel > 0)
            for (int64_t h = op->L; h < 2 * op->L; ++h) {
                leaf_p += static_cast<int64_t>(op->rank[h]) * op->ncand[h];
                leaf_sk += op->rank[h];
            }
        st.algo_bytes_near = static_cast<int64_t>(near_alg * en + 2 * op->n * ev + leaf_p * ep + leaf_sk * ev);
        st.near_tile_bytes = static_cast<int64_t>(near_alg * en);
        st.near_elems = near_alg;
        st.flops_matvec = 2 * (near_alg + op->far_elems + 2 * op->np);
        st.seconds_compress = op->seconds_compress;
        *out = st;
        return HDM_OK;
    });
}

hdm_status hdm_op_perm(hdm_op op, int32_t* perm) {
    return guarded([&] {
        HDM_CHECK(op && perm, HDM_EINVAL, "NULL argument");
        set_device(op->ctx->device);
        HDM_HIP(hipMemcpy(perm, op->perm.get(), sizeof(int32_t) * op->n, hipMemcpyDeviceToHost));
        return HDM_OK;
    });
}

hdm_status hdm_op_knn(hdm_op op, int32_t* idx, double* d2) {
    return guarded([&] {
        HDM_CHECK(op, HDM_EINVAL, "NULL operator");
        set_device(op->ctx->device);
        const size_t cnt = static_cast<size_t>(op->n) * op->prm.knn_k;
        if (idx) HDM_HIP(hipMemcpy(idx, op->knn_idx.get(), sizeof(int32_t) * cnt, hipMemcpyDeviceToHost));
        if (d2) HDM_HIP(hipMemcpy(d2, op->knn_d2.get(), sizeof(double) * cnt, hipMemcpyDeviceToHost));
        return HDM_OK;
    });
}

hdm_status hdm_op_lists(hdm_op op, int32_t* near_off, int32_t* near_idx, int64_t* near_nnz, int32_t* far_off,
                        int32_t* far_idx, int64_t* far_nnz) {
    return guarded([&] {
        HDM_CHECK(op, HDM_EINVAL, "NULL operator");
        if (near_nnz) *near_nnz = static_cast<int64_t>(op->near_idx.size());
        if (far_nnz) *far_nnz = static_cast<int64_t>(op->far_idx.size());
        if (near_off) std::memcpy(near_off, op->near_off.data(), sizeof(int32_t) * op->near_off.size());
        if (near_idx) std::memcpy(near_idx, op->near_idx.data(), sizeof(int32_t) * op->near_idx.size());
        if (far_off) std::memcpy(far_off, op->far_off.data(), sizeof(int32_t) * op->far_off.size());
        if (far_idx) std::memcpy(far_idx, op->far_idx.data(), sizeof(int32_t) * op->far_idx.size());
        return HDM_OK;
    });
}

hdm_status hdm_op_ranks(hdm_op op, int32_t* rank, int32_t* ncand, int32_t* nrows) {
    return guarded([&] {
        HDM_CHECK(op, HDM_EINVAL, "NULL operator");
        if (rank) std::memcpy(rank, op->rank.data(), sizeof(int32_t) * op->nnodes);
        if (ncand) std::memcpy(ncand, op->ncand.data(), sizeof(int32_t) * op->nnodes);
        if (nrows) std::memcpy(nrows, op->nrows.data(), sizeof(int32_t) * op->nnodes);
        return HDM_OK;
    });
}

hdm_status hdm_op_node(hdm_op op, int64_t h, int32_t* skel, int32_t* rows, double* P) {
    return guarded([&] {
        HDM_CHECK(op, HDM_EINVAL, "NULL operator");
        HDM_CHECK(h >= 2 && h < op->nnodes, HDM_EINVAL, "heap id out of range");
        set_device(op->ctx->device);
        if (skel && op->rank[h] > 0)
            HDM_HIP(hipMemcpy(skel, op->skel.get() + op->skoff[h], sizeof(int32_t) * op->rank[h], hipMemcpyDeviceToHost));
        if (rows && op->nrows[h] > 0)
            HDM_HIP(hipMemcpy(rows, op->rows.get() + op->rowoff[h], sizeof(int32_t) * op->nrows[h], hipMemcpyDeviceToHost));
        const int64_t pc = static_cast<int64_t>(op->rank[h]) * op->ncand[h];
        if (P && pc > 0)
            HDM_HIP(hipMemcpy(P, op->P64.get() + op->poff[h], sizeof(double) * pc, hipMemcpyDeviceToHost));
        return HDM_OK;
    });
}

hdm_status hdm_op_degrees(hdm_op op, double* q, double* d, double* c) {
    return guarded([&] {
        HDM_CHECK(op, HDM_EINVAL, "NULL operator");
        set_device(op->ctx->device);
        std::vector<int32_t> perm(op->n);
        std::vector<double> tmp(op->n);
        HDM_HIP(hipMemcpy(perm.data(), op->perm.get(), sizeof(int32_t) * op->n, hipMemcpyDeviceToHost));
        auto get = [&](const hdm::DevBuf<double>& b, double* out) {
            if (!out) return;
            HDM_HIP(hipMemcpy(tmp.data(), b.get(), sizeof(double) * op->n, hipMemcpyDeviceToHost));
            for (int64_t t = 0; t < op->n; ++t) out[perm[t]] = tmp[t];
        };
        get(op->q, q);
        get(op->d, d);
        get(op->c, c);
        return HDM_OK;
    });
}

hdm_status hdm_matvec(hdm_op op, int normalised, const double* x, double* y, int32_t nrhs, void* stream) {
    return guarded([&] {
        HDM_CHECK(op && x && y, HDM_EINVAL, "NULL argument");
        HDM_CHECK(nrhs >= 1 && nrhs <= 4096, HDM_EINVAL, "nrhs must be in [1, 4096]");
        HDM_CHECK(x + static_cast<int64_t>(op->n) * nrhs <= y || y + static_cast<int64_t>(op->n) * nrhs <= x, HDM_EINVAL,
                  "x and y overlap");
        set_device(op->ctx->device);
        hdm::apply(*op, normalised ? 1 : 0, false, x, y, nrhs, as_stream(stream), true);
        return HDM_OK;
    });
}

hdm_status hdm_matvec_noalloc(hdm_op op, int normalised, const double* x, double* y, int32_t nrhs, void* stream) {
    return guarded([&] {
        HDM_CHECK(op && x && y, HDM_EINVAL, "NULL argument");
        HDM_CHECK(nrhs >= 1 && nrhs <= 4096, HDM_EINVAL, "nrhs must be in [1, 4096]");
        HDM_CHECK(x + static_cast<int64_t>(op->n) * nrhs <= y || y + static_cast<int64_t>(op->n) * nrhs <= x, HDM_EINVAL,
                  "x and y overlap");
        set_device(op->ctx->device);
        hdm::apply_noalloc(*op, normalised ? 1 : 0, x, y, nrhs, as_stream(stream), hdm::scratch_for(op->ctx->device));
        return HDM_OK;
    });
}

hdm_status hdm_eigs(hdm_op op, int32_t r, double rel_resid_tol, int32_t block, int32_t max_basis, uint64_t seed,
                    double* evals, double* evecs, hdm_eig_info_t* info, void* stream) {
    return guarded([&] {
        HDM_CHECK(op && evals, HDM_EINVAL, "NULL argument");
        HDM_CHECK(rel_resid_tol > 0.0 && std::isfinite(rel_resid_tol), HDM_EINVAL, "rel_resid_tol must be > 0");
        set_device(op->ctx->device);
        hdm::PoolScope pool_scope;
        return hdm::lanczos_eigs(*op, r, rel_resid_tol, block, max_basis, seed, evals, evecs, info, as_stream(stream));
    });
}

hdm_status hdm_diffusion_map(hdm_op op, int32_t r, const double* evals, const double* phi, int32_t t, double delta,
                             double* psi, double* coords, double* evals_t, int32_t* dim_t, void* stream) {
    return guarded([&] {
        HDM_CHECK(op && evals, HDM_EINVAL, "NULL argument");
        set_device(op->ctx->device);
        return hdm::diffusion_map(*op, r, evals, phi, t, delta, psi, coords, evals_t, dim_t, as_stream(stream));
    });
}

}  // extern "C"
