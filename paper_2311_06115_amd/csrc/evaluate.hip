// Evaluation of the compressed operator K~ = D + S + UV (Eq. (3)) and of the
// alpha = 1 normalised operator S~ x = c * K~ (c * x) (Alg. 1), once per Lanczos
// step.  Phases, all owner-computes with fixed reduction order (deterministic):
//   N2S  upward:   skeleton weights  w~_h = P_h w_h (leaf), P_h [w~_l; w~_r]
//   S2S  far:      skeleton potentials u~_h = sum_{g in Far(h)} K(skel_h, skel_g) w~_g
//   S2N  downward: [u~_l; u~_r] += P_h^T u~_h; leaves fold P^T u~ into the output
//   L2L  near:     u_a += sum_{b in Near(a)} K(a, b) w_b   (streams the near tiles)
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "op.hpp"

namespace hdm {

namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kChunk = 64;    // columns per near-field work item

// ---- element types --------------------------------------------------------
struct bf16_t { uint16_t v; };
struct f16_t { _Float16 v; };

__device__ __host__ inline float to_f(double x) { return static_cast<float>(x); }
__device__ inline float to_f(float x) { return x; }
__device__ inline float to_f(bf16_t x) { return __uint_as_float(static_cast<uint32_t>(x.v) << 16); }
__device__ inline float to_f(f16_t x) { return static_cast<float>(x.v); }
__device__ inline double to_d(double x) { return x; }
__device__ inline double to_d(float x) { return x; }

template <typename T>
__device__ inline T from_d(double x);
template <>
__device__ inline double from_d<double>(double x) { return x; }
template <>
__device__ inline float from_d<float>(double x) { return static_cast<float>(x); }
template <>
__device__ inline bf16_t from_d<bf16_t>(double x) {
    // round to nearest even on the float32 bit pattern
    const uint32_t u = __float_as_uint(static_cast<float>(x));
    const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
    return bf16_t{static_cast<uint16_t>(r >> 16)};
}
template <>
__device__ inline f16_t from_d<f16_t>(double x) { return f16_t{static_cast<_Float16>(static_cast<float>(x))}; }

// value of a stored tile element in the accumulation type A
template <typename A, typename T>
__device__ inline A val(T x) { return static_cast<A>(to_f(x)); }
template <>
__device__ inline double val<double, double>(double x) { return x; }

// deterministic wave sum (butterfly)
template <typename A>
__device__ inline A wave_sum(A v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// ---- vector staging ------------------------------------------------------
template <typename V>
__global__ void k_prep(int64_t n, int nrhs, const double* x, const int32_t* perm, const double* scale, V* w) {
    const int64_t pos = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (pos >= n) return;
    const int32_t i = perm[pos];
    const double sc = scale ? scale[pos] : 1.0;
    for (int c = 0; c < nrhs; ++c) w[c * n + pos] = static_cast<V>(sc * x[c * n + i]);
}

// ---- dot products of one row per wave (lanes stride the columns) -------------
template <typename V, typename TM, typename GX>
__device__ inline V row_dot(const TM* row, int nc, GX x) {
    const int lane = threadIdx.x % kWave;
    V acc = 0;
    int j = lane;
    for (; j + 3 * kWave < nc; j += 4 * kWave) {
        const TM p0 = row[j], p1 = row[j + kWave], p2 = row[j + 2 * kWave], p3 = row[j + 3 * kWave];
        const V x0 = x(j), x1 = x(j + kWave), x2 = x(j + 2 * kWave), x3 = x(j + 3 * kWave);
        acc += val<V>(p0) * x0;
        acc += val<V>(p1) * x1;
        acc += val<V>(p2) * x2;
        acc += val<V>(p3) * x3;
    }
    for (; j < nc; j += kWave) acc += val<V>(row[j]) * x(j);
    return wave_sum(acc);
}

// ---- N2S: one level of skeleton weights, one wave per (node, row) -------------
//   leaf:  w~_h = P_h w_h;   inner: w~_h = P_h [w~_left; w~_right]
template <typename V, typename TP>
__global__ void k_n2s(const RowTask* tasks, int64_t ntask, int leaf, const int64_t* start, const int32_t* ncand,
                      const int64_t* skoff, const int64_t* poff, const TP* P, const V* w, int64_t ldw, V* skw,
                      int64_t ldsk, int nrhs) {
    const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x / kWave) + threadIdx.x / kWave;
    if (t >= ntask) return;
    const RowTask T = tasks[t];
    const int nc = ncand[T.h];
    const TP* row = P + poff[T.h] + static_cast<int64_t>(T.i) * nc;
    for (int c = 0; c < nrhs; ++c) {
        const V* in = leaf ? w + c * ldw + start[T.h] : skw + c * ldsk + skoff[2 * T.h];
        const V acc = row_dot<V>(row, nc, [&](int j) { return in[j]; });
        if (threadIdx.x % kWave == 0) skw[c * ldsk + skoff[T.h] + T.i] = acc;
    }
}

// ---- S2S: far field between skeletons, one wave per (node, row) -----------------
template <typename V, typename TF>
__global__ void k_s2s(const RowTask* tasks, int64_t ntask, const int64_t* skoff, const int64_t* boff,
                      const int32_t* cols, const int64_t* colbase, const int32_t* colmap, const TF* far,
                      const float* fscale, const V* skw, V* sku, int64_t ldsk, int nrhs) {
    const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x / kWave) + threadIdx.x / kWave;
    if (t >= ntask) return;
    const RowTask T = tasks[t];
    const int nc = cols[T.h];
    const TF* row = far + boff[T.h] + static_cast<int64_t>(T.i) * nc;
    const int32_t* cm = colmap + colbase[T.h];
    const V sc = fscale ? static_cast<V>(fscale[T.h]) : V(1);
    for (int c = 0; c < nrhs; ++c) {
        const V* x = skw + c * ldsk;
        const V acc = row_dot<V>(row, nc, [&](int j) { return x[cm[j]]; });
        if (threadIdx.x % kWave == 0) sku[c * ldsk + skoff[T.h] + T.i] = acc * sc;
    }
}

// ---- L2L: stream the near tiles; one wave per work item ---------------------
// Lane l owns RPL consecutive rows (16 bytes of tile per lane per column) of
// each 64*RPL-row pass over the item's rows; the item's columns are consecutive
// tree positions, so w is read as a wave-uniform value.
template <typename V, typename TN>
__global__ void __launch_bounds__(kBlock) k_l2l(const NearItem* items, int64_t nitems, const TN* tiles,
                                                const float* tscale, const V* w, int64_t ldw, V* part,
                                                int64_t ldp, int nrhs) {
    constexpr int RPL = 16 / sizeof(TN);
    const int64_t it = blockIdx.x * static_cast<int64_t>(blockDim.x / kWave) + threadIdx.x / kWave;
    if (it >= nitems) return;
    const NearItem I = items[it];
    const int lane = threadIdx.x % kWave;
    const int rend = min(I.ld, I.row0 + I.nrows);
    const V sc = tscale ? static_cast<V>(tscale[I.tile]) : V(1);
    for (int c = 0; c < nrhs; ++c) {
        const V* wc = w + c * ldw + I.col_pos;
        for (int r0 = I.row0; r0 < rend; r0 += kWave * RPL) {
            const int row = r0 + lane * RPL;
            if (row >= rend) continue;
            V acc[RPL];
#pragma unroll
            for (int r = 0; r < RPL; ++r) acc[r] = 0;
            const TN* col = tiles + I.tile_off + row;
            int j = 0;
            for (; j + 4 <= I.ncols; j += 4) {
                TN v0[RPL], v1[RPL], v2[RPL], v3[RPL];
                __builtin_memcpy(v0, col + static_cast<int64_t>(j) * I.ld, sizeof(v0));
                __builtin_memcpy(v1, col + static_cast<int64_t>(j + 1) * I.ld, sizeof(v1));
                __builtin_memcpy(v2, col + static_cast<int64_t>(j + 2) * I.ld, sizeof(v2));
                __builtin_memcpy(v3, col + static_cast<int64_t>(j + 3) * I.ld, sizeof(v3));
                const V w0 = wc[j] * sc, w1 = wc[j + 1] * sc, w2 = wc[j + 2] * sc, w3 = wc[j + 3] * sc;
#pragma unroll
                for (int r = 0; r < RPL; ++r) {
                    acc[r] += val<V>(v0[r]) * w0;
                    acc[r] += val<V>(v1[r]) * w1;
                    acc[r] += val<V>(v2[r]) * w2;
                    acc[r] += val<V>(v3[r]) * w3;
                }
            }
            for (; j < I.ncols; ++j) {
                TN v0[RPL];
                __builtin_memcpy(v0, col + static_cast<int64_t>(j) * I.ld, sizeof(v0));
                const V w0 = wc[j] * sc;
#pragma unroll
                for (int r = 0; r < RPL; ++r) acc[r] += val<V>(v0[r]) * w0;
            }
            V* out = part + c * ldp + I.part_off + row;
#pragma unroll
            for (int r = 0; r < RPL; ++r) out[r] = acc[r];
        }
    }
}

// ---- combine: downward pass, near partial sums, scale, scatter ---------------
// One workgroup per leaf.  It walks the leaf's ancestors top-down,
//   u~_child = S2S(child) + (P_parent^T u~_parent)[child's columns],
// (the S2N pass restricted to one path), applies P_leaf^T, adds the near-field
// partial sums of the leaf's rows and writes the scaled result in original order.
constexpr int kMaxRank = 512;
template <typename V, typename TP>
__global__ void __launch_bounds__(kBlock) k_combine(const LeafPlan* leaves, const V* part, int64_t ldp, int depth,
                                                    const int32_t* rank, const int32_t* ncand, const int64_t* skoff,
                                                    const int64_t* poff, const TP* P, const V* sku, int64_t ldsk,
                                                    const int32_t* perm, const double* scale, int64_t n, double* y,
                                                    int nrhs) {
    __shared__ V tot[2][kMaxRank];
    const LeafPlan lp = leaves[blockIdx.x];
    for (int c = 0; c < nrhs; ++c) {
        int cur = 0;
        int rleaf = 0;
        if (depth >= 1) {
            const int64_t a1 = lp.heap >> (depth - 1);
            for (int i = threadIdx.x; i < rank[a1]; i += blockDim.x) tot[0][i] = sku[c * ldsk + skoff[a1] + i];
            __syncthreads();
            for (int lvl = 2; lvl <= depth; ++lvl) {
                const int64_t node = lp.heap >> (depth - lvl), par = node >> 1;
                const int rp = rank[par], ncp = ncand[par], rn = rank[node];
                const int off = (node & 1) ? rank[2 * par] : 0;
                const TP* Pm = P + poff[par] + off;
                for (int j = threadIdx.x; j < rn; j += blockDim.x) {
                    V acc = 0;
                    int i = 0;
                    for (; i + 8 <= rp; i += 8) {
                        TP pv[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) pv[u] = Pm[static_cast<int64_t>(i + u) * ncp + j];
#pragma unroll
                        for (int u = 0; u < 8; ++u) acc += static_cast<V>(pv[u]) * tot[cur][i + u];
                    }
                    for (; i < rp; ++i) acc += static_cast<V>(Pm[static_cast<int64_t>(i) * ncp + j]) * tot[cur][i];
                    tot[cur ^ 1][j] = sku[c * ldsk + skoff[node] + j] + acc;
                }
                __syncthreads();
                cur ^= 1;
            }
            rleaf = rank[lp.heap];
        }
        const TP* Pl = P + poff[lp.heap];
        const V* pc = part + c * ldp + lp.part_off;
        for (int j = threadIdx.x; j < lp.rows; j += blockDim.x) {
            V near = 0;
            int q = 0;
            for (; q + 8 <= lp.nitems; q += 8) {
                V x[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) x[u] = pc[static_cast<int64_t>(q + u) * lp.ld + j];
#pragma unroll
                for (int u = 0; u < 8; ++u) near += x[u];
            }
            for (; q < lp.nitems; ++q) near += pc[static_cast<int64_t>(q) * lp.ld + j];
            V f = 0;
            int i = 0;
            for (; i + 8 <= rleaf; i += 8) {
                TP pv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) pv[u] = Pl[static_cast<int64_t>(i + u) * lp.rows + j];
#pragma unroll
                for (int u = 0; u < 8; ++u) f += static_cast<V>(pv[u]) * tot[cur][i + u];
            }
            for (; i < rleaf; ++i) f += static_cast<V>(Pl[static_cast<int64_t>(i) * lp.rows + j]) * tot[cur][i];
            const int64_t pos = lp.start + j;
            const double sc = scale ? scale[pos] : 1.0;
            y[c * n + perm[pos]] = sc * static_cast<double>(near + f);
        }
        __syncthreads();
    }
}

// ---- normalisation and precision conversion --------------------------------
__global__ void k_fill(double* x, int64_t n, double v) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i < n) x[i] = v;
}

// q (original order) -> tree order; x = 1/q for the second product
__global__ void k_deg1(const double* q_orig, const int32_t* perm, int64_t n, double* q_tree, double* xinv,
                       int* bad) {
    const int64_t pos = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (pos >= n) return;
    const int32_t i = perm[pos];
    const double q = q_orig[i];
    q_tree[pos] = q;
    if (!(q > 0.0)) atomicOr(bad, 1);
    xinv[i] = 1.0 / q;
}

// d = (K~ q^-1) / q, c = 1 / (q sqrt(d))
__global__ void k_deg2(const double* kq_orig, const int32_t* perm, int64_t n, const double* q_tree, double* d_tree,
                       double* c_tree, int* bad) {
    const int64_t pos = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (pos >= n) return;
    const double q = q_tree[pos];
    const double d = kq_orig[perm[pos]] / q;
    d_tree[pos] = d;
    if (!(d > 0.0)) atomicOr(bad, 1);
    c_tree[pos] = 1.0 / (q * sqrt(d));
}

// per tile: max |value| (block reduction)
__global__ void k_tile_max(const double* src, const int64_t* off, const int64_t* cnt, float* scale) {
    __shared__ double sm[kBlock];
    const int64_t t = blockIdx.x;
    double m = 0.0;
    for (int64_t e = threadIdx.x; e < cnt[t]; e += blockDim.x) m = fmax(m, fabs(src[off[t] + e]));
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) scale[t] = sm[0] > 0.0 ? static_cast<float>(sm[0]) : 1.0f;
}

template <typename T>
__global__ void k_convert(const double* src, const int64_t* off, const int64_t* cnt, const float* scale, T* dst) {
    const int64_t t = blockIdx.y;
    const double inv = scale ? 1.0 / static_cast<double>(scale[t]) : 1.0;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < cnt[t];
         e += static_cast<int64_t>(gridDim.x) * blockDim.x)
        dst[off[t] + e] = from_d<T>(src[off[t] + e] * inv);
}

__global__ void k_to_f32(const double* src, float* dst, int64_t n) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i < n) dst[i] = static_cast<float>(src[i]);
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
size_t Op::footprint() const {
    return xf.bytes() + xu.bytes() + perm.bytes() + iperm.bytes() + knn_idx.bytes() + knn_d2.bytes() + skel.bytes() +
           P64.bytes() + P32.bytes() + rows.bytes() + near64.bytes() + nearT.bytes() + near_scale.bytes() +
           far64.bytes() + farT.bytes() + far_scale.bytes() + far_colmap.bytes() + d_items.bytes() +
           d_leaves.bytes() + q.bytes() + d.bytes() + c.bytes() + w_tree.bytes() + u_tree.bytes() + skw.bytes() +
           sku.bytes() + part.bytes();
}

static int rows_per_lane(int dt) { return 16 / static_cast<int>(dtype_size(dt)); }

void build_eval_plan(Op& op, hipStream_t s) {
    const int64_t L = op.L;
    op.levels.assign(op.depth + 1, NodeLevel{});
    std::vector<int32_t> heaps;
    op.heaps_off.assign(op.depth + 2, 0);
    for (int lvl = 0; lvl <= op.depth; ++lvl) {
        op.heaps_off[lvl] = static_cast<int64_t>(heaps.size());
        op.levels[lvl].level = lvl;
        for (int64_t h = int64_t(1) << lvl; h < (int64_t(1) << (lvl + 1)); ++h) {
            if (lvl >= 1) {
                op.levels[lvl].heap.push_back(static_cast<int32_t>(h));
                heaps.push_back(static_cast<int32_t>(h));
            }
        }
    }
    op.heaps_off[op.depth + 1] = static_cast<int64_t>(heaps.size());
    op.d_heaps = to_device(heaps, s);
    op.d_rank = to_device(op.rank, s);
    op.d_ncand = to_device(op.ncand, s);
    op.d_skoff = to_device(op.skoff, s);
    op.d_poff = to_device(op.poff, s);
    op.d_far_block_off = to_device(op.far_block_off, s);
    op.d_far_cols = to_device(op.far_cols, s);
    op.d_far_colbase = to_device(op.far_colbase, s);
    // near-field items: per leaf, per row group, per near tile, per column chunk
    const int rpl = rows_per_lane(op.prm.near_prec);
    const int rg = kWave * rpl;
    op.near_rows_per_group = rg;
    op.items.clear();
    op.leaves.clear();
    int64_t part = 0;
    for (int64_t a = 0; a < L; ++a) {
        const int64_t ha = L + a;
        const int32_t ld = op.near_ld[a];
        LeafPlan lp{};
        lp.part_off = part;
        lp.ld = ld;
        lp.start = static_cast<int32_t>(op.start[ha]);
        lp.rows = static_cast<int32_t>(op.size[ha]);
        lp.heap = static_cast<int32_t>(ha);
        lp.ngroups = (ld + rg - 1) / rg;
        int per_group = 0;
        for (int32_t t = op.near_off[a]; t < op.near_off[a + 1]; ++t) {
            const int64_t nb = op.size[L + op.near_idx[t]];
            per_group += static_cast<int>((nb + kChunk - 1) / kChunk);
        }
        lp.nitems = per_group;
        for (int g = 0; g < lp.ngroups; ++g) {
            int q = 0;
            for (int32_t t = op.near_off[a]; t < op.near_off[a + 1]; ++t) {
                const int64_t hb = L + op.near_idx[t];
                const int64_t nb = op.size[hb];
                for (int64_t c0 = 0; c0 < nb; c0 += kChunk, ++q) {
                    NearItem I{};
                    I.tile_off = op.near_tile_off[t] + c0 * ld;
                    I.part_off = part + static_cast<int64_t>(q) * ld;
                    I.ld = ld;
                    I.row0 = g * rg;
                    I.ncols = static_cast<int32_t>(std::min<int64_t>(kChunk, nb - c0));
                    I.col_pos = static_cast<int32_t>(op.start[hb] + c0);
                    I.tile = t;
                    I.nrows = rg;
                    op.items.push_back(I);
                }
            }
        }
        part += static_cast<int64_t>(per_group) * ld;
        op.leaves.push_back(lp);
    }
    op.part_elems = part;
    op.d_items = to_device(op.items, s);
    op.d_leaves = to_device(op.leaves, s);
    // one row task per skeleton row, grouped by level from the leaves up; the
    // same list, taken whole, gives the far-field (S2S) rows
    std::vector<RowTask> tasks;
    op.row_begin.assign(op.depth + 1, 0);
    op.row_count.assign(op.depth + 1, 0);
    for (int lvl = op.depth; lvl >= 1; --lvl) {
        op.row_begin[lvl] = static_cast<int64_t>(tasks.size());
        for (int64_t h = int64_t(1) << lvl; h < (int64_t(1) << (lvl + 1)); ++h)
            for (int32_t i = 0; i < op.rank[h]; ++i) tasks.push_back(RowTask{static_cast<int32_t>(h), i});
        op.row_count[lvl] = static_cast<int64_t>(tasks.size()) - op.row_begin[lvl];
    }
    op.row_total = static_cast<int64_t>(tasks.size());
    op.d_row_tasks = to_device(tasks, s);
    if (!op.side) HDM_HIP(hipStreamCreateWithFlags(&op.side, hipStreamNonBlocking));
    if (!op.ev_fork) HDM_HIP(hipEventCreateWithFlags(&op.ev_fork, hipEventDisableTiming));
    if (!op.ev_join) HDM_HIP(hipEventCreateWithFlags(&op.ev_join, hipEventDisableTiming));
    HDM_HIP(hipStreamSynchronize(s));
}

Op::~Op() {
    if (side) (void)hipStreamSynchronize(side);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (side) (void)hipStreamDestroy(side);
}

static void ensure_ws(Op& op, int nrhs, size_t vbytes) {
    if (op.ws_nrhs >= nrhs && op.w_tree.bytes() >= static_cast<size_t>(op.n) * nrhs * vbytes) return;
    op.w_tree.alloc(static_cast<size_t>(op.n) * nrhs * 8);
    op.skw.alloc(static_cast<size_t>(std::max<int64_t>(op.nskel, 1)) * nrhs * 8);
    op.sku.alloc(static_cast<size_t>(std::max<int64_t>(op.nskel, 1)) * nrhs * 8);
    op.part.alloc(static_cast<size_t>(std::max<int64_t>(op.part_elems, 1)) * nrhs * 8);
    op.ws_nrhs = nrhs;
}

template <typename V, typename TN, typename TF, typename TP>
static void apply_t(Op& op, bool normalised, const TN* near, const float* nscale, const TF* far, const float* fscale,
                    const TP* P, const double* x, double* y, int nrhs, hipStream_t s) {
    ensure_ws(op, nrhs, sizeof(V));
    const int64_t n = op.n;
    V* w = reinterpret_cast<V*>(op.w_tree.get());
    V* skw = reinterpret_cast<V*>(op.skw.get());
    V* sku = reinterpret_cast<V*>(op.sku.get());
    V* part = reinterpret_cast<V*>(op.part.get());
    const int64_t ldsk = std::max<int64_t>(op.nskel, 1);
    const int64_t ldp = std::max<int64_t>(op.part_elems, 1);
    const double* scale = normalised ? op.c.get() : nullptr;
    Ctx* cx = op.ctx;
    {
        KernelEvents ev(cx, HDM_PHASE_PREP);
        hipExtLaunchKernelGGL((k_prep<V>), dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, ev.start, ev.stop, 0, n, nrhs,
                              x, op.perm.get(), scale, w);
    }
    // the upward pass and the far field run on a side stream while the near field streams its tiles
    const bool tree = op.nskel > 0;
    const int wpb = kBlock / kWave;
    if (tree) {
        HDM_HIP(hipEventRecord(op.ev_fork, s));
        HDM_HIP(hipStreamWaitEvent(op.side, op.ev_fork, 0));
        {
            PhaseScope ph(cx, HDM_PHASE_N2S, op.side);
            for (int lvl = op.depth; lvl >= 1; --lvl) {
                const int64_t t0 = op.row_begin[lvl], nt = op.row_count[lvl];
                if (nt == 0) continue;
                hipLaunchKernelGGL((k_n2s<V, TP>), dim3(ceil_div(nt, wpb)), dim3(kBlock), 0, op.side,
                                   op.d_row_tasks.get() + t0, nt, lvl == op.depth ? 1 : 0, op.d_start.get(),
                                   op.d_ncand.get(), op.d_skoff.get(), op.d_poff.get(), P, w, n, skw, ldsk, nrhs);
            }
        }
        {
            KernelEvents ev(cx, HDM_PHASE_S2S);
            const int64_t nt = op.row_total;
            hipExtLaunchKernelGGL((k_s2s<V, TF>), dim3(ceil_div(nt, wpb)), dim3(kBlock), 0, op.side, ev.start, ev.stop,
                                  0, op.d_row_tasks.get(), nt, op.d_skoff.get(), op.d_far_block_off.get(),
                               op.d_far_cols.get(), op.d_far_colbase.get(), op.far_colmap.get(), far, fscale, skw, sku,
                               ldsk, nrhs);
        }
        HDM_HIP(hipEventRecord(op.ev_join, op.side));
    }
    {
        KernelEvents ev(cx, HDM_PHASE_L2L);
        const int64_t nit = static_cast<int64_t>(op.items.size());
        hipExtLaunchKernelGGL((k_l2l<V, TN>), dim3(ceil_div(nit, wpb)), dim3(kBlock), 0, s, ev.start, ev.stop, 0,
                              op.d_items.get(), nit, near, nscale, w, n, part, ldp, nrhs);
    }
    if (tree) HDM_HIP(hipStreamWaitEvent(s, op.ev_join, 0));
    {
        KernelEvents ev(cx, HDM_PHASE_COMBINE);
        hipExtLaunchKernelGGL((k_combine<V, TP>), dim3(op.L), dim3(kBlock), 0, s, ev.start, ev.stop, 0,
                              op.d_leaves.get(), part, ldp,
                           tree ? op.depth : 0, op.d_rank.get(), op.d_ncand.get(), op.d_skoff.get(), op.d_poff.get(),
                           P, sku, ldsk, op.perm.get(), scale, n, y, nrhs);
    }
    check_launch("apply");
}

void apply(Op& op, int normalised, bool exact64, const double* x, double* y, int nrhs, hipStream_t s) {
    if (exact64 || (op.prm.near_prec == HDM_F64 && op.prm.far_prec == HDM_F64)) {
        HDM_CHECK(op.near64.n > 0 || op.near_elems == 0, HDM_EINTERNAL, "float64 tiles are not resident");
    HDM_CHECK(op.prm.max_rank_s <= kMaxRank, HDM_EINTERNAL, "rank above the combine kernel's limit");
        apply_t<double, double, double, double>(op, normalised, op.near64.get(), nullptr, op.far64.get(), nullptr,
                                                op.P64.get(), x, y, nrhs, s);
        return;
    }
    const float* ns = op.near_scale.n ? op.near_scale.get() : nullptr;
    const float* fs = op.far_scale.n ? op.far_scale.get() : nullptr;
    const float* P = op.P32.get();
    auto far_dispatch = [&](auto near_ptr) {
        using TN = std::remove_cv_t<std::remove_pointer_t<decltype(near_ptr)>>;
        switch (op.prm.far_prec) {
            case HDM_F32:
                apply_t<float, TN, float, float>(op, normalised, near_ptr, ns, reinterpret_cast<const float*>(op.farT.get()),
                                                 fs, P, x, y, nrhs, s);
                break;
            case HDM_BF16:
                apply_t<float, TN, bf16_t, float>(op, normalised, near_ptr, ns,
                                                  reinterpret_cast<const bf16_t*>(op.farT.get()), fs, P, x, y, nrhs, s);
                break;
            case HDM_F16:
                apply_t<float, TN, f16_t, float>(op, normalised, near_ptr, ns,
                                                 reinterpret_cast<const f16_t*>(op.farT.get()), fs, P, x, y, nrhs, s);
                break;
            default: fail(HDM_EINVAL, "unsupported far precision with reduced near precision");
        }
    };
    switch (op.prm.near_prec) {
        case HDM_F32: far_dispatch(reinterpret_cast<const float*>(op.nearT.get())); break;
        case HDM_BF16: far_dispatch(reinterpret_cast<const bf16_t*>(op.nearT.get())); break;
        case HDM_F16: far_dispatch(reinterpret_cast<const f16_t*>(op.nearT.get())); break;
        default: fail(HDM_EINVAL, "unsupported near precision");
    }
}

// q = K~ 1, d = Q^-1 K~ Q^-1 1, c = 1 / (q sqrt(d)), with float64 tiles
void normalise_degrees(Op& op, hipStream_t s) {
    const int64_t n = op.n;
    DevBuf<double> ones(n), qo(n), xinv(n), kq(n);
    DevBuf<int> bad(1);
    HDM_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int), s));
    op.q.alloc(n);
    op.d.alloc(n);
    op.c.alloc(n);
    hipLaunchKernelGGL(k_fill, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, ones.get(), n, 1.0);
    apply(op, 0, true, ones.get(), qo.get(), 1, s);
    hipLaunchKernelGGL(k_deg1, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, qo.get(), op.perm.get(), n, op.q.get(),
                       xinv.get(), bad.get());
    apply(op, 0, true, xinv.get(), kq.get(), 1, s);
    hipLaunchKernelGGL(k_deg2, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, kq.get(), op.perm.get(), n, op.q.get(),
                       op.d.get(), op.c.get(), bad.get());
    check_launch("degrees");
    int hb = 0;
    bad.download(&hb, 1, s);
    HDM_HIP(hipStreamSynchronize(s));
    HDM_CHECK(hb == 0, HDM_ENUMERIC, "non-positive degree in the alpha = 1 normalisation");
}

template <typename T>
static void convert_tiles(const DevBuf<double>& src, const std::vector<int64_t>& off, const std::vector<int64_t>& cnt,
                          bool scaled, DevBuf<char>& dst, DevBuf<float>& scale, int64_t elems, hipStream_t s) {
    dst.alloc(static_cast<size_t>(std::max<int64_t>(elems, 1)) * sizeof(T));
    if (off.empty()) return;
    DevBuf<int64_t> doff = to_device(off, s), dcnt = to_device(cnt, s);
    float* sp = nullptr;
    if (scaled) {
        scale.alloc(off.size());
        hipLaunchKernelGGL(k_tile_max, dim3(off.size()), dim3(kBlock), 0, s, src.get(), doff.get(), dcnt.get(),
                           scale.get());
        sp = scale.get();
    }
    for (size_t base = 0; base < off.size(); base += 65535) {
        const int nb = static_cast<int>(std::min<size_t>(65535, off.size() - base));
        hipLaunchKernelGGL((k_convert<T>), dim3(64, nb), dim3(kBlock), 0, s, src.get(), doff.get() + base,
                           dcnt.get() + base, sp ? sp + base : nullptr, reinterpret_cast<T*>(dst.get()));
    }
    check_launch("convert");
    HDM_HIP(hipStreamSynchronize(s));
}

void convert_eval_precision(Op& op, hipStream_t s) {
    if (op.prm.near_prec == HDM_F64 && op.prm.far_prec == HDM_F64) return;
    HDM_CHECK(op.prm.near_prec != HDM_F64 && op.prm.far_prec != HDM_F64, HDM_EINVAL,
              "float64 tiles cannot be mixed with reduced-precision tiles");
    // near: one scale per tile (pair)
    std::vector<int64_t> noff, ncnt;
    const int64_t L = op.L;
    for (int64_t a = 0; a < L; ++a)
        for (int32_t t = op.near_off[a]; t < op.near_off[a + 1]; ++t) {
            noff.push_back(op.near_tile_off[t]);
            ncnt.push_back(static_cast<int64_t>(op.near_ld[a]) * op.size[L + op.near_idx[t]]);
        }
    // far: one scale per node block (indexed by heap id)
    std::vector<int64_t> foff(op.nnodes, 0), fcnt(op.nnodes, 0);
    for (int64_t h = 0; h < op.nnodes; ++h) {
        foff[h] = op.far_block_off[h];
        fcnt[h] = static_cast<int64_t>(op.rank[h]) * op.far_cols[h];
    }
    auto go = [&](int prec, const DevBuf<double>& src, const std::vector<int64_t>& off, const std::vector<int64_t>& cnt,
                  DevBuf<char>& dst, DevBuf<float>& scale, int64_t elems) {
        switch (prec) {
            case HDM_F32: convert_tiles<float>(src, off, cnt, false, dst, scale, elems, s); break;
            case HDM_BF16: convert_tiles<bf16_t>(src, off, cnt, true, dst, scale, elems, s); break;
            case HDM_F16: convert_tiles<f16_t>(src, off, cnt, true, dst, scale, elems, s); break;
            default: fail(HDM_EINVAL, "bad tile precision");
        }
    };
    go(op.prm.near_prec, op.near64, noff, ncnt, op.nearT, op.near_scale, op.near_elems);
    go(op.prm.far_prec, op.far64, foff, fcnt, op.farT, op.far_scale, op.far_elems);
    op.P32.alloc(std::max<int64_t>(op.np, 1));
    if (op.np > 0)
        hipLaunchKernelGGL(k_to_f32, dim3(ceil_div(op.np, kBlock)), dim3(kBlock), 0, s, op.P64.get(), op.P32.get(), op.np);
    check_launch("P to f32");
    HDM_HIP(hipStreamSynchronize(s));
    // the float64 tiles were only needed for the degrees
    op.near64.release();
    op.far64.release();
}

}  // namespace hdm
