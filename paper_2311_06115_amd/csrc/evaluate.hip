// Evaluation of the compressed operator K~ = D + S + UV (Eq. (3)) and of the
// alpha = 1 normalised operator S~ x = c * K~ (c * x) (Alg. 1), once per Lanczos
// step.  Phases, all owner-computes with fixed reduction order (deterministic):
//   N2S  upward:   skeleton weights  w~_h = P_h w_h (leaf), P_h [w~_l; w~_r]
//   S2S  far:      skeleton potentials u~_h = sum_{g in Far(h)} K(skel_h, skel_g) w~_g
//   S2N  downward: [u~_l; u~_r] += P_h^T u~_h; leaves fold P^T u~ into the output
//   L2L  near:     u_a += sum_{b in Near(a)} K(a, b) w_b   (streams the near tiles)
#include <cstring>
#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>

#include "op.hpp"

namespace hdm {

namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kChunk = 64;    // columns per near-field work item
constexpr int kOtfRunItems = 8;   // items per run of the on-the-fly float64 near field

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

// ---- batches ----------------------------------------------------------------
// Per-launch arguments of a batched product, passed by value: the operators'
// descriptors, the prefix of work units over the operators, and each
// operator's vectors.
struct Batch {
    int nops, nrhs;
    int flip;                     // near field: work items taken in reverse order
    int up;                       // near field: leading workgroups that run the upward pass
    const OpDev* op[kMaxBatch];
    int64_t pre[kMaxBatch + 1];
    int32_t arg[kMaxBatch];       // per operator: tree level (N2S), or for prep and combine bit 0: normalised,
                                  // bit 1: the vectors are in tree order (no gather or scatter)
    const double* x[kMaxBatch];
    double* y[kMaxBatch];
};

__device__ inline int batch_op(const Batch& b, int64_t unit) {
    int o = 0;
    while (o + 1 < b.nops && unit >= b.pre[o + 1]) ++o;
    return o;
}

// ---- vector staging: w = c * x in tree order ------------------------------------
template <typename V>
__global__ void k_prep(Batch b) {
    const int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (u >= b.pre[b.nops]) return;
    const int o = batch_op(b, u);
    const OpDev& D = *b.op[o];
    const int64_t pos = u - b.pre[o];
    const int64_t i = (b.arg[o] & 2) ? pos : D.perm[pos];
    const double sc = (b.arg[o] & 1) ? D.c[pos] : 1.0;
    V* w = static_cast<V*>(D.w);
    for (int c = 0; c < b.nrhs; ++c) w[c * D.n + pos] = static_cast<V>(sc * b.x[o][c * D.n + i]);
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

// ---- N2S: one tree level per operator (arg = level), one wave per skeleton row --
//   leaf:  w~_h = P_h w_h;   inner: w~_h = P_h [w~_left; w~_right]
template <typename V, typename TP>
__global__ void k_n2s(Batch b) {
    const int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x / kWave) + threadIdx.x / kWave;
    if (u >= b.pre[b.nops]) return;
    const int o = batch_op(b, u);
    const OpDev& D = *b.op[o];
    const int lvl = b.arg[o];
    const RowTask T = D.rows[D.row_begin[lvl] + (u - b.pre[o])];
    const int nc = D.ncand[T.h];
    const TP* row = static_cast<const TP*>(D.P) + D.poff[T.h] + static_cast<int64_t>(T.i) * nc;
    V* skw = static_cast<V*>(D.skw);
    for (int c = 0; c < b.nrhs; ++c) {
        const V* in = lvl == D.depth ? static_cast<const V*>(D.w) + c * D.n + D.start[T.h]
                                     : skw + c * D.ldsk + D.skoff[2 * T.h];
        const V acc = row_dot<V>(row, nc, [&](int j) { return in[j]; });
        if (threadIdx.x % kWave == 0) skw[c * D.ldsk + D.skoff[T.h] + T.i] = acc;
    }
}

// ---- S2S: far field between skeletons, one wave per skeleton row ----------------
template <typename V, typename TF>
__global__ void k_s2s(Batch b) {
    const int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x / kWave) + threadIdx.x / kWave;
    if (u >= b.pre[b.nops]) return;
    const int o = batch_op(b, u);
    const OpDev& D = *b.op[o];
    const RowTask T = D.rows[u - b.pre[o]];
    const int nc = D.far_cols[T.h];
    const TF* row = static_cast<const TF*>(D.far) + D.far_off[T.h] + static_cast<int64_t>(T.i) * nc;
    const int32_t* cm = D.far_colmap + D.far_colbase[T.h];
    const V sc = D.fscale ? static_cast<V>(D.fscale[T.h]) : V(1);
    const V* skw = static_cast<const V*>(D.skw);
    V* sku = static_cast<V*>(D.sku);
    for (int c = 0; c < b.nrhs; ++c) {
        const V* x = skw + c * D.ldsk;
        const V acc = row_dot<V>(row, nc, [&](int j) { return x[cm[j]]; });
        if (threadIdx.x % kWave == 0) sku[c * D.ldsk + D.skoff[T.h] + T.i] = acc * sc;
    }
}

// ---- upward pass: leaf level carried by the near-field launch -----------------
// One operator, one right-hand side: the first b.up workgroups of the near-field
// grid, one per leaf, form the leaves' skeleton weights w~_h = P_h w_h with the
// same row dot products as k_n2s.  They need only the staged vector, so they run
// beside the tile streaming; the levels above follow in their own launch.
template <typename V>
__device__ inline void leaf_n2s(const Batch& b, int64_t leaf) {
    const OpDev& D = *b.op[0];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const int64_t h = D.L + leaf;
    const int rk = D.rank[h], nc = D.ncand[h];
    const V* Ph = static_cast<const V*>(D.P) + D.poff[h];
    const V* in = static_cast<const V*>(D.w) + D.start[h];
    V* out = static_cast<V*>(D.skw) + D.skoff[h];
    for (int i = wave; i < rk; i += nw) {
        const V acc = row_dot<V>(Ph + static_cast<int64_t>(i) * nc, nc, [&](int j) { return in[j]; });
        if (lane == 0) out[i] = acc;
    }
}

// The leaf skeletons under an inner node h at level lvl are one contiguous run
// of skeleton slots (leaves take the first slots, in heap order): from the slot
// of its first leaf, nlk long.
struct LeafRun {
    int64_t base;
    int nlk, nlk_left;
};
__device__ inline LeafRun leaf_run(const int64_t* skoff, const int32_t* rank, int depth, int64_t h, int lvl) {
    const int sh = depth - lvl;
    const int64_t fl = h << sh, ll = ((h + 1) << sh) - 1, lm = ((2 * h + 1) << (sh - 1)) - 1;
    LeafRun r;
    r.base = skoff[fl];
    r.nlk = static_cast<int>(skoff[ll] + rank[ll] - r.base);
    r.nlk_left = static_cast<int>(skoff[lm] + rank[lm] - r.base);
    return r;
}

// ---- composites of the nested bases (built once per operator) -------------------
// The skeleton weights of an inner node are a fixed linear map of the leaf
// skeleton weights under it: w~_h = C_h w~_leaves(h), with
//   C_h = P_h [C_left 0; 0 C_right]   and a leaf's C the identity,
// so C_h = P_h one level above the leaves.  One launch per level from the leaves
// up; a wave per (row of C_h, 64 of its columns) (grid y = column chunk), eight
// child rows loaded at a time; float64 from P's float64 copy, also stored
// rounded to float32 for the evaluation-precision products.
constexpr int kComposeBatch = 8;
__global__ void k_compose(const double* P64, const int64_t* poff, const int32_t* rank, const int32_t* ncand,
                          const int64_t* skoff, const int64_t* coff, const RowTask* rows, int64_t row0,
                          int64_t nrows, int depth, int lvl, double* C64, float* C32) {
    const int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x / kWave) + threadIdx.x / kWave;
    if (u >= nrows) return;
    const RowTask T = rows[row0 + u];
    const int64_t h = T.h;
    const LeafRun lr = leaf_run(skoff, rank, depth, h, lvl);
    const int c = static_cast<int>(blockIdx.y) * kWave + static_cast<int>(threadIdx.x % kWave);
    if (c >= lr.nlk) return;
    const double* Prow = P64 + poff[h] + static_cast<int64_t>(T.i) * ncand[h];
    double acc = 0.0;
    if (lvl == depth - 1) {
        acc = Prow[c];
    } else {
        // the child whose leaves hold column c, and c within its run
        const bool left = c < lr.nlk_left;
        const int64_t ch = left ? 2 * h : 2 * h + 1;
        const int rc = rank[ch], nlk_c = left ? lr.nlk_left : lr.nlk - lr.nlk_left;
        const double* Pc = Prow + (left ? 0 : rank[2 * h]);
        const double* Cc = C64 + coff[ch] + (left ? c : c - lr.nlk_left);
        for (int j0 = 0; j0 < rc; j0 += kComposeBatch) {
            double pv[kComposeBatch], cv[kComposeBatch];
#pragma unroll
            for (int t = 0; t < kComposeBatch; ++t) {
                const int j = min(j0 + t, rc - 1);
                pv[t] = Pc[j];
                cv[t] = Cc[static_cast<int64_t>(j) * nlk_c];
            }
#pragma unroll
            for (int t = 0; t < kComposeBatch; ++t)
                if (j0 + t < rc) acc += pv[t] * cv[t];
        }
    }
    const int64_t o = coff[h] + static_cast<int64_t>(T.i) * lr.nlk + c;
    C64[o] = acc;
    C32[o] = static_cast<float>(acc);
}

// ---- upper levels of the upward pass in one launch, one wave per skeleton row ----
//   w~_h = C_h w~_leaves(h)  for every inner node below the root
template <typename V>
__global__ void k_n2s_up(Batch b) {
    const int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x / kWave) + threadIdx.x / kWave;
    if (u >= b.pre[b.nops]) return;
    const int o = batch_op(b, u);
    const OpDev& D = *b.op[o];
    const RowTask T = D.rows[D.row_count[D.depth] + (u - b.pre[o])];
    const int64_t h = T.h;
    const int lvl = 63 - __builtin_clzll(static_cast<unsigned long long>(h));
    const LeafRun lr = leaf_run(D.skoff, D.rank, D.depth, h, lvl);
    const V* row = static_cast<const V*>(D.comp) + D.coff[h] + static_cast<int64_t>(T.i) * lr.nlk;
    V* skw = static_cast<V*>(D.skw);
    const V* in = skw + lr.base;
    const V acc = row_dot<V>(row, lr.nlk, [&](int j) { return in[j]; });
    if (threadIdx.x % kWave == 0) skw[D.skoff[h] + T.i] = acc;
}

// The same for several right-hand sides: each lane keeps one partial sum per
// column and every composite element is loaded once (columns past nrhs repeat
// the last one so that the loads issue together; only the stores are guarded)
template <typename V>
__global__ void k_n2s_up_m(Batch b) {
    const int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x / kWave) + threadIdx.x / kWave;
    if (u >= b.pre[b.nops]) return;
    const int o = batch_op(b, u);
    const OpDev& D = *b.op[o];
    const RowTask T = D.rows[D.row_count[D.depth] + (u - b.pre[o])];
    const int64_t h = T.h;
    const int lvl = 63 - __builtin_clzll(static_cast<unsigned long long>(h));
    const LeafRun lr = leaf_run(D.skoff, D.rank, D.depth, h, lvl);
    const V* row = static_cast<const V*>(D.comp) + D.coff[h] + static_cast<int64_t>(T.i) * lr.nlk;
    V* skw = static_cast<V*>(D.skw);
    const V* in = skw + lr.base;
    const int lane = threadIdx.x % kWave;
    const int last = b.nrhs - 1;
    V acc[kMaxRhs];
#pragma unroll
    for (int c = 0; c < kMaxRhs; ++c) acc[c] = 0;
    for (int j = lane; j < lr.nlk; j += kWave) {
        const V p = row[j];
#pragma unroll
        for (int c = 0; c < kMaxRhs; ++c) acc[c] += p * in[min(c, last) * D.ldsk + j];
    }
#pragma unroll
    for (int c = 0; c < kMaxRhs; ++c) {
        if (c >= b.nrhs) break;
        const V t = wave_sum(acc[c]);
        if (lane == 0) skw[c * D.ldsk + D.skoff[h] + T.i] = t;
    }
}

__device__ inline int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// read-only descriptors through the constant address space: scalar loads,
// which do not wait behind the tile loads in flight
typedef const __attribute__((address_space(4))) NearItem cNearItem;
typedef const __attribute__((address_space(4))) float cfloat;

// ---- L2L: stream the near tiles; one wave per work item ---------------------
// Lane l owns RPL consecutive rows (16 bytes of tile per lane per column) of
// each 64*RPL-row pass over the item's rows; the item's columns are consecutive
// tree positions, so w is read as a wave-uniform value.
template <typename V, typename TN>
__device__ __forceinline__ void l2l_one(const Batch& b, const OpDev& D, int64_t ui, int lane) {
    constexpr int RPL = 16 / sizeof(TN);
    const NearItem I = D.items1[ui];
    const int rend = min(I.ld, I.row0 + I.nrows);
    const V sc = D.nscale ? static_cast<V>(D.nscale[I.tile]) : V(1);
    const TN* tiles = static_cast<const TN*>(D.near);
    const V* wc = static_cast<const V*>(D.w) + I.col_pos;
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
        V* out = static_cast<V*>(D.part) + I.part_off + row;
#pragma unroll
        for (int r = 0; r < RPL; ++r) out[r] = acc[r];
    }
}

// Several right-hand sides: each tile element is read once per group of CG
// columns.  Lane l keeps RPL rows x CG columns of sums.  The group's weights of
// the item's columns (one per right-hand side and tile column, the same for
// every lane) are staged in the wave's slice of shared memory, one tile column's
// CG weights contiguous, and read back as broadcasts; the tile's scale
// multiplies the finished sums.  Columns past the last right-hand side repeat
// its weights and store nothing.
template <typename TN> constexpr int kL2lRpl = 16 / static_cast<int>(sizeof(TN));
template <typename TN> constexpr int kL2lCols = kMaxRhs < 64 / kL2lRpl<TN> ? kMaxRhs : 64 / kL2lRpl<TN>;

typedef uint32_t u4_t __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) u4_t gu4_t;
// 16 bytes from global memory as a global (not flat) load
template <typename T>
__device__ inline void gload_16b(T (&dst)[16 / sizeof(T)], const T* p) {
    const u4_t v = *(gu4_t*)(p);
    __builtin_memcpy(dst, &v, 16);
}
template <typename T>
__device__ inline T gload1(const T* p) { return *(const __attribute__((address_space(1))) T*)(p); }

template <typename V, typename TN>
__device__ __forceinline__ void l2l_multi(const Batch& b, const OpDev& D, int64_t ui, int lane, V* ws) {
    constexpr int RPL = kL2lRpl<TN>;
    constexpr int CG = kL2lCols<TN>;
    constexpr int JB = 4;   // tile columns per step; the next step's loads are in flight meanwhile
    cNearItem* Ip = (cNearItem*)D.items + ui;
    const int64_t tile_off = Ip->tile_off, part_off = Ip->part_off;
    const int ld = Ip->ld, row0 = Ip->row0, ncols = Ip->ncols, col_pos = Ip->col_pos, tile = Ip->tile;
    const int rend = min(ld, row0 + Ip->nrows);
    const V sc = D.nscale ? static_cast<V>(*((cfloat*)D.nscale + tile)) : V(1);
    const TN* tiles = static_cast<const TN*>(D.near) + tile_off;
    const int64_t n = D.n, ldp = D.ldp;
    const int last = b.nrhs - 1;
    const int nsteps = (ncols + JB - 1) / JB;
    for (int c0 = 0; c0 <= last; c0 += CG) {
        {   // lane j stages tile column j's weights (ncols <= 64); zeros past the item's columns
            const int j = min(lane, ncols - 1);
            const V* wj = static_cast<const V*>(D.w) + col_pos + j;
            V wv[CG];
#pragma unroll
            for (int c = 0; c < CG; ++c) wv[c] = gload1(wj + min(c0 + c, last) * n);
#pragma unroll
            for (int c = 0; c < CG; ++c) wv[c] = lane < ncols ? wv[c] : V(0);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_memcpy(ws + lane * CG, wv, sizeof(wv));
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        for (int r0 = row0; r0 < rend; r0 += kWave * RPL) {
            const int row = r0 + lane * RPL;
            // lanes past the item's rows read its last row group and store nothing
            const TN* col = tiles + min(row, rend - 1) / RPL * RPL;
            V acc[RPL][CG];
#pragma unroll
            for (int r = 0; r < RPL; ++r)
#pragma unroll
                for (int c = 0; c < CG; ++c) acc[r][c] = 0;
            // steps past the item's columns read its last column (their weights are zero)
            auto load = [&](int step, TN (&t)[JB][RPL]) {
#pragma unroll
                for (int q = 0; q < JB; ++q)
                    gload_16b(t[q], col + static_cast<int64_t>(min(step * JB + q, ncols - 1)) * ld);
            };
            TN cur[JB][RPL], nxt[JB][RPL];
            load(0, cur);
            for (int st = 0; st < nsteps; ++st) {
                load(min(st + 1, nsteps - 1), nxt);
#pragma unroll
                for (int q = 0; q < JB; ++q) {
                    V w0[CG];
                    __builtin_memcpy(w0, ws + (st * JB + q) * CG, sizeof(w0));
#pragma unroll
                    for (int c = 0; c < CG; ++c)
#pragma unroll
                        for (int r = 0; r < RPL; ++r) acc[r][c] += val<V>(cur[q][r]) * w0[c];
                }
#pragma unroll
                for (int q = 0; q < JB; ++q)
#pragma unroll
                    for (int r = 0; r < RPL; ++r) cur[q][r] = nxt[q][r];
            }
            if (row < rend) {
                V* out = static_cast<V*>(D.part) + part_off + row;
#pragma unroll
                for (int c = 0; c < CG; ++c) {
                    if (c0 + c > last) break;
#pragma unroll
                    for (int r = 0; r < RPL; ++r) out[(c0 + c) * ldp + r] = acc[r][c] * sc;
                }
            }
        }
    }
}

// kMulti: several right-hand sides (a kernel of its own, so that the
// single-column kernel keeps its small register footprint: 60 against 101
// VGPRs, 8 against 4 waves per SIMD)
template <typename V, typename TN, bool kUp, bool kMulti>
__global__ void __launch_bounds__(kBlock) k_l2l(Batch b) {
    if (kUp && static_cast<int>(blockIdx.x) < b.up) {
        leaf_n2s<V>(b, blockIdx.x);
        return;
    }
    int64_t u = (blockIdx.x - b.up) * static_cast<int64_t>(blockDim.x / kWave) + threadIdx.x / kWave;
    u = uni(static_cast<int>(u));   // wave-uniform: the descriptors load as scalars
    if (u >= b.pre[b.nops]) return;
    if (b.flip) u = b.pre[b.nops] - 1 - u;
    const int o = batch_op(b, u);
    const OpDev& D = *b.op[o];
    const int lane = threadIdx.x % kWave;
    if constexpr (kMulti) {
        __shared__ V wstage[kBlock / kWave][kWave * kL2lCols<TN>];
        l2l_multi<V, TN>(b, D, u - b.pre[o], lane, wstage[threadIdx.x / kWave]);
    } else {
        l2l_one<V, TN>(b, D, u - b.pre[o], lane);
    }
}

// ---- combine: downward pass, near partial sums, scale, scatter ---------------
// One workgroup per leaf.  It walks the leaf's ancestors top-down,
//   u~_child = S2S(child) + (P_parent^T u~_parent)[child's columns],
// (the S2N pass restricted to one path), applies P_leaf^T, adds the near-field
// partial sums of the leaf's rows and writes the scaled result in original order.
constexpr int kMaxRank = 512;
// Single right-hand side (several go to k_combine_m).  One workgroup of
// kCombBlock threads per leaf, in three phases, so that a leaf pays a few memory
// round trips rather than several per ancestor:
//  1. the ranks and offsets along the leaf's path, one level per thread;
//  2. every load that does not depend on the chain, issued together: the
//     path's P slices and far-field values staged in shared memory as one flat
//     array, the near partial sums of the leaf's first rows (four quarters of
//     the workgroup take a quarter of the items each, items in order) and the
//     leaf's P entries (a quarter of its skeleton rows each), and the scale and
//     destination of each row;
//  3. the downward chain from shared memory, then per row the quarters' near
//     sums and P_leaf^T u~ sums added in a fixed order, the alpha = 1 scale and
//     the scatter to the original order.
constexpr int kCombBlock = 1024;
constexpr int kCombQ = kCombBlock / 4;
constexpr int kChainStageBytes = 65536;
// near partial sums and P_leaf entries in flight per thread (halved for float64
// so that the workgroup's 1024 threads fit their registers)
template <typename V> constexpr int kNearBatch = sizeof(V) == 4 ? 16 : 8;
template <typename V> constexpr int kLeafBatch = sizeof(V) == 4 ? 16 : 8;

template <typename V, typename TP>
__global__ void __launch_bounds__(kCombBlock) k_combine(Batch b) {
    constexpr int kStage = kChainStageBytes / static_cast<int>(sizeof(V));
    __shared__ V tot[2][kMaxRank];
    __shared__ V chain[kStage];
    __shared__ V quarter[2][4][kCombQ];
    __shared__ int m_rn[kMaxLevels + 1], m_rp[kMaxLevels + 1], m_ncp[kMaxLevels + 1], m_cs[kMaxLevels + 1];
    __shared__ int64_t m_pb[kMaxLevels + 1], m_sk[kMaxLevels + 1], m_cb[kMaxLevels + 1], m_pleaf;
    const int64_t u = blockIdx.x;
    const int o = batch_op(b, u);
    const OpDev& D = *b.op[o];
    const LeafPlan lp = D.leaves1[u - b.pre[o]];   // one column
    const bool comp = D.s2n_comp1 && D.row_total > 0 && D.depth >= 2;
    const TP* P = static_cast<const TP*>(D.P);
    const V* sku = static_cast<const V*>(D.sku);
    const V* pc = static_cast<const V*>(D.part) + lp.part_off;
    const int depth = D.row_total > 0 ? D.depth : 0;
    const int tid = threadIdx.x;
    // 1. the node at level lvl of the path is heap >> (depth - lvl)
    if (tid >= 1 && tid <= depth) {
        const int64_t node = static_cast<int64_t>(lp.heap) >> (depth - tid);
        m_rn[tid] = D.rank[node];
        m_sk[tid] = D.skoff[node];
        if (tid >= 2) {
            const int64_t par = node >> 1;
            m_rp[tid] = D.rank[par];
            m_ncp[tid] = D.ncand[par];
            m_pb[tid] = D.poff[par] + ((node & 1) ? D.rank[2 * par] : 0);
        }
        if (comp && tid < depth) {
            // the leaf's block of columns in the composite of its ancestor at level tid
            const LeafRun lr = leaf_run(D.skoff, D.rank, depth, node, tid);
            m_cs[tid] = lr.nlk;
            m_cb[tid] = D.coff[node] + (D.skoff[lp.heap] - lr.base);
        }
    }
    if (tid == 0 && depth >= 1) m_pleaf = D.poff[lp.heap];
    __syncthreads();
    // level lvl's slice of the chain buffer: rp x rn of P_parent (the node's
    // columns), then the node's rn far-field values; through the composites
    // (comp): for each ancestor level, its rn far-field values, then the leaf's
    // block of its composite (rn x rleaf), and after all levels the per-level sums
    // the walk starts at level 1, or at the leaf when a per-level downward pass
    // (or the composites) completes every potential
    const int top = (D.s2n_levels || comp) && depth >= 1 ? depth : 1;
    const int rleaf = depth >= 1 ? m_rn[depth] : 0;
    int64_t need = 0;
    if (comp)
        for (int lvl = 1; lvl < depth; ++lvl) need += static_cast<int64_t>(m_rn[lvl]) * (1 + rleaf);
    else
        for (int lvl = top + 1; lvl <= depth; ++lvl) need += static_cast<int64_t>(m_rp[lvl] + 1) * m_rn[lvl];
    const bool staged = need <= kStage;

    // 2. independent loads
    if (depth >= 1)
        for (int i = tid; i < m_rn[top]; i += kCombBlock) tot[0][i] = sku[m_sk[top] + i];
    if (comp) {
        // need <= kStage (the host enables comp only where the whole staging fits);
        // a leaf of rank 0 has no potentials to form
        const int nd = rleaf > 0 ? static_cast<int>(need) : 0;
        const V* Cm = static_cast<const V*>(D.comp);
        int lvl = 1, lo = 0, sz = m_rn[1] * (1 + rleaf);
        for (int g0 = tid; g0 < nd; g0 += 8 * kCombBlock) {
            V x[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int g = min(g0 + t * kCombBlock, nd - 1);
                while (g >= lo + sz) {
                    lo += sz;
                    ++lvl;
                    sz = m_rn[lvl] * (1 + rleaf);
                }
                const int rn = m_rn[lvl], e = g - lo;
                x[t] = e < rn ? sku[m_sk[lvl] + e]
                              : Cm[m_cb[lvl] + static_cast<int64_t>((e - rn) / rleaf) * m_cs[lvl] + (e - rn) % rleaf];
            }
#pragma unroll
            for (int t = 0; t < 8; ++t)
                if (g0 + t * kCombBlock < nd) chain[g0 + t * kCombBlock] = x[t];
        }
    } else if (staged && need > 0) {
        // need <= kStage here, so the flat index fits in 32 bits; each thread's
        // elements come in increasing order, so its level only advances
        const int nd = static_cast<int>(need);
        int lvl = top + 1, lo = 0, sz = (m_rp[top + 1] + 1) * m_rn[top + 1];
        for (int g0 = tid; g0 < nd; g0 += 8 * kCombBlock) {
            V x[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int g = min(g0 + t * kCombBlock, nd - 1);
                while (g >= lo + sz) {
                    lo += sz;
                    ++lvl;
                    sz = (m_rp[lvl] + 1) * m_rn[lvl];
                }
                const int rn = m_rn[lvl];
                const int e = g - lo, pe = m_rp[lvl] * rn;
                x[t] = e < pe ? static_cast<V>(P[m_pb[lvl] + static_cast<int64_t>(e / rn) * m_ncp[lvl] + e % rn])
                              : sku[m_sk[lvl] + (e - pe)];
            }
#pragma unroll
            for (int t = 0; t < 8; ++t)
                if (g0 + t * kCombBlock < nd) chain[g0 + t * kCombBlock] = x[t];
        }
    }
    const int q = tid / kCombQ, jq = tid % kCombQ;
    const int per = (lp.nitems + 3) / 4;
    const int i0 = min(lp.nitems, q * per), i1 = min(lp.nitems, i0 + per);
    const int pr = (rleaf + 3) / 4;
    const int k0 = min(rleaf, q * pr), k1 = min(rleaf, k0 + pr);
    const TP* Pl = P + (depth >= 1 ? m_pleaf : 0);
    auto near_sum = [&](int j) {
        V near = 0;
        if (j < lp.rows) {
            // the last batch clamps its indexes and adds only the items in range
            for (int it = i0; it < i1; it += kNearBatch<V>) {
                V x[kNearBatch<V>];
#pragma unroll
                for (int t = 0; t < kNearBatch<V>; ++t) x[t] = pc[static_cast<int64_t>(min(it + t, i1 - 1)) * lp.ld + j];
#pragma unroll
                for (int t = 0; t < kNearBatch<V>; ++t)
                    if (it + t < i1) near += x[t];
            }
        }
        return near;
    };
    TP pv[kLeafBatch<V>];
    auto leaf_load = [&](int k, int j) {
        const int jc = min(j, lp.rows - 1);
#pragma unroll
        for (int t = 0; t < kLeafBatch<V>; ++t) pv[t] = Pl[static_cast<int64_t>(min(k + t, k1 - 1)) * lp.rows + jc];
    };
    const V near0 = near_sum(jq);
    const bool pre = k1 > k0 && k1 - k0 <= kLeafBatch<V>;
    if (pre) leaf_load(k0, jq);
    double sc0 = 1.0;
    int64_t dst0 = 0;
    if (q == 0 && jq < lp.rows) {
        const int64_t pos = lp.start + jq;
        sc0 = (b.arg[o] & 1) ? D.c[pos] : 1.0;
        dst0 = (b.arg[o] & 2) ? pos : D.perm[pos];
    }
    __syncthreads();

    // 3. downward pass.  Through the composites: u~_leaf = S2S(leaf) + the sum
    // over ancestors h of (the leaf's block of C_h)^T S2S(h), every (level, row)
    // sum at once from shared memory, the levels added in order.
    if (comp && rleaf > 0) {
        const int nd = static_cast<int>(need);
        for (int e = tid; e < (depth - 1) * rleaf; e += kCombBlock) {
            const int lvl = 1 + e / rleaf, j = e % rleaf;
            int off = 0;
            for (int l = 1; l < lvl; ++l) off += m_rn[l] * (1 + rleaf);
            const int rn = m_rn[lvl];
            const V* S = chain + off;
            const V* Cb = chain + off + rn + j;
            V acc = 0;
            for (int i = 0; i < rn; ++i) acc += Cb[i * rleaf] * S[i];
            chain[nd + e] = acc;
        }
        __syncthreads();
        for (int j = tid; j < rleaf; j += kCombBlock) {
            V s = tot[0][j];
            for (int l = 0; l < depth - 1; ++l) s += chain[nd + l * rleaf + j];
            tot[0][j] = s;
        }
        __syncthreads();
    }
    // downward chain: u~_child = S2S(child) + (P_parent^T u~_parent)[child's columns]
    int cur = 0;
    int64_t off = 0;
    for (int lvl = top + 1; lvl <= depth; ++lvl) {
        const int rp = m_rp[lvl], rn = m_rn[lvl];
        for (int j = tid; j < rn; j += kCombBlock) {
            V acc = 0;
            if (staged) {
                const V* Ps = chain + off;
                for (int i = 0; i < rp; ++i) acc += Ps[i * rn + j] * tot[cur][i];
                tot[cur ^ 1][j] = Ps[static_cast<int64_t>(rp) * rn + j] + acc;
            } else {
                const TP* Pm = P + m_pb[lvl];
                const int ncp = m_ncp[lvl];
                for (int i = 0; i < rp; ++i) acc += static_cast<V>(Pm[static_cast<int64_t>(i) * ncp + j]) * tot[cur][i];
                tot[cur ^ 1][j] = sku[m_sk[lvl] + j] + acc;
            }
        }
        off += static_cast<int64_t>(rp + 1) * rn;
        __syncthreads();
        cur ^= 1;
    }
    for (int j0 = 0; j0 < lp.rows; j0 += kCombQ) {
        const int j = j0 + jq;
        const V near = j0 == 0 ? near0 : near_sum(j);
        V f = 0;
        for (int k = k0; k < k1; k += kLeafBatch<V>) {
            if (!(pre && j0 == 0)) leaf_load(k, j);
#pragma unroll
            for (int t = 0; t < kLeafBatch<V>; ++t)
                if (k + t < k1) f += static_cast<V>(pv[t]) * tot[cur][k + t];
        }
        quarter[0][q][jq] = near;
        quarter[1][q][jq] = f;
        __syncthreads();
        if (q == 0 && j < lp.rows) {
            const V nsum = (quarter[0][0][jq] + quarter[0][1][jq]) + (quarter[0][2][jq] + quarter[0][3][jq]);
            const V fsum = (quarter[1][0][jq] + quarter[1][1][jq]) + (quarter[1][2][jq] + quarter[1][3][jq]);
            double sc = sc0;
            int64_t dst = dst0;
            if (j0 > 0) {
                const int64_t pos = lp.start + j;
                sc = (b.arg[o] & 1) ? D.c[pos] : 1.0;
                dst = (b.arg[o] & 2) ? pos : D.perm[pos];
            }
            b.y[o][dst] = sc * static_cast<double>(nsum + fsum);
        }
        __syncthreads();
    }
}


// cnt values into shared memory, dst[e] = load(e), the workgroup's kBlock threads
// with eight loads in flight each (the loads of a batch are issued before its stores)
template <typename V, typename Load>
__device__ inline void stage_batched(int cnt, Load&& load, V* dst) {
    for (int e0 = threadIdx.x; e0 < cnt; e0 += 8 * kBlock) {
        V v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = load(min(e0 + q * kBlock, cnt - 1));
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (e0 + q * kBlock < cnt) dst[e0 + q * kBlock] = v[q];
    }
}

// ---- S2N by level (operators with large ranks) ---------------------------------
// u~_h = S2S(h) + (P_parent^T u~_parent)[h's columns] for every node h of level
// lvl (b.arg), in place on the far-field potentials, parents' potentials already
// complete: one workgroup per node, thread j owns column j of the parent's P
// slice (consecutive threads read consecutive entries of a P row) and sums over
// the parent's rows in increasing order, the arithmetic of the combine's walk.
template <typename V, typename TP>
__global__ void __launch_bounds__(kBlock) k_s2n(Batch b) {
    const int64_t u = blockIdx.x;
    const int o = batch_op(b, u);
    const OpDev& D = *b.op[o];
    const int lvl = b.arg[o];
    const int64_t h = (int64_t(1) << lvl) + (u - b.pre[o]);
    const int64_t p = h >> 1;
    const int rn = D.rank[h], rp = D.rank[p], ncp = D.ncand[p];
    const int coff = (h & 1) ? D.rank[2 * p] : 0;
    const TP* Pp = static_cast<const TP*>(D.P) + D.poff[p] + coff;
    V* sku = static_cast<V*>(D.sku);
    const int64_t sp = D.skoff[p], sh = D.skoff[h];
    constexpr int IB = 16;   // rows of P in flight per thread
    for (int j = threadIdx.x; j < rn; j += blockDim.x) {
        V acc = 0;
        // the last batch clamps its indexes and adds only the rows in range
        for (int i0 = 0; i0 < rp; i0 += IB) {
            V pv[IB], uv[IB];
#pragma unroll
            for (int t = 0; t < IB; ++t) {
                const int i = min(i0 + t, rp - 1);
                pv[t] = static_cast<V>(Pp[static_cast<int64_t>(i) * ncp + j]);
                uv[t] = sku[sp + i];
            }
#pragma unroll
            for (int t = 0; t < IB; ++t)
                if (i0 + t < rp) acc += pv[t] * uv[t];
        }
        sku[sh + j] = sku[sh + j] + acc;
    }
}

// Several right-hand sides: workgroup (node h of level lvl, 64 of its rank
// columns from 64 blockIdx.y on); lane l owns column j = 64 blockIdx.y + l.  The
// parent's potentials are staged in shared memory kS2nRows rows at a time (one
// row's kMaxRhs values together, read back as broadcasts); wave w adds the rows
// w, w + 4, ... in increasing order, and the four waves' sums are added in wave
// order.
constexpr int kS2nRows = 256;

template <typename V, typename TP>
__global__ void __launch_bounds__(kBlock) k_s2n_m(Batch b) {
    constexpr int NW = kBlock / kWave;
    static_assert(NW * kWave <= kS2nRows, "the waves' sums reuse the staging rows");
    __shared__ V st[kS2nRows * kMaxRhs];
    const int64_t u = blockIdx.x;
    const int o = batch_op(b, u);
    const OpDev& D = *b.op[o];
    const int lvl = b.arg[o];
    const int64_t h = (int64_t(1) << lvl) + (u - b.pre[o]);
    const int64_t p = h >> 1;
    const int rn = D.rank[h];
    const int j0 = static_cast<int>(blockIdx.y) * kWave;
    if (j0 >= rn) return;   // the whole workgroup
    const int rp = D.rank[p], ncp = D.ncand[p];
    const int coff = (h & 1) ? D.rank[2 * p] : 0;
    const TP* Pp = static_cast<const TP*>(D.P) + D.poff[p] + coff;
    V* sku = static_cast<V*>(D.sku);
    const int64_t ldsk = D.ldsk, sp = D.skoff[p], sh = D.skoff[h];
    const int last = b.nrhs - 1;
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int j = min(j0 + lane, rn - 1);
    V acc[kMaxRhs];
#pragma unroll
    for (int c = 0; c < kMaxRhs; ++c) acc[c] = 0;
    constexpr int IB = 4;   // rows of P in flight per lane
    for (int r0 = 0; r0 < rp; r0 += kS2nRows) {
        const int nrow = min(kS2nRows, rp - r0);
        __syncthreads();   // the previous rows are read
        stage_batched(nrow * kMaxRhs, [&](int e) {
            const int i = e / kMaxRhs, c = e % kMaxRhs;
            return sku[min(c, last) * ldsk + sp + r0 + i];
        }, st);
        __syncthreads();
        for (int i = w; i < nrow; i += NW * IB) {
            V pv[IB];
#pragma unroll
            for (int t = 0; t < IB; ++t)
                pv[t] = static_cast<V>(Pp[static_cast<int64_t>(r0 + min(i + t * NW, nrow - 1)) * ncp + j]);
#pragma unroll
            for (int t = 0; t < IB; ++t) {
                if (i + t * NW >= nrow) break;
                V pot[kMaxRhs];
                __builtin_memcpy(pot, st + (i + t * NW) * kMaxRhs, sizeof(pot));
#pragma unroll
                for (int c = 0; c < kMaxRhs; ++c) acc[c] += pv[t] * pot[c];
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kMaxRhs; ++c) st[(w * kMaxRhs + c) * kWave + lane] = acc[c];
    __syncthreads();
    for (int e = threadIdx.x; e < kMaxRhs * kWave; e += kBlock) {
        const int c = e / kWave, l = e % kWave;
        if (c > last || j0 + l >= rn) continue;
        V t = st[c * kWave + l];
#pragma unroll
        for (int q = 1; q < NW; ++q) t += st[(q * kMaxRhs + c) * kWave + l];
        V* dst = sku + c * ldsk + sh + j0 + l;
        *dst = *dst + t;
    }
}

// ---- several right-hand sides (2 <= nrhs <= 16) -------------------------------
// The same phases with every matrix element loaded once for all columns: each
// lane keeps one partial sum per right-hand side.
template <typename V, typename TP>
__global__ void k_n2s_m(Batch b) {
    const int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x / kWave) + threadIdx.x / kWave;
    if (u >= b.pre[b.nops]) return;
    const int o = batch_op(b, u);
    const OpDev& D = *b.op[o];
    const int lvl = b.arg[o];
    const RowTask T = D.rows[D.row_begin[lvl] + (u - b.pre[o])];
    const int nc = D.ncand[T.h];
    const TP* row = static_cast<const TP*>(D.P) + D.poff[T.h] + static_cast<int64_t>(T.i) * nc;
    V* skw = static_cast<V*>(D.skw);
    const bool leaf = lvl == D.depth;
    const V* in = leaf ? static_cast<const V*>(D.w) + D.start[T.h] : skw + D.skoff[2 * T.h];
    const int64_t ldin = leaf ? D.n : D.ldsk;
    const int lane = threadIdx.x % kWave;
    V acc[kMaxRhs];
#pragma unroll
    for (int c = 0; c < kMaxRhs; ++c) acc[c] = 0;
    // loads are unconditional (columns past nrhs repeat the last one) so that
    // they issue together; only the stores are guarded
    const int last = b.nrhs - 1;
    for (int j = lane; j < nc; j += kWave) {
        const V p = val<V>(row[j]);
#pragma unroll
        for (int c = 0; c < kMaxRhs; ++c) acc[c] += p * in[min(c, last) * ldin + j];
    }
#pragma unroll
    for (int c = 0; c < kMaxRhs; ++c) {
        if (c >= b.nrhs) break;
        const V t = wave_sum(acc[c]);
        if (lane == 0) skw[c * D.ldsk + D.skoff[T.h] + T.i] = t;
    }
}

// The same rows, workgroups per node of level lvl (b.arg), kN2sNodeRows rows
// each (blockIdx.y: the chunk of rows): the node's input (its points' staged
// values at the leaves, its children's skeleton values above) in shared memory,
// kMaxRhs columns of nc values, then each wave forms four rows at once with
// k_n2s_m's arithmetic per row (lane l: the candidates l, l + 64, ... in
// increasing order, then the wave's butterfly); the input values read from
// shared memory serve the four rows.
constexpr int kN2sWaveRows = 4;
constexpr int kN2sNodeRows = kN2sWaveRows * (kBlock / kWave);

template <typename V, typename TP>
__global__ void __launch_bounds__(kBlock) k_n2s_node_m(Batch b) {
    extern __shared__ char n2s_dyn[];
    V* xin = reinterpret_cast<V*>(n2s_dyn);
    const int64_t u = blockIdx.x;
    const int o = batch_op(b, u);
    const OpDev& D = *b.op[o];
    const int lvl = b.arg[o];
    const int64_t h = (int64_t(1) << lvl) + (u - b.pre[o]);
    const int nc = D.ncand[h], rk = D.rank[h];
    const int i0 = static_cast<int>(blockIdx.y) * kN2sNodeRows;
    if (i0 >= rk) return;   // the whole workgroup
    const bool leaf = lvl == D.depth;
    const V* in = leaf ? static_cast<const V*>(D.w) + D.start[h] : static_cast<const V*>(D.skw) + D.skoff[2 * h];
    const int64_t ldin = leaf ? D.n : D.ldsk;
    const int last = b.nrhs - 1;
    stage_batched(kMaxRhs * nc, [&](int e) {
        const int c = e / nc, j = e % nc;
        return in[min(c, last) * ldin + j];
    }, xin);
    __syncthreads();
    const TP* P = static_cast<const TP*>(D.P) + D.poff[h];
    V* skw = static_cast<V*>(D.skw);
    const int lane = threadIdx.x % kWave;
    const int ir = i0 + (static_cast<int>(threadIdx.x) / kWave) * kN2sWaveRows;   // the wave's first row
    if (ir >= rk) return;
    const TP* rows[kN2sWaveRows];
#pragma unroll
    for (int t = 0; t < kN2sWaveRows; ++t) rows[t] = P + static_cast<int64_t>(min(ir + t, rk - 1)) * nc;
    V acc[kN2sWaveRows][kMaxRhs];
#pragma unroll
    for (int t = 0; t < kN2sWaveRows; ++t)
#pragma unroll
        for (int c = 0; c < kMaxRhs; ++c) acc[t][c] = 0;
    for (int j = lane; j < nc; j += kWave) {
        V p[kN2sWaveRows];
#pragma unroll
        for (int t = 0; t < kN2sWaveRows; ++t) p[t] = val<V>(rows[t][j]);
#pragma unroll
        for (int c = 0; c < kMaxRhs; ++c) {
            const V x = xin[c * nc + j];
#pragma unroll
            for (int t = 0; t < kN2sWaveRows; ++t) acc[t][c] += p[t] * x;
        }
    }
#pragma unroll
    for (int t = 0; t < kN2sWaveRows; ++t)
#pragma unroll
        for (int c = 0; c < kMaxRhs; ++c)
            if (ir + t < rk && c <= last) {   // wave-uniform
                const V s = wave_sum(acc[t][c]);
                if (lane == 0) skw[c * D.ldsk + D.skoff[h] + ir + t] = s;
            }
}
// largest shared-memory input of k_n2s_node_m (nodes with more candidates take k_n2s_m)
constexpr int kN2sNodeBytes = 65536;

template <typename V, typename TF>
__global__ void k_s2s_m(Batch b) {
    const int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x / kWave) + threadIdx.x / kWave;
    if (u >= b.pre[b.nops]) return;
    const int o = batch_op(b, u);
    const OpDev& D = *b.op[o];
    const RowTask T = D.rows[u - b.pre[o]];
    const int nc = D.far_cols[T.h];
    const TF* row = static_cast<const TF*>(D.far) + D.far_off[T.h] + static_cast<int64_t>(T.i) * nc;
    const int32_t* cm = D.far_colmap + D.far_colbase[T.h];
    const V sc = D.fscale ? static_cast<V>(D.fscale[T.h]) : V(1);
    const V* skw = static_cast<const V*>(D.skw);
    V* sku = static_cast<V*>(D.sku);
    const int lane = threadIdx.x % kWave;
    V acc[kMaxRhs];
#pragma unroll
    for (int c = 0; c < kMaxRhs; ++c) acc[c] = 0;
    const int last = b.nrhs - 1;
    for (int j = lane; j < nc; j += kWave) {
        const V p = val<V>(row[j]);
        const int64_t col = cm[j];
#pragma unroll
        for (int c = 0; c < kMaxRhs; ++c) acc[c] += p * skw[min(c, last) * D.ldsk + col];
    }
#pragma unroll
    for (int c = 0; c < kMaxRhs; ++c) {
        if (c >= b.nrhs) break;
        const V t = wave_sum(acc[c]);
        if (lane == 0) sku[c * D.ldsk + D.skoff[T.h] + T.i] = t * sc;
    }
}

// ---- several right-hand sides: partial sums of busy leaves pre-added ------------
// A leaf near many others has many near-field items, each with its own partial
// sums; the one workgroup that combines the leaf would add them all.  Here the
// items of such a leaf are added in groups of gstep, in item order, into the
// group's first item (grid: leaf x group x column), so that its combine reads
// one partial per group.
template <typename V>
__global__ void __launch_bounds__(kBlock) k_part_reduce(Batch b) {
    const int64_t u = blockIdx.x;
    const int o = batch_op(b, u);
    const OpDev& D = *b.op[o];
    const LeafPlan lp = D.leaves[u - b.pre[o]];
    const int k = static_cast<int>(blockIdx.y), c = static_cast<int>(blockIdx.z);
    const int q0 = k * lp.gstep;
    if (lp.gstep <= 1 || q0 >= lp.nitems) return;
    const int cnt = min(lp.gstep, lp.nitems - q0);
    V* pc = static_cast<V*>(D.part) + c * D.ldp + lp.part_off + static_cast<int64_t>(q0) * lp.ld;
    for (int j = threadIdx.x; j < lp.rows; j += blockDim.x) {
        V x[kReduceGroup];
#pragma unroll
        for (int t = 0; t < kReduceGroup; ++t) x[t] = pc[static_cast<int64_t>(min(t, cnt - 1)) * lp.ld + j];
        V acc = x[0];
#pragma unroll
        for (int t = 1; t < kReduceGroup; ++t)
            if (t < cnt) acc += x[t];
        pc[j] = acc;
    }
}

// combine for several right-hand sides: the ancestor potentials of all columns
// sit side by side in shared memory, so each P element is read once.  One
// workgroup of kCombBlock threads per leaf, in the phases of k_combine: the
// ranks and offsets along the path; the leaf's potentials, either through the
// composites of its ancestors (s2n_comp: one step, no chain), or already formed
// by a per-level downward pass (s2n_multi), or else by the chain walk from level
// 1 with the path's P slices staged in shared memory in one batch (where they
// fit); then per row the near partial sums (float32: two halves of the workgroup
// over half of the items each, added in a fixed order, two items of every column
// in flight) and P_leaf^T u~ with eight of its entries in flight.
template <typename V> constexpr int kStageM = sizeof(V) == 4 ? kMaxRhs * (kCombBlock / 2) : 1024;
template <typename V> constexpr bool kSplitM = sizeof(V) == 4;
template <typename V> constexpr int kItemBatchM = sizeof(V) == 4 ? 2 : 1;

template <typename V, typename TP>
__global__ void __launch_bounds__(kCombBlock) k_combine_m(Batch b) {
    constexpr int kHalf = kCombBlock / 2;
    constexpr int IB = kItemBatchM<V>;
    __shared__ V tot[2][kMaxRhs * kMaxRank];
    __shared__ V stage[kStageM<V>];   // the chain's P slices, then the second half's near sums
    __shared__ int m_rn[kMaxLevels + 1], m_rp[kMaxLevels + 1], m_ncp[kMaxLevels + 1], m_cs[kMaxLevels + 1],
        m_so[kMaxLevels + 1];
    __shared__ int64_t m_pb[kMaxLevels + 1], m_sk[kMaxLevels + 1], m_cb[kMaxLevels + 1], m_pleaf;
    const int64_t u = blockIdx.x;
    const int o = batch_op(b, u);
    const OpDev& D = *b.op[o];
    const LeafPlan lp = D.leaves[u - b.pre[o]];
    const bool comp = D.s2n_comp && D.row_total > 0 && D.depth >= 2;
    const TP* P = static_cast<const TP*>(D.P);
    const V* sku = static_cast<const V*>(D.sku);
    const int depth = D.row_total > 0 ? D.depth : 0;
    const int nr = b.nrhs, last = nr - 1;   // loads past nrhs repeat the last column (unguarded, batched)
    const int64_t ldp = D.ldp, ldsk = D.ldsk;
    const int tid = threadIdx.x;
    if (tid >= 1 && tid <= depth) {
        const int64_t node = static_cast<int64_t>(lp.heap) >> (depth - tid);
        m_rn[tid] = D.rank[node];
        m_sk[tid] = D.skoff[node];
        if (tid >= 2) {
            const int64_t par = node >> 1;
            m_rp[tid] = D.rank[par];
            m_ncp[tid] = D.ncand[par];
            m_pb[tid] = D.poff[par] + ((node & 1) ? D.rank[2 * par] : 0);
        }
        if (comp && tid < depth) {
            // the leaf's block of columns in the composite of its ancestor at level tid
            const LeafRun lr = leaf_run(D.skoff, D.rank, depth, node, tid);
            m_cs[tid] = lr.nlk;
            m_cb[tid] = D.coff[node] + (D.skoff[lp.heap] - lr.base);
        }
    }
    if (tid == 0 && depth >= 1) m_pleaf = D.poff[lp.heap];
    __syncthreads();
    // the walk starts at level 1, or at the leaf when a per-level downward pass
    // (or the composites below) completes every potential
    const int top = (D.s2n_multi || comp) && depth >= 1 ? depth : 1;
    if (depth >= 1) {
        const int r1 = m_rn[top];
        for (int e = tid; e < nr * r1; e += kCombBlock) {
            const int c = e / r1, i = e % r1;
            tot[0][c * kMaxRank + i] = sku[c * ldsk + m_sk[top] + i];
        }
    }
    // Through the composites: the leaf's potentials are its own far field plus,
    // for each ancestor h (levels 1 .. depth - 1), the leaf's block of columns of
    // C_h transposed times h's far field (the chain of P slices from h down to
    // the leaf is that block).  The ancestors' far fields are staged in shared
    // memory, every (level, column, row) sum is formed at once into the second
    // potential buffer, and the levels are added in order.  The host enables this
    // only where both fit (nr x the ancestors' ranks <= the staging, (depth - 1) x
    // nr x the leaf's rank <= one potential buffer).
    if (comp) {
        const int rleaf = m_rn[depth], nl = depth - 1, per = nr * rleaf;
        int so = 0;
        for (int lvl = 1; lvl < depth; ++lvl) {
            const int rn = m_rn[lvl];
            if (tid == 0) m_so[lvl] = so;
            for (int e = tid; e < nr * rn; e += kCombBlock) stage[so + e] = sku[(e / rn) * ldsk + m_sk[lvl] + e % rn];
            so += nr * rn;
        }
        __syncthreads();
        const V* Cm = static_cast<const V*>(D.comp);
        for (int e = tid; e < nl * per; e += kCombBlock) {
            const int lvl = 1 + e / per, r = e % per, c = r / rleaf, j = r % rleaf;
            const int rn = m_rn[lvl], cs = m_cs[lvl];
            const V* Sv = stage + m_so[lvl] + c * rn;
            const V* Cp = Cm + m_cb[lvl] + j;
            V acc = 0;
            for (int i0 = 0; i0 < rn; i0 += 8) {
                V cv[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) cv[t] = Cp[static_cast<int64_t>(min(i0 + t, rn - 1)) * cs];
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    if (i0 + t < rn) acc += cv[t] * Sv[i0 + t];
            }
            tot[1][e] = acc;
        }
        __syncthreads();
        for (int e = tid; e < per; e += kCombBlock) {
            V s = tot[0][(e / rleaf) * kMaxRank + e % rleaf];
            for (int l = 0; l < nl; ++l) s += tot[1][l * per + e];
            tot[0][(e / rleaf) * kMaxRank + e % rleaf] = s;
        }
    }
    // the chain walk; as many consecutive levels' P slices as fit are staged in
    // shared memory at a time (one batch of loads), a level too large for it
    // reads P from global memory
    int cur = 0;
    for (int l0 = top + 1; l0 <= depth;) {
        int l1 = l0, nd = 0;
        while (l1 <= depth && nd + m_rp[l1] * m_rn[l1] <= kStageM<V>) {
            nd += m_rp[l1] * m_rn[l1];
            ++l1;
        }
        const bool staged = l1 > l0;
        if (!staged) l1 = l0 + 1;
        if (staged && nd > 0) {
            // each thread's elements come in increasing order, so its level only advances
            int lvl = l0, lo = 0, sz = m_rp[l0] * m_rn[l0];
            for (int g0 = tid; g0 < nd; g0 += 8 * kCombBlock) {
                V x[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int g = min(g0 + t * kCombBlock, nd - 1);
                    while (g >= lo + sz) {
                        lo += sz;
                        ++lvl;
                        sz = m_rp[lvl] * m_rn[lvl];
                    }
                    const int rn = m_rn[lvl], e = g - lo;
                    x[t] = static_cast<V>(P[m_pb[lvl] + static_cast<int64_t>(e / rn) * m_ncp[lvl] + e % rn]);
                }
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    if (g0 + t * kCombBlock < nd) stage[g0 + t * kCombBlock] = x[t];
            }
        }
        __syncthreads();
        int off = 0;
        for (int lvl = l0; lvl < l1; ++lvl) {
            const int rp = m_rp[lvl], rn = m_rn[lvl], ncp = m_ncp[lvl];
            const TP* Pm = P + m_pb[lvl];
            for (int j = tid; j < rn; j += kCombBlock) {
                V sv[kMaxRhs];
#pragma unroll
                for (int c = 0; c < kMaxRhs; ++c) sv[c] = sku[min(c, last) * ldsk + m_sk[lvl] + j];
                V acc[kMaxRhs];
#pragma unroll
                for (int c = 0; c < kMaxRhs; ++c) acc[c] = 0;
                if (staged) {
                    const V* Ps = stage + off;
                    for (int i = 0; i < rp; ++i) {
                        const V p = Ps[i * rn + j];
#pragma unroll
                        for (int c = 0; c < kMaxRhs; ++c) acc[c] += p * tot[cur][min(c, last) * kMaxRank + i];
                    }
                } else {
                    for (int i = 0; i < rp; ++i) {
                        const V p = static_cast<V>(Pm[static_cast<int64_t>(i) * ncp + j]);
#pragma unroll
                        for (int c = 0; c < kMaxRhs; ++c) acc[c] += p * tot[cur][min(c, last) * kMaxRank + i];
                    }
                }
#pragma unroll
                for (int c = 0; c < kMaxRhs; ++c)
                    if (c < nr) tot[cur ^ 1][c * kMaxRank + j] = sv[c] + acc[c];
            }
            off += rp * rn;
            __syncthreads();
            cur ^= 1;
        }
        l0 = l1;
    }
    __syncthreads();
    const int rleaf = depth >= 1 ? m_rn[depth] : 0;
    const TP* Pl = P + (depth >= 1 ? m_pleaf : 0);
    const V* pc = static_cast<const V*>(D.part) + lp.part_off;
    const int half = kSplitM<V> ? tid / kHalf : 0;
    const int jt = kSplitM<V> ? tid % kHalf : tid;
    constexpr int rstep = kSplitM<V> ? kHalf : kCombBlock;
    // a busy leaf's partial sums were pre-added in groups: one per group
    const int gs = max(lp.gstep, 1);
    const int ng = (lp.nitems + gs - 1) / gs;
    const int64_t qld = static_cast<int64_t>(gs) * lp.ld;
    const int ih = kSplitM<V> ? (ng + 1) / 2 : ng;
    const int i0 = min(ng, half * ih), i1 = min(ng, i0 + ih);
    for (int j0 = 0; j0 < lp.rows; j0 += rstep) {
        const int j = j0 + jt;
        const bool live = j < lp.rows;
        V f[kMaxRhs];
#pragma unroll
        for (int c = 0; c < kMaxRhs; ++c) f[c] = 0;
        if (live) {
            // IB items in flight; the last batch clamps and adds only the items in range
            for (int q = i0; q < i1; q += IB) {
                V x[IB][kMaxRhs];
#pragma unroll
                for (int t = 0; t < IB; ++t) {
                    const V* pq = pc + static_cast<int64_t>(min(q + t, i1 - 1)) * qld + j;
#pragma unroll
                    for (int c = 0; c < kMaxRhs; ++c) x[t][c] = pq[min(c, last) * ldp];
                }
#pragma unroll
                for (int t = 0; t < IB; ++t)
                    if (q + t < i1) {
#pragma unroll
                        for (int c = 0; c < kMaxRhs; ++c) f[c] += x[t][c];
                    }
            }
        }
        if (kSplitM<V>) {
            if (half == 1 && live)
                for (int c = 0; c < nr; ++c) stage[c * kHalf + jt] = f[c];
            __syncthreads();
        }
        if (half == 0 && live) {
            if (kSplitM<V>)
                for (int c = 0; c < nr; ++c) f[c] += stage[c * kHalf + jt];
            for (int i = 0; i < rleaf; i += 8) {
                TP pv[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) pv[t] = Pl[static_cast<int64_t>(min(i + t, rleaf - 1)) * lp.rows + j];
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    if (i + t < rleaf) {
                        const V p = static_cast<V>(pv[t]);
#pragma unroll
                        for (int c = 0; c < kMaxRhs; ++c) f[c] += p * tot[cur][min(c, last) * kMaxRank + i + t];
                    }
            }
            const int64_t pos = lp.start + j;
            const double sc = (b.arg[o] & 1) ? D.c[pos] : 1.0;
            const int64_t dst = (b.arg[o] & 2) ? pos : D.perm[pos];
#pragma unroll
            for (int c = 0; c < kMaxRhs; ++c)
                if (c < nr) b.y[o][c * D.n + dst] = sc * static_cast<double>(f[c]);
        }
        if (kSplitM<V>) __syncthreads();   // stage is rewritten by the next rows
    }
}

// ---- half-precision near field on matrix cores --------------------------------
// Packed tile layout: the block of near pair (a, b) is ld_a x kc_b (kc_b = |b|
// rounded up to 8, zero padded) and element (r, k) sits at
// ((k / 8) * ld_a + r) * 8 + k % 8, so one lane's 16-byte load is the 8
// consecutive columns of one row that a 16x16x32 matrix instruction takes.
// The vectors are staged per leaf as w = s (hi + lo) with hi, lo in float16
// and s a power of two per leaf and column, so that the pair carries about 22
// bits of w whatever its range; partial sums are float32.
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef float f4_t __attribute__((ext_vector_type(4)));
constexpr int kMmaRowTiles = 8;   // 16-row tiles per work item

// stage w = c * x (tree order, float32) and its half-precision hi/lo pair per
// leaf; one workgroup per leaf.  The halves of padded position p and column c
// sit at (p / 8) 8 nrhs + 8 c + p % 8: the 8 consecutive points of one column
// that a matrix-core lane takes are 16 contiguous bytes, and those of the
// nrhs columns follow each other.
__global__ void __launch_bounds__(kCombBlock) k_prep_mma(Batch b) {
    __shared__ float smax[kMaxRhs];
    const int64_t u = blockIdx.x;
    const int o = batch_op(b, u);
    const OpDev& D = *b.op[o];
    const int64_t a = u - b.pre[o];
    const LeafPlan lp = D.leaves[a];
    const int nr = lp.rows, nrhs = b.nrhs;
    const int kc = (nr + 7) & ~7;
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const bool norm = b.arg[o] & 1, gather = !(b.arg[o] & 2);
    float* w = static_cast<float*>(D.w);
    // w in float32 and each column's largest magnitude: one wave per column, eight
    // points per lane in flight (a column's values are loaded before any is stored)
    for (int c = wave; c < nrhs; c += nw) {
        const double* x = b.x[o] + static_cast<int64_t>(c) * D.n;
        float* wc = w + static_cast<int64_t>(c) * D.n + lp.start;
        float m = 0.0f;
        for (int p0 = 0; p0 < nr; p0 += 8 * kWave) {
            float v[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int64_t pos = lp.start + min(p0 + t * kWave + lane, nr - 1);
                const double sc = norm ? D.c[pos] : 1.0;
                v[t] = static_cast<float>(sc * x[gather ? D.perm[pos] : pos]);
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int p = p0 + t * kWave + lane;
                if (p < nr) {
                    wc[p] = v[t];
                    m = fmaxf(m, fabsf(v[t]));
                }
            }
        }
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, kWave));
        if (lane == 0) smax[c] = m;
    }
    __syncthreads();   // w and the maxima are complete (the workgroup's own stores)
    _Float16* hi = static_cast<_Float16*>(D.wh);
    _Float16* lo = hi + kMaxRhs * D.ldw;
    // the halves of 8 consecutive points of one column per thread: two 16-byte stores
    const int groups = kc / 8;
    for (int e = threadIdx.x; e < nrhs * groups; e += blockDim.x) {
        const int c = e / groups, g = e % groups;
        const float m = smax[c];
        const int ex = m > 0.0f ? ilogbf(m) : 0;
        h8_t hv, lv;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int p = g * 8 + q;
            float h = 0.0f, l = 0.0f;
            if (p < nr) {
                const float v = ldexpf(w[c * D.n + lp.start + p], 13 - ex);   // |v| < 2^14
                const _Float16 vh = static_cast<_Float16>(v);
                h = static_cast<float>(vh);
                l = v - h;
            }
            hv[q] = static_cast<_Float16>(h);
            lv[q] = static_cast<_Float16>(l);
        }
        const int64_t at = (lp.wpad + g * 8) * nrhs + c * 8;
        *reinterpret_cast<h8_t*>(hi + at) = hv;
        *reinterpret_cast<h8_t*>(lo + at) = lv;
        if (g == 0) D.wsc[a * kMaxRhs + c] = ldexpf(1.0f, ex - 13);
    }
    if (a == 0 && threadIdx.x < 8) hi[2 * kMaxRhs * D.ldw + threadIdx.x] = static_cast<_Float16>(0.0f);   // the zero block
}

// Workgroups over segments of the packed near field.  A segment is a run of
// tile steps (32 columns of one tile) of one leaf; it may start or end inside a
// tile.  With several columns the plan gives each workgroup an equal share of
// all steps (a list of segments), so every wave streams the same number of steps
// and the launch ends with its waves busy (runs of whole tiles per wave, two
// rounds of items over the wave slots, had left the last ~100 us of the launch
// half empty); with one column each workgroup takes one tile.  The four waves of
// a workgroup take the same segments, each for its own group of at most 8 row
// tiles of 16 rows (wave g takes groups g, g + 4, ...).  A segment's products
// are scaled by tile and vector scales at the end of each of its tiles' columns
// and added in step order; the segment writes one partial-sum slot of its leaf,
// so the result does not depend on when or where it runs.
//
// The steps of a segment form one sequence, software-pipelined: the loads of
// step s + 1 (8 A fragments, 2 B fragments, 16 bytes per lane each) are issued
// before the matrix instructions of step s, so every wave keeps two steps of
// tile data in flight.  No load is guarded: a row past the group (or past the
// tile) reads the group's last row, whose products land in output rows that are
// never stored, and a column group past the tile reads the tile's last group
// against a zero B fragment; B lanes past nrhs or past the tile read a block of
// zeros kept after the staged vectors.
typedef const __attribute__((address_space(1))) h8_t gh8_t;

// a 16-byte load through a global-memory pointer (not a flat one)
__device__ inline h8_t gload16(const _Float16* p) { return *(gh8_t*)(p); }

struct MmaStep {
    h8_t a[kMmaRowTiles];
    h8_t bh, bl;
};

// position in a segment's step sequence: tile q of the segment and its fields
// (wave-uniform), columns k0 .. k0 + 31 up to kend (the tile's padded width, or
// where the segment stops inside its last tile), the tile's scale and the vector
// scale of this lane's column
struct MmaPos {
    int q, k0, kc, kend, col_pos;
    int64_t tile_off;
    float ts;
    float wl;   // vector scale of this lane's column (column li of the B operand)
};


__device__ inline void mma_tile(const OpDev& D, int t, int li, MmaPos& p) {
    cNearItem* T = (cNearItem*)D.tiles + t;
    p.kc = (T->ncols + 7) & ~7;
    p.kend = p.kc;
    p.col_pos = T->col_pos;
    p.tile_off = T->tile_off;
    p.ts = D.nscale ? *((cfloat*)D.nscale + T->tile) : 1.0f;
    p.wl = D.wsc[static_cast<int64_t>(T->leaf_b) * kMaxRhs + li];
}

template <bool kUp>
__global__ void __launch_bounds__(kBlock) k_l2l_mma(Batch b) {
    if (kUp && static_cast<int>(blockIdx.x) < b.up) {
        leaf_n2s<float>(b, blockIdx.x);
        return;
    }
    int64_t wg = static_cast<int64_t>(blockIdx.x) - b.up;
    if (wg >= b.pre[b.nops]) return;
    if (b.flip) wg = b.pre[b.nops] - 1 - wg;
    const int o = batch_op(b, wg);
    const OpDev& D = *b.op[o];
    const bool multi = b.nrhs > 1;
    // no workgroup list: one segment per workgroup
    const int32_t* wlist = multi ? D.wseg : D.wseg1;
    const int64_t wi = wg - b.pre[o];
    const int seg0 = wlist ? wlist[wi] : static_cast<int>(wi);
    const int nseg = wlist ? wlist[wi + 1] - seg0 : 1;
    cNearItem* segs = (cNearItem*)(multi ? D.items : D.items1);
    const int lane = threadIdx.x % kWave, li = lane % 16, g = lane / 16;
    const int wave = uni(static_cast<int>(threadIdx.x) / kWave);
    const int nrhs = b.nrhs;
    const bool jv = li < nrhs;   // B operand: column li of the vectors
    const int lc = min(li, nrhs - 1);
    const _Float16* whi = static_cast<const _Float16*>(D.wh) + 8 * lc;
    const int64_t lo_off = kMaxRhs * D.ldw;
    const _Float16* zero = static_cast<const _Float16*>(D.wh) + 2 * lo_off;   // 8 zero halves
    const _Float16* near = static_cast<const _Float16*>(D.near);
    float* part = static_cast<float*>(D.part) + static_cast<int64_t>(li) * (multi ? D.ldp : D.ldp1);
    // flip (every other product): the workgroups, and each workgroup's segments,
    // in reverse order, so that a product starts on the tiles the previous one
    // read last (still cached); each segment keeps its own order and slot, so
    // the sums do not change
    for (int k = 0; k < nseg; ++k) {
        cNearItem* Ip = segs + (b.flip ? seg0 + nseg - 1 - k : seg0 + k);
        const struct {
            int64_t part_off;
            int32_t ld, tile, ntiles, kbeg, kend;
        } I = {Ip->part_off, Ip->ld, Ip->tile, Ip->ntiles, Ip->kbeg, Ip->kend};
        const int ntiles = I.ntiles;
        const int rt = (I.ld + 15) / 16;   // row tiles of the leaf
        const int groups = max((rt + kMmaRowTiles - 1) / kMmaRowTiles, min(kBlock / kWave, rt));
        const int64_t ld8 = static_cast<int64_t>(I.ld) * 8;
        for (int grp = wave; grp < groups; grp += kBlock / kWave) {
            const int nrt = rt / groups + (grp < rt % groups ? 1 : 0);
            const int row0 = 16 * (grp * (rt / groups) + min(grp, rt % groups));
            // element offset (in halves) of this lane's row in each row tile, clamped to the group
            int roff[kMmaRowTiles];
#pragma unroll
            for (int t = 0; t < kMmaRowTiles; ++t) roff[t] = min(row0 + 16 * min(t, nrt - 1) + li, I.ld - 1) * 8;
            auto load = [&](const MmaPos& p, MmaStep& st) {
                const int kg = p.k0 + 8 * g;               // this lane's 8 columns
                const int kgc = min(kg, p.kc - 8);
                const _Float16* tp = near + p.tile_off + (kgc / 8) * ld8;
#pragma unroll
                for (int t = 0; t < kMmaRowTiles; ++t) st.a[t] = gload16(tp + roff[t]);
                // B lanes past nrhs or past the tile read the zero block
                const bool bv = jv && kg < p.kc;
                const _Float16* wq = whi + (static_cast<int64_t>(p.col_pos) + kgc) * nrhs;
                st.bh = gload16(bv ? wq : zero);
                st.bl = gload16(bv ? wq + lo_off : zero);
            };
            // the next position; false past the segment's last step
            auto advance = [&](MmaPos& p) {
                p.k0 += 32;
                if (p.k0 < p.kend) return true;
                p.k0 = 0;
                ++p.q;
                if (p.q >= ntiles) return false;
                mma_tile(D, I.tile + p.q, li, p);
                if (p.q == ntiles - 1) p.kend = I.kend;
                return true;
            };
            f4_t tot[kMmaRowTiles], acc[kMmaRowTiles];
#pragma unroll
            for (int t = 0; t < kMmaRowTiles; ++t) {
                tot[t] = f4_t{0.0f, 0.0f, 0.0f, 0.0f};
                acc[t] = f4_t{0.0f, 0.0f, 0.0f, 0.0f};
            }
            auto compute = [&](const MmaStep& st, const MmaPos& p) {
#pragma unroll
                for (int t = 0; t < kMmaRowTiles; ++t) {
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(st.a[t], st.bh, acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(st.a[t], st.bl, acc[t], 0, 0, 0);
                }
                if (p.k0 + 32 >= p.kend) {   // the tile's last step here: scale and add in tile order
                    const float sc = jv ? p.ts * p.wl : 0.0f;
#pragma unroll
                    for (int t = 0; t < kMmaRowTiles; ++t) {
                        tot[t] += f4_t{acc[t][0] * sc, acc[t][1] * sc, acc[t][2] * sc, acc[t][3] * sc};
                        acc[t] = f4_t{0.0f, 0.0f, 0.0f, 0.0f};
                    }
                }
            };
            // two step buffers in turn: the loads of one step are in flight while the
            // matrix instructions of the previous one run
            MmaStep s0, s1;
            MmaPos p0{};
            p0.q = 0;
            mma_tile(D, I.tile, li, p0);
            p0.k0 = I.kbeg;
            if (ntiles == 1) p0.kend = I.kend;
            load(p0, s0);
            // (past the last step the loads repeat the current position: unconditional
            // loads keep the loop free of branches around them, so each step waits only
            // for its own loads)
            for (;;) {
                MmaPos p1 = p0;
                const bool m1 = advance(p1);
                load(m1 ? p1 : p0, s1);
                compute(s0, p0);
                if (!m1) break;
                p0 = p1;
                const bool m0 = advance(p0);
                load(m0 ? p0 : p1, s0);
                compute(s1, p1);
                if (!m0) break;
            }
            // lane holds rows 4 g + q (q < 4) of column li of every row tile
            if (jv) {
                float* out = part + I.part_off;
#pragma unroll
                for (int t = 0; t < kMmaRowTiles; ++t) {
                    const int r = row0 + 16 * t + 4 * g;
                    if (t < nrt && r < I.ld) *reinterpret_cast<f4_t*>(out + r) = tot[t];
                }
            }
        }
    }
}

// packed half-precision copy of the near tiles (layout above); rows past the
// leaf and columns past |b| are zero
__global__ void k_pack_near(const double* src, const int64_t* off64, const int64_t* offp, const int32_t* ld,
                            const int32_t* na, const int32_t* nb, const float* scale, _Float16* dst) {
    const int64_t t = blockIdx.y;
    const int l = ld[t], rows = na[t], cols = nb[t];
    const int groups = (cols + 7) / 8;
    const double inv = scale ? 1.0 / static_cast<double>(scale[t]) : 1.0;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < static_cast<int64_t>(groups) * l;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int kg = static_cast<int>(e / l), r = static_cast<int>(e % l);
        h8_t v;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int k = kg * 8 + q;
            const double x = (r < rows && k < cols) ? src[off64[t] + static_cast<int64_t>(k) * l + r] * inv : 0.0;
            v[q] = static_cast<_Float16>(static_cast<float>(x));
        }
        *reinterpret_cast<h8_t*>(dst + offp[t] + e * 8) = v;
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
           P64.bytes() + P32.bytes() + C64.bytes() + C32.bytes() + rows.bytes() + near64.bytes() + nearT.bytes() + near_scale.bytes() +
           far64.bytes() + farT.bytes() + far_scale.bytes() + far_colmap.bytes() + d_items.bytes() +
           d_leaves.bytes() + q.bytes() + d.bytes() + c.bytes() + w_tree.bytes() + skw.bytes() + sku.bytes() +
           part.bytes() + plan_blob.bytes() + wh.bytes() + wsc.bytes() + d_items_mma[0].bytes() + d_items_mma[1].bytes() + d_tiles_mma.bytes() +
           d_leaves_mma[0].bytes() + d_leaves_mma[1].bytes() + d_wseg_mma[0].bytes() + d_wseg_mma[1].bytes() +
           d_otf_runs.bytes() + d_leaves_otf.bytes();
}

void Lane::init(LanePool* from) {
    if (side) return;
    pool = from;
    if (from) {
        std::lock_guard<std::mutex> g(from->mu);
        if (!from->free.empty()) {
            const LanePool::Entry e = from->free.back();
            from->free.pop_back();
            side = e.side;
            fork = e.fork;
            join = e.join;
            ready = e.ready;
            return;
        }
    }
    HDM_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
    HDM_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    HDM_HIP(hipEventCreateWithFlags(&join, hipEventDisableTiming));
    HDM_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
}

Lane::~Lane() {
    if (!side) return;
    (void)hipStreamSynchronize(side);
    if (pool) {
        std::lock_guard<std::mutex> g(pool->mu);
        pool->free.push_back(LanePool::Entry{side, fork, join, ready});
        return;
    }
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (ready) (void)hipEventDestroy(ready);
    (void)hipStreamDestroy(side);
}

LanePool::~LanePool() {
    for (const Entry& e : free) {
        (void)hipStreamSynchronize(e.side);
        (void)hipEventDestroy(e.fork);
        (void)hipEventDestroy(e.join);
        (void)hipEventDestroy(e.ready);
        (void)hipStreamDestroy(e.side);
    }
}

static int rows_per_lane(int dt) { return 16 / static_cast<int>(dtype_size(dt)); }

// workspaces of the product for up to nrhs right-hand sides (8-byte elements
// so that either vector type fits)
static void ensure_ws(Op& op, int nrhs) {
    if (op.ws_nrhs >= nrhs) return;
    op.w_tree.alloc(static_cast<size_t>(op.n) * nrhs * 8);
    op.skw.alloc(static_cast<size_t>(std::max<int64_t>(op.nskel, 1)) * nrhs * 8);
    op.sku.alloc(static_cast<size_t>(std::max<int64_t>(op.nskel, 1)) * nrhs * 8);
    // the several-column plans hold nrhs columns, the packed one-column plan one
    const int64_t pe = std::max<int64_t>(std::max(op.part_elems, op.part_elems_mma[1]) * nrhs, op.part_elems_mma[0]);
    op.part.alloc(static_cast<size_t>(std::max<int64_t>(pe, 1)) * 8);
    op.ws_nrhs = nrhs;
}

// (re)writes both descriptors of the operator into device memory
static void publish_descriptors(Op& op, hipStream_t s) {
    auto fill = [&](OpDev& D, bool f64) {
        D.n = op.n;
        D.depth = op.depth;
        D.L = op.L;
        D.perm = op.perm.get();
        D.c = op.c.get();
        D.start = op.d_start.get();
        D.rank = op.d_rank;
        D.ncand = op.d_ncand;
        D.skoff = op.d_skoff;
        D.poff = op.d_poff;
        D.P = f64 ? static_cast<const void*>(op.P64.get()) : static_cast<const void*>(op.P32.get());
        D.rows = op.d_row_tasks;
        for (int l = 0; l < kMaxLevels; ++l) {
            D.row_begin[l] = l < static_cast<int>(op.row_begin.size()) ? op.row_begin[l] : 0;
            D.row_count[l] = l < static_cast<int>(op.row_count.size()) ? op.row_count[l] : 0;
        }
        D.row_total = op.row_total;
        D.far_off = op.d_far_block_off;
        D.far_cols = op.d_far_cols;
        D.far_colbase = op.d_far_colbase;
        D.far_colmap = op.far_colmap.get();
        D.far = f64 ? static_cast<const void*>(op.far64.get()) : static_cast<const void*>(op.farT.get());
        D.fscale = (!f64 && op.far_scale.n) ? op.far_scale.get() : nullptr;
        D.items = D.items1 = op.d_items.get();
        D.nitems = D.nitems1 = static_cast<int64_t>(op.items.size());
        D.tiles = nullptr;
        D.wseg = D.wseg1 = nullptr;
        D.near = f64 ? static_cast<const void*>(op.near64.get()) : static_cast<const void*>(op.nearT.get());
        D.nscale = (!f64 && op.near_scale.n) ? op.near_scale.get() : nullptr;
        D.leaves = D.leaves1 = op.d_leaves.get();
        if (f64 && op.near_direct) {   // the on-the-fly near field's runs
            D.leaves = D.leaves1 = op.d_leaves_otf.get();
        }
        D.w = op.w_tree.get();
        D.skw = op.skw.get();
        D.sku = op.sku.get();
        D.part = op.part.get();
        D.ldsk = std::max<int64_t>(op.nskel, 1);
        D.ldp = D.ldp1 = std::max<int64_t>(f64 && op.near_direct ? op.part_elems_otf : op.part_elems, 1);
        D.wh = nullptr;
        D.wsc = nullptr;
        D.ldw = 0;
        D.comp = op.ncomp > 0 ? (f64 ? static_cast<const void*>(op.C64.get()) : static_cast<const void*>(op.C32.get()))
                              : nullptr;
        D.coff = op.d_coff;
        D.s2n_levels = op.s2n_levels ? 1 : 0;
        D.s2n_multi = op.s2n_by_levels(true, f64) ? 1 : 0;
        D.s2n_comp = op.s2n_comp && !f64 && op.ncomp > 0 ? 1 : 0;
        D.s2n_comp1 = op.ncomp > 0 && !op.s2n_levels && op.depth >= 2 &&
                              op.comp1_stage <= kChainStageBytes / static_cast<int64_t>(f64 ? sizeof(double) : sizeof(float))
                          ? 1
                          : 0;
        if (!f64 && op.packed) {   // matrix-core plan of the packed half-precision tiles
            D.items = op.d_items_mma[1].get();
            D.nitems = static_cast<int64_t>(op.items_mma[1].size());
            D.leaves = op.d_leaves_mma[1].get();
            D.ldp = std::max<int64_t>(op.part_elems_mma[1], 1);
            D.items1 = op.d_items_mma[0].get();
            D.nitems1 = static_cast<int64_t>(op.items_mma[0].size());
            D.leaves1 = op.d_leaves_mma[0].get();
            D.ldp1 = std::max<int64_t>(op.part_elems_mma[0], 1);
            D.tiles = op.d_tiles_mma.get();
            D.wseg = op.wseg_one[1] ? nullptr : op.d_wseg_mma[1].get();
            D.wseg1 = op.wseg_one[0] ? nullptr : op.d_wseg_mma[0].get();
            D.wh = op.wh.get();
            D.wsc = op.wsc.get();
            D.ldw = op.ldw;
        }
    };
    fill(op.host64, true);
    fill(op.hostT, false);
    if (!op.dev64.n) op.dev64.alloc(1);
    if (!op.devT.n) op.devT.alloc(1);
    // the uploads read op.host64 / op.hostT (or a staged copy of them), which
    // outlive the copies: no wait here
    op.dev64.upload(&op.host64, 1, s);
    op.devT.upload(&op.hostT, 1, s);
}

static void check_near_plan(const Op& op);

// Plan of the packed half-precision near field (k_l2l_mma): per near pair an
// ld_a x kc_b packed tile, the tiles of one leaf consecutive in memory.  The
// work is the sequence of tile steps (32 columns of one tile, all rows of its
// leaf), leaf after leaf.
// * Several columns: each workgroup takes a contiguous share of it, the shares
//   equal to within one step, cut into segments at leaf boundaries (one
//   partial-sum slot of ld_a rows per segment: few partial sums to write and
//   add).  The workgroup count is 7/8 of what the device holds at once, fewer
//   where a share would fall below kMmaMinSteps steps: the upward and far passes
//   run on a side stream beside this launch and need the rest (N = 100000, 16
//   columns: all slots 309 us for the near field but 534 us for the product, 7/8
//   329 and 509 us, 6/8 344 and 489 us; runs of whole tiles, one wave each, had
//   taken 349 and 575 us).
// * One column: one workgroup per tile (many short items, which the hardware
//   hands to whichever compute unit frees first; equal shares measured 275
//   against 264 us).
// Vectors are staged with every leaf padded to a multiple of 8 points.
constexpr int kMmaMinSteps = 16;
constexpr int kMmaShare8 = 7;        // eighths of the device's workgroups given to several columns
constexpr bool kMmaTileWgs1 = true;  // one column: one workgroup per tile instead of equal shares

static void build_mma_plan(Op& op, hipStream_t s) {
    const int64_t L = op.L;
    op.packed = true;
    std::vector<int64_t> wpad(L);
    op.ldw = 0;
    for (int64_t b = 0; b < L; ++b) {
        wpad[b] = op.ldw;
        op.ldw += (op.size[L + b] + 7) / 8 * 8;
    }
    packed_near_offsets(op);
    // workgroups the device holds at once, per kernel ([0] one column, [1] several)
    int dev = 0, ncu = 0;
    HDM_HIP(hipGetDevice(&dev));
    HDM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    int occ[2] = {0, 0};
    HDM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[0], k_l2l_mma<true>, kBlock, 0));
    HDM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[1], k_l2l_mma<false>, kBlock, 0));
    const int64_t wgs[2] = {static_cast<int64_t>(std::max(occ[0], 1)) * std::max(ncu, 1),
                            static_cast<int64_t>(std::max(occ[1], 1)) * std::max(ncu, 1)};
    op.tiles_mma.clear();
    int64_t off = 0;
    for (int64_t a = 0; a < L; ++a) {
        const int32_t ld = op.near_ld[a];
        for (int32_t t = op.near_off[a]; t < op.near_off[a + 1]; ++t) {
            const int32_t b = op.near_idx[t];
            const int64_t nb = op.size[L + b];
            NearItem T{};
            T.tile_off = off;
            T.ld = ld;
            T.ncols = static_cast<int32_t>(nb);
            T.col_pos = static_cast<int32_t>(wpad[b]);
            T.tile = t;
            T.leaf_b = b;
            T.ntiles = 1;
            op.tiles_mma.push_back(T);
            off += static_cast<int64_t>(ld) * ((nb + 7) / 8 * 8);
        }
    }
    op.near_elems_mma = off;
    // steps per tile and per leaf
    std::vector<int64_t> leaf_steps(L, 0);
    for (int64_t a = 0; a < L; ++a)
        for (int32_t t = op.near_off[a]; t < op.near_off[a + 1]; ++t)
            leaf_steps[a] += ceil_div((op.tiles_mma[t].ncols + 7) / 8 * 8, 32);
    int64_t total = 0;
    for (int64_t a = 0; a < L; ++a) total += leaf_steps[a];
    for (int k = 0; k < 2; ++k) {
        std::vector<NearItem>& items = op.items_mma[k];
        std::vector<LeafPlan>& leaves = op.leaves_mma[k];
        std::vector<int32_t>& wseg = op.wseg_mma[k];
        items.clear();
        leaves.clear();
        wseg.clear();
        op.red_groups_mma[k] = 0;
        const bool per_tile = k == 0 && kMmaTileWgs1;
        const int64_t cap = k == 0 ? wgs[0] : std::max<int64_t>(1, wgs[1] * kMmaShare8 / 8);
        const int64_t P = std::max<int64_t>(1, std::min<int64_t>(cap, ceil_div(total, kMmaMinSteps)));
        const int64_t Q = std::max<int64_t>(1, ceil_div(total, P));   // steps per workgroup
        // every leaf's segments, in order: cut at each multiple of Q of the
        // global step position
        int64_t part = 0, pos = 0;
        for (int64_t a = 0; a < L; ++a) {
            const int64_t ha = L + a;
            const int32_t ld = op.near_ld[a];
            LeafPlan lp{};
            lp.part_off = part;
            lp.ld = ld;
            lp.start = static_cast<int32_t>(op.start[ha]);
            lp.rows = static_cast<int32_t>(op.size[ha]);
            lp.heap = static_cast<int32_t>(ha);
            lp.wpad = wpad[a];
            int32_t nseg = 0;
            // one workgroup per tile
            for (int32_t t = op.near_off[a]; per_tile && t < op.near_off[a + 1]; ++t) {
                wseg.push_back(static_cast<int32_t>(items.size()));
                NearItem I = op.tiles_mma[t];
                I.part_off = part + static_cast<int64_t>(nseg) * ld;
                I.row0 = 0;
                I.nrows = ld;
                I.kbeg = 0;
                I.kend = (I.ncols + 7) / 8 * 8;
                items.push_back(I);
                ++nseg;
            }
            // leaf-local step range [lo, hi) of each segment
            for (int64_t lo = 0; !per_tile && lo < leaf_steps[a];) {
                const int64_t gpos = pos + lo;
                if (gpos % Q == 0) wseg.push_back(static_cast<int32_t>(items.size()));
                const int64_t hi = std::min(leaf_steps[a], lo + (Q - gpos % Q));
                // tiles holding steps lo and hi - 1
                NearItem I{};
                int64_t acc = 0;
                int32_t t0 = -1, t1 = -1;
                for (int32_t t = op.near_off[a]; t < op.near_off[a + 1]; ++t) {
                    const int64_t st = ceil_div((op.tiles_mma[t].ncols + 7) / 8 * 8, 32);
                    if (t0 < 0 && lo < acc + st) {
                        t0 = t;
                        I.kbeg = static_cast<int32_t>(32 * (lo - acc));
                    }
                    if (hi <= acc + st) {
                        t1 = t;
                        const int32_t kc = (op.tiles_mma[t].ncols + 7) / 8 * 8;
                        I.kend = static_cast<int32_t>(std::min<int64_t>(kc, 32 * (hi - acc)));
                        break;
                    }
                    acc += st;
                }
                const NearItem& T0 = op.tiles_mma[t0];
                I.tile_off = T0.tile_off;
                I.part_off = part + static_cast<int64_t>(nseg) * ld;
                I.ld = ld;
                I.row0 = 0;
                I.nrows = ld;
                I.ncols = T0.ncols;
                I.col_pos = T0.col_pos;
                I.tile = t0;
                I.leaf_b = T0.leaf_b;
                I.ntiles = t1 - t0 + 1;
                items.push_back(I);
                ++nseg;
                lo = hi;
            }
            pos += leaf_steps[a];
            lp.nitems = nseg;
            lp.ngroups = std::max(ceil_div((ld + 15) / 16, kMmaRowTiles), std::min<int>(kBlock / kWave, (ld + 15) / 16));
            lp.gstep = nseg > kReduceAbove ? kReduceGroup : 1;
            if (lp.gstep > 1) op.red_groups_mma[k] = std::max(op.red_groups_mma[k], ceil_div(nseg, kReduceGroup));
            part += static_cast<int64_t>(nseg) * ld;
            leaves.push_back(lp);
        }
        wseg.push_back(static_cast<int32_t>(items.size()));
        op.wseg_one[k] = wseg.size() == items.size() + 1;
        op.part_elems_mma[k] = part;
    }
    op.ldw = std::max<int64_t>(op.ldw, 0);
    check_near_plan(op);
    for (int k = 0; k < 2; ++k) {
        op.d_items_mma[k] = to_device(op.items_mma[k], s);
        op.d_leaves_mma[k] = to_device(op.leaves_mma[k], s);
        op.d_wseg_mma[k] = to_device(op.wseg_mma[k], s);
    }
    op.d_tiles_mma = to_device(op.tiles_mma, s);
    op.wh.alloc((static_cast<size_t>(std::max<int64_t>(op.ldw, 1)) * 2 * kMaxRhs + 8) * sizeof(_Float16));
    op.wsc.alloc(static_cast<size_t>(L) * kMaxRhs);
}


// Host-side bounds checks of every launch descriptor against the extent of the
// buffer it indexes, before the descriptors are uploaded: a plan that would
// read or write outside a buffer is an HDM_EINTERNAL error, not a launch.
static void check_near_plan(const Op& op) {
    const int64_t L = op.L;
    const int64_t pairs = static_cast<int64_t>(op.near_idx.size());
    auto bad = [](const char* what) { fail(HDM_EINTERNAL, std::string("near-field plan: ") + what); };
    for (const NearItem& I : op.items) {
        if (I.tile < 0 || I.tile >= pairs) bad("tile index");
        if (I.ncols < 1 || I.ld < 1 || I.row0 < 0 || I.row0 >= I.ld) bad("item shape");
        if (I.tile_off < 0 || I.tile_off + static_cast<int64_t>(I.ncols) * I.ld > op.near_elems) bad("tile extent");
        if (I.part_off < 0 || I.part_off + I.ld > op.part_elems) bad("partial-sum extent");
        if (I.col_pos < 0 || I.col_pos + I.ncols > op.n) bad("vector extent");
    }
    if (static_cast<int64_t>(op.leaves.size()) != L) bad("leaf count");
    for (const LeafPlan& lp : op.leaves) {
        if (lp.heap < L || lp.heap >= 2 * L) bad("leaf heap id");
        if (lp.rows < 1 || lp.rows > lp.ld || lp.start < 0 || lp.start + lp.rows > op.n) bad("leaf rows");
        if (lp.part_off < 0 || lp.part_off + static_cast<int64_t>(lp.nitems) * lp.ld > op.part_elems) bad("leaf partials");
    }
    // on-the-fly runs: consecutive items of one leaf and row group, slots inside the leaf's
    if (static_cast<int64_t>(op.leaves_otf.size()) != L) bad("on-the-fly leaf count");
    for (const OtfRun& R : op.otf_runs) {
        if (R.item < 0 || R.count < 1 || static_cast<int64_t>(R.item) + R.count > static_cast<int64_t>(op.items.size()))
            bad("on-the-fly run items");
        const NearItem& I0 = op.items[R.item];
        const NearItem& I1 = op.items[R.item + R.count - 1];
        if (I0.row0 != I1.row0 || I0.ld != I1.ld || I0.row_pos != I1.row_pos) bad("on-the-fly run across leaves");
        if (R.part_off < 0 || R.part_off + I0.ld > op.part_elems_otf) bad("on-the-fly partial-sum extent");
    }
    for (const LeafPlan& lp : op.leaves_otf)
        if (lp.part_off < 0 || lp.part_off + static_cast<int64_t>(lp.nitems) * lp.ld > op.part_elems_otf)
            bad("on-the-fly leaf partials");
    if (op.packed) {
        if (static_cast<int64_t>(op.tiles_mma.size()) != pairs) bad("packed tile records");
        for (int64_t t = 0; t < pairs; ++t) {
            const NearItem& T = op.tiles_mma[t];
            if (T.tile != t || T.leaf_b < 0 || T.leaf_b >= L || T.ncols < 1) bad("packed tile index");
            const int64_t kc = (static_cast<int64_t>(T.ncols) + 7) / 8 * 8;
            if (T.tile_off < 0 || T.tile_off + kc * T.ld > op.near_elems_mma) bad("packed tile extent");
            if (T.col_pos < 0 || T.col_pos + kc > op.ldw) bad("staged vector extent");
        }
        for (int k = 0; k < 2; ++k) {
            const std::vector<NearItem>& segs = op.items_mma[k];
            const std::vector<LeafPlan>& leaves = op.leaves_mma[k];
            if (static_cast<int64_t>(leaves.size()) != L) bad("packed leaf count");
            // segments: leaf after leaf, each leaf's in slot order, inside the leaf's tiles
            size_t si = 0;
            for (int64_t a = 0; a < L; ++a) {
                const LeafPlan& lp = leaves[a];
                if (lp.nitems < 1 || lp.ld != op.near_ld[a]) bad("packed leaf plan");
                if (lp.part_off < 0 || lp.part_off + static_cast<int64_t>(lp.nitems) * lp.ld > op.part_elems_mma[k])
                    bad("packed leaf partials");
                if (lp.wpad < 0 || lp.wpad + (lp.rows + 7) / 8 * 8 > op.ldw) bad("packed leaf vector");
                for (int32_t q = 0; q < lp.nitems; ++q, ++si) {
                    if (si >= segs.size()) bad("packed segment count");
                    const NearItem& I = segs[si];
                    if (I.tile < op.near_off[a] || I.ntiles < 1 || I.tile + I.ntiles > op.near_off[a + 1])
                        bad("packed segment tiles");
                    if (I.tile_off != op.tiles_mma[I.tile].tile_off || I.ld != lp.ld) bad("packed segment start");
                    const int32_t kc0 = (op.tiles_mma[I.tile].ncols + 7) / 8 * 8;
                    const int32_t kc1 = (op.tiles_mma[I.tile + I.ntiles - 1].ncols + 7) / 8 * 8;
                    if (I.kbeg < 0 || I.kbeg % 32 != 0 || I.kbeg >= kc0) bad("packed segment first column");
                    if (I.kend < 1 || I.kend > kc1 || (I.kend != kc1 && I.kend % 32 != 0)) bad("packed segment end column");
                    if (I.ntiles == 1 && I.kbeg >= I.kend) bad("packed segment columns");
                    if (I.part_off != lp.part_off + static_cast<int64_t>(q) * lp.ld) bad("packed segment slot");
                }
            }
            if (si != segs.size()) bad("packed segment count");
            const std::vector<int32_t>& wseg = op.wseg_mma[k];
            if (wseg.size() < 2 || wseg.front() != 0 || wseg.back() != static_cast<int32_t>(segs.size()))
                bad("packed workgroup segments");
            for (size_t w = 0; w + 1 < wseg.size(); ++w)
                if (wseg[w + 1] <= wseg[w]) bad("packed workgroup segments");
        }
    }
}

static void check_eval_plan(const Op& op, const std::vector<RowTask>& tasks) {
    const int64_t NN = op.nnodes, L = op.L;
    auto bad = [](const char* what) { fail(HDM_EINTERNAL, std::string("evaluation plan: ") + what); };
    int64_t far_cols_total = 0;
    for (int64_t h = 2; h < NN; ++h) {
        const int64_t rk = op.rank[h], nc = op.ncand[h];
        if (rk < 0 || rk > nc || (h >= L && rk > kMaxRank)) bad("rank");
        if (rk > kMaxRank && !op.s2n_levels) bad("inner rank above the combine's walk without the level-wise pass");
        if (op.skoff[h] < 0 || op.skoff[h] + rk > op.nskel) bad("skeleton extent");
        if (op.poff[h] < 0 || op.poff[h] + rk * nc > op.np) bad("interpolation extent");
        if (h >= L && nc != op.size[h]) bad("leaf candidates are not its points");
        if (h < L && nc != op.rank[2 * h] + op.rank[2 * h + 1]) bad("inner candidates are not the children's skeletons");
        if (op.far_block_off[h] < 0 || op.far_block_off[h] + rk * op.far_cols[h] > std::max<int64_t>(op.far_elems, 0))
            bad("far block extent");
        if (op.far_colbase[h] < 0 || op.far_colbase[h] + op.far_cols[h] > static_cast<int64_t>(op.far_colmap.n))
            bad("far column map extent");
        far_cols_total += op.far_cols[h];
        if (op.ncomp > 0 && h < L) {
            const int lvl = 63 - __builtin_clzll(static_cast<unsigned long long>(h));
            const int sh = op.depth - lvl;
            const int64_t fl = h << sh, ll = ((h + 1) << sh) - 1;
            const int64_t nlk = op.skoff[ll] + op.rank[ll] - op.skoff[fl];
            if (nlk < 0 || op.coff[h] < 0 || op.coff[h] + rk * nlk > op.ncomp) bad("composite extent");
        }
    }
    if (far_cols_total > static_cast<int64_t>(op.far_colmap.n)) bad("far column map size");
    for (const RowTask& t : tasks)
        if (t.h < 2 || t.h >= NN || t.i < 0 || t.i >= op.rank[t.h]) bad("row task");
}

// The near-field part of the evaluation plan (work items and per-leaf plans):
// it needs only the tree and the near lists, so the operator builds it while
// the skeletonisation runs.
void build_near_plan(Op& op, hipStream_t s) {
    const int64_t L = op.L;
    // near-field items: per leaf, per row group, per near tile, per column chunk
    const int rg = kWave * rows_per_lane(op.prm.near_prec);
    op.near_rows_per_group = rg;
    op.items.clear();
    op.leaves.clear();
    int64_t part = 0;
    op.red_groups = 0;
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
        lp.gstep = per_group > kReduceAbove ? kReduceGroup : 1;
        if (lp.gstep > 1) op.red_groups = std::max(op.red_groups, ceil_div(per_group, kReduceGroup));
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
                    I.row_pos = lp.start;
                    I.row_n = lp.rows;
                    op.items.push_back(I);
                }
            }
        }
        part += static_cast<int64_t>(per_group) * ld;
        op.leaves.push_back(lp);
    }
    op.part_elems = part;
    // runs of the on-the-fly float64 near field: kOtfRunItems consecutive items of
    // one leaf and row group (512 columns), one partial-sum slot per run
    op.otf_runs.clear();
    op.leaves_otf.clear();
    int64_t opart = 0, it = 0;
    for (int64_t a = 0; a < L; ++a) {
        LeafPlan lp = op.leaves[a];
        const int per_group = lp.nitems;
        const int nrun = ceil_div(per_group, kOtfRunItems);
        lp.part_off = opart;
        lp.nitems = nrun;
        lp.gstep = 1;
        for (int g = 0; g < lp.ngroups; ++g)
            for (int r = 0; r < nrun; ++r) {
                OtfRun R{};
                R.item = static_cast<int32_t>(it + static_cast<int64_t>(g) * per_group + r * kOtfRunItems);
                R.count = std::min(kOtfRunItems, per_group - r * kOtfRunItems);
                R.part_off = opart + static_cast<int64_t>(r) * lp.ld;
                op.otf_runs.push_back(R);
            }
        it += static_cast<int64_t>(lp.ngroups) * per_group;
        opart += static_cast<int64_t>(nrun) * lp.ld;
        op.leaves_otf.push_back(lp);
    }
    op.part_elems_otf = opart;
    if (op.prm.near_prec == HDM_F16) build_mma_plan(op, s);
    check_near_plan(op);
    op.d_items = to_device(op.items, s);
    op.d_leaves = to_device(op.leaves, s);
    op.d_otf_runs = to_device(op.otf_runs, s);
    op.d_leaves_otf = to_device(op.leaves_otf, s);
}

// the rest of the plan, once the skeletons are known
void build_eval_plan(Op& op, hipStream_t s) {
    // one row task per skeleton row, grouped by level from the leaves up; the
    // same list, taken whole, gives the far-field (S2S) rows
    std::vector<RowTask> tasks;
    op.row_begin.assign(kMaxLevels, 0);
    op.row_count.assign(kMaxLevels, 0);
    for (int lvl = op.depth; lvl >= 1; --lvl) {
        op.row_begin[lvl] = static_cast<int64_t>(tasks.size());
        for (int64_t h = int64_t(1) << lvl; h < (int64_t(1) << (lvl + 1)); ++h)
            for (int32_t i = 0; i < op.rank[h]; ++i) tasks.push_back(RowTask{static_cast<int32_t>(h), i});
        op.row_count[lvl] = static_cast<int64_t>(tasks.size()) - op.row_begin[lvl];
    }
    op.row_total = static_cast<int64_t>(tasks.size());
    HDM_CHECK(static_cast<int64_t>(op.rank.size()) == op.nnodes && static_cast<int64_t>(op.far_cols.size()) == op.nnodes,
              HDM_EINTERNAL, "per-node arrays");
    // composites of the nested bases, where they are not much larger than the
    // inner nodes' P (one launch then forms every level above the leaves)
    op.coff.assign(static_cast<size_t>(2 * op.L), 0);
    op.ncomp = 0;
    {
        int64_t comp = 0, inner_p = 0;
        bool nested = true;   // an inner node's candidates are its children's skeletons
        for (int64_t h = 2; h < op.L; ++h)
            nested = nested && op.ncand[h] == op.rank[2 * h] + op.rank[2 * h + 1];
        for (int lvl = op.depth - 1; lvl >= 1; --lvl) {
            const int sh = op.depth - lvl;
            for (int64_t h = int64_t(1) << lvl; h < (int64_t(1) << (lvl + 1)); ++h) {
                const int64_t fl = h << sh, ll = ((h + 1) << sh) - 1;
                const int64_t nlk = op.skoff[ll] + op.rank[ll] - op.skoff[fl];
                op.coff[h] = comp;
                comp += op.rank[h] * nlk;
                inner_p += static_cast<int64_t>(op.rank[h]) * op.ncand[h];
            }
        }
        // Used where the extra entries cost less to stream than the per-level
        // launches they save: at most 16M more than the inner nodes' P (a few MB at
        // the S-curve sizes; the MNIST-shaped operator, every rank at the cap, would
        // read 117M entries per product instead of P's 33M and keeps the per-level
        // launches)
        if (nested && op.depth >= 2 && comp <= inner_p + (int64_t(16) << 20)) op.ncomp = comp;
        // The combine walks each leaf's path down from the root, re-reading the
        // ancestors' P slices once per leaf; where that re-reads more than 16M
        // entries beyond the slices themselves (every rank at the cap of the
        // MNIST-shaped operator: 117M against 33M) the downward pass runs once per
        // product instead, one launch per level, with the same arithmetic.
        int64_t chain = 0, slices = 0;
        for (int64_t h = 2; h < 2 * op.L; ++h) {
            const int64_t e = static_cast<int64_t>(op.rank[h >> 1]) * op.rank[h];
            slices += e;
            int64_t under = 1;   // leaves below h
            for (int64_t g = h; g < op.L; g <<= 1) under <<= 1;
            chain += e * under;
        }
        op.s2n_levels = nested && op.depth >= 2 && chain > slices + (int64_t(16) << 20);
        // ranks above the combine's 512 potentials are only ever held by inner
        // nodes (leaves: at most 512 by the parameter rules): pass them level-wise
        int max_inner = 0;
        for (int64_t h = 2; h < op.L; ++h) max_inner = std::max(max_inner, static_cast<int>(op.rank[h]));
        if (max_inner > kMaxRank) op.s2n_levels = true;
        // several right-hand sides: always level by level (one launch per level
        // on the side stream, beside the near field, instead of a chain of
        // dependent steps per leaf in the combine)
        op.s2n_multi = op.s2n_levels || (nested && op.depth >= 2);
        // through the composites instead, where every leaf's ancestors' potentials
        // (16 columns) fit the combine's staging and the per-level sums its second
        // potential buffer
        op.s2n_comp = op.ncomp > 0 && !op.s2n_levels && op.depth >= 2;
        for (int64_t h = op.L; op.s2n_comp && h < 2 * op.L; ++h) {
            int64_t anc = 0;
            for (int64_t g = h >> 1; g >= 2; g >>= 1) anc += op.rank[g];
            if (anc * kMaxRhs > kStageM<float> || int64_t(op.depth - 1) * op.rank[h] * kMaxRhs > kMaxRhs * kMaxRank)
                op.s2n_comp = false;
        }
        op.lvl_max_nc.assign(kMaxLevels + 1, 0);
        op.lvl_max_rank.assign(kMaxLevels + 1, 0);
        for (int64_t h = 2; h < 2 * op.L; ++h) {
            int lvl = 0;
            while ((int64_t(2) << lvl) <= h) ++lvl;
            op.lvl_max_nc[lvl] = std::max(op.lvl_max_nc[lvl], static_cast<int32_t>(op.ncand[h]));
            op.lvl_max_rank[lvl] = std::max(op.lvl_max_rank[lvl], static_cast<int32_t>(op.rank[h]));
        }
        op.max_leaf_rank = 0;
        for (int64_t h = op.L; h < 2 * op.L; ++h) op.max_leaf_rank = std::max(op.max_leaf_rank, static_cast<int>(op.rank[h]));
        op.comp1_stage = 0;
        for (int64_t h = op.L; h < 2 * op.L; ++h) {
            int64_t anc = 0;
            for (int64_t g = h >> 1; g >= 2; g >>= 1) anc += op.rank[g];
            op.comp1_stage = std::max(op.comp1_stage, anc * (1 + op.rank[h]) + int64_t(op.depth - 1) * op.rank[h]);
        }
    }
    check_eval_plan(op, tasks);
    // the skeleton-dependent arrays in one allocation and one copy
    std::vector<char> blob;
    auto add = [&](const void* src, size_t bytes) {
        const size_t off = (blob.size() + 255) / 256 * 256;
        blob.resize(off + bytes);
        if (bytes) std::memcpy(blob.data() + off, src, bytes);
        return off;
    };
    const size_t o_rank = add(op.rank.data(), op.rank.size() * sizeof(int32_t));
    const size_t o_ncand = add(op.ncand.data(), op.ncand.size() * sizeof(int32_t));
    const size_t o_skoff = add(op.skoff.data(), op.skoff.size() * sizeof(int64_t));
    const size_t o_poff = add(op.poff.data(), op.poff.size() * sizeof(int64_t));
    const size_t o_fbo = add(op.far_block_off.data(), op.far_block_off.size() * sizeof(int64_t));
    const size_t o_fc = add(op.far_cols.data(), op.far_cols.size() * sizeof(int32_t));
    const size_t o_fcb = add(op.far_colbase.data(), op.far_colbase.size() * sizeof(int64_t));
    const size_t o_tasks = add(tasks.data(), tasks.size() * sizeof(RowTask));
    const size_t o_coff = add(op.coff.data(), op.coff.size() * sizeof(int64_t));
    blob.resize(blob.size() + 256);   // every piece, empty ones included, points inside the allocation
    op.plan_blob.alloc(blob.size());
    op.plan_blob.upload(blob.data(), blob.size(), s);
    char* base = op.plan_blob.get();
    op.d_rank = reinterpret_cast<const int32_t*>(base + o_rank);
    op.d_ncand = reinterpret_cast<const int32_t*>(base + o_ncand);
    op.d_skoff = reinterpret_cast<const int64_t*>(base + o_skoff);
    op.d_poff = reinterpret_cast<const int64_t*>(base + o_poff);
    op.d_far_block_off = reinterpret_cast<const int64_t*>(base + o_fbo);
    op.d_far_cols = reinterpret_cast<const int32_t*>(base + o_fc);
    op.d_far_colbase = reinterpret_cast<const int64_t*>(base + o_fcb);
    op.d_row_tasks = reinterpret_cast<const RowTask*>(base + o_tasks);
    op.d_coff = reinterpret_cast<const int64_t*>(base + o_coff);
    op.C64.release();
    op.C32.release();
    if (op.ncomp > 0) {
        op.C64.alloc(static_cast<size_t>(op.ncomp));
        op.C32.alloc(static_cast<size_t>(op.ncomp));
        const int wpb = kBlock / kWave;
        for (int lvl = op.depth - 1; lvl >= 1; --lvl) {
            const int64_t nr = op.row_count[lvl];
            if (nr == 0) continue;
            const int sh = op.depth - lvl;
            int64_t maxnlk = 1;
            for (int64_t h = int64_t(1) << lvl; h < (int64_t(1) << (lvl + 1)); ++h)
                maxnlk = std::max(maxnlk, op.skoff[((h + 1) << sh) - 1] + op.rank[((h + 1) << sh) - 1] - op.skoff[h << sh]);
            hipLaunchKernelGGL(k_compose, dim3(ceil_div(nr, wpb), ceil_div(maxnlk, kWave)), dim3(kBlock), 0, s,
                               op.P64.get(), op.d_poff,
                               op.d_rank, op.d_ncand, op.d_skoff, op.d_coff, op.d_row_tasks, op.row_begin[lvl], nr,
                               op.depth, lvl, op.C64.get(), op.C32.get());
        }
        check_launch("composites");
    }
    op.lane.init(op.ctx ? &op.ctx->lanes : nullptr);
    ensure_ws(op, 1);
    publish_descriptors(op, s);
}

// shared memory of k_n2s_node_m at tree level lvl
static size_t n2s_node_bytes(const Op& op, int lvl, size_t vsize) {
    return static_cast<size_t>(kMaxRhs) * static_cast<size_t>(op.lvl_max_nc[lvl]) * vsize;
}

template <typename V, typename TN, typename TF, typename TP>
static void apply_t(const ApplyReq* reqs, int nops, bool f64, int normalised, int nrhs, hipStream_t s, Lane& lane,
                    Ctx* cx) {
    // half-precision near tiles are packed for the matrix cores (float64 products use the plain layout)
    constexpr bool mma = std::is_same<TN, f16_t>::value;
    const bool multi = nrhs > 1;
    Batch b{};
    b.nops = nops;
    b.nrhs = nrhs;
    for (int o = 0; o < nops; ++o) {
        b.op[o] = reqs[o].desc ? reqs[o].desc : (f64 ? reqs[o].op->dev64.get() : reqs[o].op->devT.get());
        b.x[o] = reqs[o].x;
        b.y[o] = reqs[o].y;
    }
    auto prefix = [&](auto count) {
        b.pre[0] = 0;
        for (int o = 0; o < nops; ++o) b.pre[o + 1] = b.pre[o] + count(*reqs[o].op, o);
        return b.pre[nops];
    };
    const int wpb = kBlock / kWave;
    {   // gather + scale into tree order
        for (int o = 0; o < nops; ++o) b.arg[o] = normalised;
        KernelEvents ev(cx, HDM_PHASE_PREP);
        if (mma) {
            const int64_t tot = prefix([](const Op& op, int) { return static_cast<int64_t>(op.L); });
            hipExtLaunchKernelGGL(k_prep_mma, dim3(tot), dim3(kCombBlock), 0, s, ev.start, ev.stop, 0, b);
        } else {
            const int64_t tot = prefix([](const Op& op, int) { return op.n; });
            hipExtLaunchKernelGGL((k_prep<V>), dim3(ceil_div(tot, kBlock)), dim3(kBlock), 0, s, ev.start, ev.stop, 0,
                                  b);
        }
    }
    bool tree = false;
    int maxdepth = 0;
    for (int o = 0; o < nops; ++o) {
        tree = tree || reqs[o].op->nskel > 0;
        maxdepth = std::max(maxdepth, reqs[o].op->depth);
    }
    // Several right-hand sides: the upward pass, the far field and the level-wise
    // downward pass run on the side stream while the near field streams on s
    // (100k, 16 columns: 545 against 586 us per product in sequence).  One
    // right-hand side: all on s, since the fork and join cost more than the
    // overlap saves (4.8 against 5.2 ms per 25-step solve at N = 32768).
    const bool overlap = tree && multi;
    hipStream_t ts = overlap ? lane.side : s;
    // The near field streams every tile once per product, more bytes than the
    // device's last-level cache holds; taking the items in reverse order on
    // every other product starts each pass on the tiles the previous one read
    // last, which are still cached.  Each item writes its own partial sums, so
    // the order does not change the result.
    // One operator and one right-hand side: the leaf level of the upward pass
    // rides in the near field's launch (its first workgroups, one per leaf), beside
    // the tile streaming; the levels above follow in one launch through the
    // composites (or one launch per level without them), then the far field.
    // float64 products of an operator without float64 near tiles (its degrees):
    // the near field evaluates the kernel on the fly
    const bool otf = f64 && reqs[0].op->near_direct;
    HDM_CHECK(!otf || (nops == 1 && !multi), HDM_EINTERNAL, "on-the-fly near field takes one operator and one column");
    const bool fuse_up = tree && !multi && nops == 1 && !otf;
    b.up = fuse_up ? static_cast<int>(reqs[0].op->L) : 0;
    auto near_field = [&] {
        // matrix cores: one workgroup per share of the plan; plain tiles: one wave per item
        const int64_t tot = prefix([multi](const Op& op, int) {
            return static_cast<int64_t>(mma ? op.wseg_mma[multi].size() - 1 : op.items.size());
        });
        b.flip = static_cast<int>(reqs[0].op->near_calls++ & 1u);
        const int64_t grid = (mma ? tot : ceil_div(tot, wpb)) + b.up;
        if (otf) {
            Op& o0 = *reqs[0].op;
            if (o0.near_ones_next && o0.part_ones.n) {   // K~ 1: its near field is already computed
                HDM_HIP(hipMemcpyAsync(o0.part.get(), o0.part_ones.get(), o0.part_ones.bytes(), hipMemcpyDeviceToDevice, s));
                o0.near_ones_next = false;
            } else {
                near_field_otf(o0, reinterpret_cast<const double*>(o0.w_tree.get()), reinterpret_cast<double*>(o0.part.get()),
                               s);
            }
            return;
        }
        KernelEvents ev(cx, HDM_PHASE_L2L);
        if (mma && fuse_up)
            hipExtLaunchKernelGGL(k_l2l_mma<true>, dim3(grid), dim3(kBlock), 0, s, ev.start, ev.stop, 0, b);
        else if (mma)
            hipExtLaunchKernelGGL(k_l2l_mma<false>, dim3(grid), dim3(kBlock), 0, s, ev.start, ev.stop, 0, b);
        else if (fuse_up)
            hipExtLaunchKernelGGL((k_l2l<V, TN, true, false>), dim3(grid), dim3(kBlock), 0, s, ev.start, ev.stop, 0, b);
        else if (multi)
            hipExtLaunchKernelGGL((k_l2l<V, TN, false, true>), dim3(grid), dim3(kBlock), 0, s, ev.start, ev.stop, 0, b);
        else
            hipExtLaunchKernelGGL((k_l2l<V, TN, false, false>), dim3(grid), dim3(kBlock), 0, s, ev.start, ev.stop, 0, b);
    };
    // several columns: busy leaves' partial sums pre-added in groups, after the near field
    auto part_reduce = [&] {
        int maxg = 0;
        for (int o = 0; o < nops; ++o)
            maxg = std::max(maxg, mma ? reqs[o].op->red_groups_mma[1] : reqs[o].op->red_groups);
        if (!multi || maxg == 0) return;
        const int64_t tot = prefix([](const Op& op, int) { return static_cast<int64_t>(op.L); });
        hipLaunchKernelGGL((k_part_reduce<V>), dim3(tot, maxg, nrhs), dim3(kBlock), 0, s, b);
    };
    if (overlap) {
        // fork after the staging; the near field goes first on s (it only needs the
        // staged vectors), so it starts while the host still issues the upward pass
        HDM_HIP(hipEventRecord(lane.fork, s));
        near_field();
        part_reduce();
        HDM_HIP(hipStreamWaitEvent(ts, lane.fork, 0));
    } else if (fuse_up) {
        near_field();
    }
    if (tree) {
        {   // N2S: the leaves (unless the near-field launch has formed them), then
            // every level above them in one launch for operators with composites,
            // level by level for the others; the same arithmetic whatever the batch
            PhaseScope ph(cx, HDM_PHASE_N2S, ts);
            auto level_launch = [&](int k, bool with_comp) {
                for (int o = 0; o < nops; ++o) b.arg[o] = reqs[o].op->depth - k;
                auto active = [&](const Op& op) {
                    const int lvl = op.depth - k;
                    return lvl >= 1 && (with_comp || op.ncomp == 0);
                };
                if (multi) {   // one workgroup per node where the inputs fit shared memory
                    size_t shm = 0;
                    for (int o = 0; o < nops; ++o)
                        if (active(*reqs[o].op)) shm = std::max(shm, n2s_node_bytes(*reqs[o].op, reqs[o].op->depth - k, sizeof(V)));
                    if (shm <= static_cast<size_t>(kN2sNodeBytes)) {
                        const int64_t nodes = prefix([&](const Op& op, int) {
                            return active(op) ? int64_t(1) << (op.depth - k) : int64_t(0);
                        });
                        int rmax = 1;
                        for (int o = 0; o < nops; ++o)
                            if (active(*reqs[o].op)) rmax = std::max(rmax, reqs[o].op->lvl_max_rank[reqs[o].op->depth - k]);
                        if (nodes > 0)
                            hipLaunchKernelGGL((k_n2s_node_m<V, TP>), dim3(nodes, ceil_div(rmax, kN2sNodeRows)), dim3(kBlock),
                                               shm, ts, b);
                        return;
                    }
                }
                const int64_t tot = prefix([&](const Op& op, int) {
                    const int lvl = op.depth - k;
                    return lvl >= 1 && (with_comp || op.ncomp == 0) ? op.row_count[lvl] : int64_t(0);
                });
                if (tot == 0) return;
                if (multi)
                    hipLaunchKernelGGL((k_n2s_m<V, TP>), dim3(ceil_div(tot, wpb)), dim3(kBlock), 0, ts, b);
                else
                    hipLaunchKernelGGL((k_n2s<V, TP>), dim3(ceil_div(tot, wpb)), dim3(kBlock), 0, ts, b);
            };
            if (!fuse_up) level_launch(0, true);
            {   // every level above the leaves in one launch through the composites
                const int64_t tot = prefix([](const Op& op, int) {
                    return op.ncomp > 0 ? op.row_total - op.row_count[op.depth] : int64_t(0);
                });
                if (tot > 0 && multi)
                    hipLaunchKernelGGL((k_n2s_up_m<V>), dim3(ceil_div(tot, wpb)), dim3(kBlock), 0, ts, b);
                else if (tot > 0)
                    hipLaunchKernelGGL((k_n2s_up<V>), dim3(ceil_div(tot, wpb)), dim3(kBlock), 0, ts, b);
            }
            for (int k = 1; k < maxdepth; ++k) level_launch(k, false);   // operators without composites
        }
        {
            const int64_t tot = prefix([](const Op& op, int) { return op.row_total; });
            KernelEvents ev(cx, HDM_PHASE_S2S);
            if (tot > 0) {
                if (multi)
                    hipExtLaunchKernelGGL((k_s2s_m<V, TF>), dim3(ceil_div(tot, wpb)), dim3(kBlock), 0, ts, ev.start,
                                          ev.stop, 0, b);
                else
                    hipExtLaunchKernelGGL((k_s2s<V, TF>), dim3(ceil_div(tot, wpb)), dim3(kBlock), 0, ts, ev.start,
                                          ev.stop, 0, b);
            }
        }
        // S2N level by level for the operators that take it (large ranks; every
        // product with several right-hand sides)
        auto levels = [multi, f64](const Op& op) { return op.s2n_by_levels(multi, f64); };
        bool any_s2n = false;
        for (int o = 0; o < nops; ++o) any_s2n = any_s2n || levels(*reqs[o].op);
        if (any_s2n) {
            PhaseScope ph(cx, HDM_PHASE_S2N, ts);
            for (int lvl = 2; lvl <= maxdepth; ++lvl) {
                for (int o = 0; o < nops; ++o) b.arg[o] = lvl;
                const int64_t tot = prefix([&](const Op& op, int) {
                    return levels(op) && lvl <= op.depth ? int64_t(1) << lvl : int64_t(0);
                });
                if (tot == 0) continue;
                if (multi) {
                    int rmax = 1;
                    for (int o = 0; o < nops; ++o)
                        if (lvl <= reqs[o].op->depth) rmax = std::max(rmax, reqs[o].op->lvl_max_rank[lvl]);
                    hipLaunchKernelGGL((k_s2n_m<V, TP>), dim3(tot, ceil_div(rmax, kWave)), dim3(kBlock), 0, ts, b);
                } else {
                    hipLaunchKernelGGL((k_s2n<V, TP>), dim3(tot), dim3(kBlock), 0, ts, b);
                }
            }
        }
    }
    if (overlap) {
        HDM_HIP(hipEventRecord(lane.join, ts));
        HDM_HIP(hipStreamWaitEvent(s, lane.join, 0));
    } else if (!fuse_up) {
        near_field();
        part_reduce();
    }
    {
        for (int o = 0; o < nops; ++o) b.arg[o] = normalised;
        const int64_t tot = prefix([](const Op& op, int) { return static_cast<int64_t>(op.L); });
        KernelEvents ev(cx, HDM_PHASE_COMBINE);
        if (multi)
            hipExtLaunchKernelGGL((k_combine_m<V, TP>), dim3(tot), dim3(kCombBlock), 0, s, ev.start, ev.stop, 0, b);
        else
            hipExtLaunchKernelGGL((k_combine<V, TP>), dim3(tot), dim3(kCombBlock), 0, s, ev.start, ev.stop, 0, b);
    }
    check_launch("apply");
}

static void apply_dispatch(const ApplyReq* reqs, int nops, bool f64, int normalised, int nrhs, hipStream_t s,
                           Lane& lane, Ctx* cx) {
    const Op& op0 = *reqs[0].op;
    if (f64) {
        apply_t<double, double, double, double>(reqs, nops, true, normalised, nrhs, s, lane, cx);
        return;
    }
    auto far_dispatch = [&](auto near_tag) {
        using TN = decltype(near_tag);
        switch (op0.prm.far_prec) {
            case HDM_F32: apply_t<float, TN, float, float>(reqs, nops, false, normalised, nrhs, s, lane, cx); break;
            case HDM_BF16: apply_t<float, TN, bf16_t, float>(reqs, nops, false, normalised, nrhs, s, lane, cx); break;
            case HDM_F16: apply_t<float, TN, f16_t, float>(reqs, nops, false, normalised, nrhs, s, lane, cx); break;
            default: fail(HDM_EINVAL, "unsupported far precision with reduced near precision");
        }
    };
    switch (op0.prm.near_prec) {
        case HDM_F32: far_dispatch(float{}); break;
        case HDM_BF16: far_dispatch(bf16_t{}); break;
        case HDM_F16: far_dispatch(f16_t{}); break;
        default: fail(HDM_EINVAL, "unsupported near precision");
    }
}

void apply_batch(const ApplyReq* reqs, int nops, int normalised, int nrhs, hipStream_t s, Lane& lane, Ctx* cx) {
    HDM_CHECK(nops >= 1 && nops <= kMaxBatch, HDM_EINVAL, "batch size out of range");
    HDM_CHECK(nrhs >= 1 && nrhs <= kMaxRhs, HDM_EINVAL, "a batched product takes 1 to 16 right-hand sides");
    const Op& op0 = *reqs[0].op;
    const bool f64 = op0.prm.near_prec == HDM_F64;
    for (int o = 0; o < nops; ++o) {
        Op& op = *reqs[o].op;
        HDM_CHECK(op.prm.near_prec == op0.prm.near_prec && op.prm.far_prec == op0.prm.far_prec, HDM_EINVAL,
                  "a batch must share its tile precisions");
        HDM_CHECK(op.max_leaf_rank <= kMaxRank, HDM_EINTERNAL, "leaf rank above the combine kernel's limit");
        if (op.ws_nrhs < nrhs) {
            ensure_ws(op, nrhs);
            publish_descriptors(op, s);
        }
    }
    apply_dispatch(reqs, nops, f64, normalised, nrhs, s, lane, cx);
}

// ---- single-operator products as a HIP graph --------------------------------
// The product's kernels (staging, near field, the upward pass level by level,
// the far field, combine) are launch-latency bound on the host: as a graph the
// whole product is one launch.  The graph is built once per (precision path,
// normalised, right-hand sides); per call only the staging node (x) and the
// combine node (y) get new arguments.  A profiling context launches eagerly, so
// that every kernel is timed by its own start and end stamps.  The replay runs
// the near field and the upward pass one after the other (about 136 us at
// N = 32768, the sum of the kernels), where eager launches overlap them on two
// streams: graphs pay off for back-to-back products, not inside an iteration
// that interleaves other kernels with each product.
struct ProductGraph {
    hipGraph_t g = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t prep = nullptr, combine = nullptr;
    hipKernelNodeParams prep_p{}, comb_p{};
    Batch prep_b{}, comb_b{};
    ~ProductGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (g) (void)hipGraphDestroy(g);
    }
};

struct Op::GraphCache {
    std::map<uint32_t, std::unique_ptr<ProductGraph>> m;
    bool broken = false;   // graph construction failed once: eager launches from then on
};

Op::~Op() { delete graphs; }

template <typename V, typename TN, typename TF, typename TP>
static void build_product_graph(Op& op, bool f64, int normalised, int nrhs, ProductGraph& G) {
    constexpr bool mma = std::is_same<TN, f16_t>::value;
    const bool multi = nrhs > 1;
    const int wpb = kBlock / kWave;
    HDM_HIP(hipGraphCreate(&G.g, 0));
    Batch base{};
    base.nops = 1;
    base.nrhs = nrhs;
    base.op[0] = f64 ? op.dev64.get() : op.devT.get();
    base.pre[0] = 0;
    auto kernel = [&](void* func, dim3 grid, Batch bb, std::vector<hipGraphNode_t> deps, hipKernelNodeParams* keep,
                      int threads = kBlock, size_t shm = 0) {
        hipKernelNodeParams p{};
        void* args[] = {&bb};
        p.func = func;
        p.gridDim = grid;
        p.blockDim = dim3(threads);
        p.sharedMemBytes = static_cast<unsigned>(shm);
        p.kernelParams = args;
        p.extra = nullptr;
        hipGraphNode_t n = nullptr;
        HDM_HIP(hipGraphAddKernelNode(&n, G.g, deps.empty() ? nullptr : deps.data(), deps.size(), &p));
        if (keep) {
            *keep = p;
            keep->kernelParams = nullptr;
        }
        return n;
    };
    // staging
    Batch bp = base;
    bp.arg[0] = normalised;
    bp.pre[1] = mma ? op.L : op.n;
    G.prep = kernel(mma ? reinterpret_cast<void*>(&k_prep_mma) : reinterpret_cast<void*>(&k_prep<V>),
                    mma ? dim3(op.L) : dim3(ceil_div(op.n, kBlock)), bp, {}, &G.prep_p, mma ? kCombBlock : kBlock);
    G.prep_b = bp;
    // near field (one column: with the leaf level of the upward pass, as in the
    // eager schedule, and the rest of the tree after it)
    Batch bl = base;
    const int64_t nitems = static_cast<int64_t>(mma ? op.wseg_mma[nrhs > 1].size() - 1 : op.items.size());
    bl.pre[1] = nitems;
    const bool fuse_up = op.nskel > 0 && !multi;
    bl.up = fuse_up ? op.L : 0;
    void* l2l_fn = mma ? (fuse_up ? reinterpret_cast<void*>(&k_l2l_mma<true>) : reinterpret_cast<void*>(&k_l2l_mma<false>))
                       : (fuse_up ? reinterpret_cast<void*>(&k_l2l<V, TN, true, false>)
                                  : multi ? reinterpret_cast<void*>(&k_l2l<V, TN, false, true>)
                                          : reinterpret_cast<void*>(&k_l2l<V, TN, false, false>));
    hipGraphNode_t near = kernel(l2l_fn, dim3((mma ? nitems : ceil_div(nitems, wpb)) + bl.up), bl, {G.prep}, nullptr);
    const int maxg = mma ? op.red_groups_mma[1] : op.red_groups;
    if (multi && maxg > 0) {
        Batch br = base;
        br.pre[1] = op.L;
        near = kernel(reinterpret_cast<void*>(&k_part_reduce<V>), dim3(op.L, maxg, nrhs), br, {near}, nullptr);
    }
    std::vector<hipGraphNode_t> comb_deps{near};
    // S2N by level after the far field, for operators with large ranks (as eager)
    auto s2n_levels = [&](hipGraphNode_t last) {
        if (!op.s2n_by_levels(multi, f64)) return last;
        for (int lvl = 2; lvl <= op.depth; ++lvl) {
            Batch bn = base;
            bn.arg[0] = lvl;
            bn.pre[1] = int64_t(1) << lvl;
            if (multi)
                last = kernel(reinterpret_cast<void*>(&k_s2n_m<V, TP>),
                              dim3(static_cast<unsigned>(bn.pre[1]), ceil_div(std::max(op.lvl_max_rank[lvl], 1), kWave)),
                              bn, {last}, nullptr);
            else
                last = kernel(reinterpret_cast<void*>(&k_s2n<V, TP>), dim3(static_cast<unsigned>(bn.pre[1])), bn, {last},
                              nullptr);
        }
        return last;
    };
    if (fuse_up) {
        hipGraphNode_t last = near;
        if (op.ncomp > 0) {
            Batch bu = base;
            bu.pre[1] = op.row_total - op.row_count[op.depth];
            if (bu.pre[1] > 0)
                last = kernel(reinterpret_cast<void*>(&k_n2s_up<V>), dim3(ceil_div(bu.pre[1], wpb)), bu, {last},
                              nullptr);
        } else {
            for (int lvl = op.depth - 1; lvl >= 1; --lvl) {
                if (op.row_count[lvl] == 0) continue;
                Batch bn = base;
                bn.arg[0] = lvl;
                bn.pre[1] = op.row_count[lvl];
                last = kernel(reinterpret_cast<void*>(&k_n2s<V, TP>), dim3(ceil_div(op.row_count[lvl], wpb)), bn,
                              {last}, nullptr);
            }
        }
        if (op.row_total > 0) {
            Batch bs = base;
            bs.pre[1] = op.row_total;
            last = kernel(reinterpret_cast<void*>(&k_s2s<V, TF>), dim3(ceil_div(op.row_total, wpb)), bs, {last},
                          nullptr);
        }
        last = s2n_levels(last);
        comb_deps = {last};
    } else if (op.nskel > 0) {
        // upward pass, leaves first, then the levels above through the composites
        // (one launch) or one launch per level, then the far field (as eager)
        hipGraphNode_t last = G.prep;
        for (int lvl = op.depth; lvl >= 1; --lvl) {
            if (op.row_count[lvl] == 0) continue;
            if (lvl < op.depth && op.ncomp > 0) {
                Batch bu = base;
                bu.pre[1] = op.row_total - op.row_count[op.depth];
                if (bu.pre[1] > 0)
                    last = kernel(multi ? reinterpret_cast<void*>(&k_n2s_up_m<V>) : reinterpret_cast<void*>(&k_n2s_up<V>),
                                  dim3(ceil_div(bu.pre[1], wpb)), bu, {last}, nullptr);
                break;
            }
            Batch bn = base;
            bn.arg[0] = lvl;
            const size_t shm = n2s_node_bytes(op, lvl, sizeof(V));
            if (multi && shm <= static_cast<size_t>(kN2sNodeBytes)) {   // one workgroup per node (as eager)
                bn.pre[1] = int64_t(1) << lvl;
                last = kernel(reinterpret_cast<void*>(&k_n2s_node_m<V, TP>),
                              dim3(static_cast<unsigned>(bn.pre[1]), ceil_div(std::max(op.lvl_max_rank[lvl], 1), kN2sNodeRows)),
                              bn, {last}, nullptr, kBlock, shm);
                continue;
            }
            bn.pre[1] = op.row_count[lvl];
            last = kernel(multi ? reinterpret_cast<void*>(&k_n2s_m<V, TP>) : reinterpret_cast<void*>(&k_n2s<V, TP>),
                          dim3(ceil_div(op.row_count[lvl], wpb)), bn, {last}, nullptr);
        }
        if (op.row_total > 0) {
            Batch bs = base;
            bs.pre[1] = op.row_total;
            last = kernel(multi ? reinterpret_cast<void*>(&k_s2s_m<V, TF>) : reinterpret_cast<void*>(&k_s2s<V, TF>),
                          dim3(ceil_div(op.row_total, wpb)), bs, {last}, nullptr);
        }
        last = s2n_levels(last);
        if (last != G.prep) comb_deps.push_back(last);
    }
    Batch bc = base;
    bc.arg[0] = normalised;
    bc.pre[1] = op.L;
    G.combine = kernel(multi ? reinterpret_cast<void*>(&k_combine_m<V, TP>) : reinterpret_cast<void*>(&k_combine<V, TP>),
                       dim3(op.L), bc, comb_deps, &G.comb_p, kCombBlock);
    G.comb_b = bc;
    HDM_HIP(hipGraphInstantiate(&G.exec, G.g, nullptr, nullptr, 0));
}

static void build_product_graph_dispatch(Op& op, bool f64, int normalised, int nrhs, ProductGraph& G) {
    if (f64) {
        build_product_graph<double, double, double, double>(op, true, normalised, nrhs, G);
        return;
    }
    auto far = [&](auto near_tag) {
        using TN = decltype(near_tag);
        switch (op.prm.far_prec) {
            case HDM_F32: build_product_graph<float, TN, float, float>(op, false, normalised, nrhs, G); break;
            case HDM_BF16: build_product_graph<float, TN, bf16_t, float>(op, false, normalised, nrhs, G); break;
            case HDM_F16: build_product_graph<float, TN, f16_t, float>(op, false, normalised, nrhs, G); break;
            default: fail(HDM_EINVAL, "unsupported far precision with reduced near precision");
        }
    };
    switch (op.prm.near_prec) {
        case HDM_F32: far(float{}); break;
        case HDM_BF16: far(bf16_t{}); break;
        case HDM_F16: far(f16_t{}); break;
        default: fail(HDM_EINVAL, "unsupported near precision");
    }
}

// one product pass through the cached graph; false when graphs are unavailable
static bool apply_graph(Op& op, bool f64, int normalised, int nrhs, const double* x, double* y, hipStream_t s) {
    Ctx* cx = op.ctx;
    if (!cx || !cx->graphs || cx->prof.on) return false;
    if (!op.graphs) op.graphs = new Op::GraphCache();
    if (op.graphs->broken) return false;
    const uint32_t key = (f64 ? 1u : 0u) | (normalised ? 2u : 0u) | (static_cast<uint32_t>(nrhs) << 2);
    auto it = op.graphs->m.find(key);
    if (it == op.graphs->m.end()) {
        std::unique_ptr<ProductGraph> G(new ProductGraph());
        try {
            build_product_graph_dispatch(op, f64, normalised, nrhs, *G);
        } catch (const Error&) {
            op.graphs->broken = true;
            (void)hipGetLastError();
            return false;
        }
        it = op.graphs->m.emplace(key, std::move(G)).first;
    }
    ProductGraph& G = *it->second;
    Batch bp = G.prep_b;
    bp.x[0] = x;
    void* pa[] = {&bp};
    hipKernelNodeParams pp = G.prep_p;
    pp.kernelParams = pa;
    HDM_HIP(hipGraphExecKernelNodeSetParams(G.exec, G.prep, &pp));
    Batch bc = G.comb_b;
    bc.y[0] = y;
    void* ca[] = {&bc};
    hipKernelNodeParams cp = G.comb_p;
    cp.kernelParams = ca;
    HDM_HIP(hipGraphExecKernelNodeSetParams(G.exec, G.combine, &cp));
    HDM_HIP(hipGraphLaunch(G.exec, s));
    return true;
}

void apply(Op& op, int normalised, bool exact64, const double* x, double* y, int nrhs, hipStream_t s, bool graph_ok,
           bool tree_order) {
    HDM_CHECK(op.max_leaf_rank <= kMaxRank, HDM_EINTERNAL, "leaf rank above the combine kernel's limit");
    HDM_CHECK(nrhs >= 1, HDM_EINVAL, "nrhs must be >= 1");
    const int per = std::min(nrhs, kMaxRhs);   // right-hand sides per pass
    if (op.ws_nrhs < per) {
        ensure_ws(op, per);
        publish_descriptors(op, s);
    }
    const bool f64 = exact64 || op.prm.near_prec == HDM_F64;
    HDM_CHECK(!f64 || op.near64.n > 0 || op.near_elems == 0 || (exact64 && op.near_direct), HDM_EINTERNAL,
              "float64 tiles are not resident");
    // the float64 products of the degree pass belong to building the operator:
    // they are not recorded as evaluation phases
    Ctx* cx = exact64 ? nullptr : op.ctx;
    for (int c0 = 0; c0 < nrhs; c0 += per) {
        const ApplyReq r{&op, x + static_cast<int64_t>(c0) * op.n, y + static_cast<int64_t>(c0) * op.n};
        const int np = std::min(per, nrhs - c0);
        if (graph_ok && !exact64 && !tree_order && apply_graph(op, f64, normalised, np, r.x, r.y, s)) continue;
        apply_dispatch(&r, 1, f64, (normalised ? 1 : 0) | (tree_order ? 2 : 0), np, s, op.lane, cx);
    }
}

// ---- allocation-free products ---------------------------------------------------
// For callers that cannot allocate device memory (graph capture, serving loops,
// harnesses that forbid it): the workspaces of a product live in this array,
// one per device, held until the process ends.  Host code never passes the
// array's name to a kernel or a copy: it uses the address hipGetSymbolAddress
// returns for the device (scratch_for).
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};   // why the address is missing, if it is

// the layout of one product's scratch: descriptor, then the workspaces, each
// 256-byte aligned; offsets in bytes
struct ScratchLayout {
    size_t desc, w, skw, sku, part, wh, wsc, total;
};
ScratchLayout scratch_layout(const Op& op, int per) {
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const bool f64 = op.prm.near_prec == HDM_F64;
    // partial sums: a several-column pass holds per columns of its plan, a
    // one-column pass (per = 1, or the last pass of nrhs > per) one of its own
    const int64_t part = f64 || !op.packed
                             ? std::max<int64_t>(op.part_elems, 1) * per
                             : std::max<int64_t>(std::max<int64_t>(op.part_elems_mma[1], 1) * per, op.part_elems_mma[0]);
    ScratchLayout L{};
    size_t at = 0;
    L.desc = at; at += up(sizeof(OpDev));
    L.w = at; at += up(static_cast<size_t>(op.n) * per * 8);
    L.skw = at; at += up(static_cast<size_t>(std::max<int64_t>(op.nskel, 1)) * per * 8);
    L.sku = at; at += up(static_cast<size_t>(std::max<int64_t>(op.nskel, 1)) * per * 8);
    L.part = at; at += up(static_cast<size_t>(part) * 8);
    L.wh = at; at += op.packed && !f64 ? up((static_cast<size_t>(std::max<int64_t>(op.ldw, 1)) * 2 * kMaxRhs + 8) * 2) : 0;
    L.wsc = at; at += op.packed && !f64 ? up(static_cast<size_t>(op.L) * kMaxRhs * sizeof(float)) : 0;
    L.total = at;
    return L;
}
}  // namespace

void scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return;   // the allocation-free product then reports it
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch[device]) return;
    void* p = nullptr;
    const hipError_t rc = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));   // the caller made `device` current
    if (rc != hipSuccess || p == nullptr) {
        (void)hipGetLastError();
        g_scratch_err[device] = rc != hipSuccess ? rc : hipErrorInvalidSymbol;
        return;
    }
    g_scratch[device] = p;
}

void* scratch_for(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    return g_scratch[device];
}

size_t noalloc_bytes(const Op& op, int per) { return scratch_layout(op, per).total; }

// The product of hdm_matvec with every workspace in `scratch` (the device's
// array): the same kernels and launch order, so the same results bit for bit.
// Host work only: a descriptor copy pointing into the scratch, uploaded to its
// head, then the launches; no allocation on the device.
void apply_noalloc(Op& op, int normalised, const double* x, double* y, int nrhs, hipStream_t s, void* scratch_dev) {
    if (!scratch_dev) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        const hipError_t why = dev >= 0 && dev < kMaxDevices ? g_scratch_err[dev] : hipErrorInvalidDevice;
        fail(HDM_EDEVICE, std::string("the allocation-free scratch array has no address on this device: ") +
                              (why != hipSuccess ? hipGetErrorString(why) : "no context was created on it"));
    }
    HDM_CHECK(op.max_leaf_rank <= kMaxRank, HDM_EINTERNAL, "leaf rank above the combine kernel's limit");
    const int per = std::min(nrhs, kMaxRhs);
    const ScratchLayout L = scratch_layout(op, per);
    if (L.total > kScratchBytes)
        fail(HDM_ENOMEM, "the product needs " + std::to_string(L.total >> 20) + " MiB of workspace for " +
                             std::to_string(per) + " right-hand sides per pass, above the " +
                             std::to_string(kScratchBytes >> 20) + " MiB allocation-free scratch");
    const bool f64 = op.prm.near_prec == HDM_F64;
    char* base = static_cast<char*>(scratch_dev);
    OpDev D = f64 ? op.host64 : op.hostT;
    D.w = base + L.w;
    D.skw = base + L.skw;
    D.sku = base + L.sku;
    D.part = base + L.part;
    if (!f64 && op.packed) {
        D.wh = base + L.wh;
        D.wsc = reinterpret_cast<float*>(base + L.wsc);
    }
    // D is pageable host memory: the copy is complete when the call returns
    HDM_HIP(hipMemcpyAsync(base + L.desc, &D, sizeof(OpDev), hipMemcpyHostToDevice, s));
    const OpDev* desc = reinterpret_cast<const OpDev*>(base + L.desc);
    for (int c0 = 0; c0 < nrhs; c0 += per) {
        ApplyReq r{&op, x + static_cast<int64_t>(c0) * op.n, y + static_cast<int64_t>(c0) * op.n, desc};
        const int np = std::min(per, nrhs - c0);
        apply_dispatch(&r, 1, f64, normalised, np, s, op.lane, nullptr);
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
    op.near_ones_next = op.part_ones.n > 0;   // the product of K~ with ones reuses the near field made early
    apply(op, 0, true, ones.get(), qo.get(), 1, s);
    op.near_ones_next = false;
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
    publish_descriptors(op, s);   // the descriptors now carry c
}

// Upload of host index arrays for a conversion: kept in `keep` (host copy and
// device buffer) when the caller does not wait for s, else temporaries.
struct Staging {
    Op::ConvKeep* keep;
    hipStream_t s;
    std::vector<DevBuf<int64_t>> t64;
    std::vector<DevBuf<int32_t>> t32;
    const int64_t* up(const std::vector<int64_t>& v) {
        if (keep) {
            keep->h64.push_back(v);
            keep->d64.push_back(to_device(keep->h64.back(), s));
            return keep->d64.back().get();
        }
        t64.push_back(to_device(v, s));
        return t64.back().get();
    }
    const int32_t* up(const std::vector<int32_t>& v) {
        if (keep) {
            keep->h32.push_back(v);
            keep->d32.push_back(to_device(keep->h32.back(), s));
            return keep->d32.back().get();
        }
        t32.push_back(to_device(v, s));
        return t32.back().get();
    }
};

template <typename T>
static void convert_tiles(const DevBuf<double>& src, const std::vector<int64_t>& off, const std::vector<int64_t>& cnt,
                          bool scaled, DevBuf<char>& dst, DevBuf<float>& scale, int64_t elems, hipStream_t s,
                          Op::ConvKeep* keep = nullptr) {
    dst.alloc(static_cast<size_t>(std::max<int64_t>(elems, 1)) * sizeof(T));
    if (off.empty()) return;
    Staging st{keep, s, {}, {}};
    st.t64.reserve(2);
    const int64_t* doff_p = st.up(off);
    const int64_t* dcnt_p = st.up(cnt);
    struct { const int64_t* p; const int64_t* get() const { return p; } } doff{doff_p}, dcnt{dcnt_p};
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
    if (!keep) HDM_HIP(hipStreamSynchronize(s));
}

// float16 near tiles in the packed matrix-core layout, one scale per tile
static void pack_near(Op& op, const std::vector<int64_t>& noff, const std::vector<int64_t>& ncnt, hipStream_t s,
                      Op::ConvKeep* keep = nullptr) {
    const int64_t L = op.L;
    const size_t nt = noff.size();
    op.nearT.alloc(static_cast<size_t>(std::max<int64_t>(op.near_elems_mma, 1)) * sizeof(_Float16));
    if (nt == 0) return;
    std::vector<int64_t> offp(nt);
    std::vector<int32_t> ld(nt), na(nt), nb(nt);
    int64_t maxg = 0;
    for (int64_t a = 0; a < L; ++a)
        for (int32_t t = op.near_off[a]; t < op.near_off[a + 1]; ++t) {
            offp[t] = op.near_tile_off_mma[t];
            ld[t] = op.near_ld[a];
            na[t] = static_cast<int32_t>(op.size[L + a]);
            nb[t] = static_cast<int32_t>(op.size[L + op.near_idx[t]]);
            maxg = std::max<int64_t>(maxg, static_cast<int64_t>(ld[t]) * ((nb[t] + 7) / 8));
            HDM_CHECK(offp[t] + static_cast<int64_t>(ld[t]) * ((nb[t] + 7) / 8 * 8) <= op.near_elems_mma &&
                          noff[t] + ncnt[t] <= op.near_elems && ncnt[t] == static_cast<int64_t>(ld[t]) * nb[t],
                      HDM_EINTERNAL, "packed near tile outside its buffer");
        }
    Staging st{keep, s, {}, {}};
    st.t64.reserve(3);
    st.t32.reserve(3);
    struct P64 { const int64_t* p; const int64_t* get() const { return p; } };
    struct P32 { const int32_t* p; const int32_t* get() const { return p; } };
    const P64 d_off{st.up(noff)}, d_cnt{st.up(ncnt)}, d_offp{st.up(offp)};
    const P32 d_ld{st.up(ld)}, d_na{st.up(na)}, d_nb{st.up(nb)};
    op.near_scale.alloc(nt);
    hipLaunchKernelGGL(k_tile_max, dim3(nt), dim3(kBlock), 0, s, op.near64.get(), d_off.get(), d_cnt.get(),
                       op.near_scale.get());
    const unsigned gx = static_cast<unsigned>(std::min<int64_t>(ceil_div(maxg, kBlock), 64));
    for (size_t base = 0; base < nt; base += 65535) {
        const int cnt = static_cast<int>(std::min<size_t>(65535, nt - base));
        hipLaunchKernelGGL(k_pack_near, dim3(gx, cnt), dim3(kBlock), 0, s, op.near64.get(), d_off.get() + base,
                           d_offp.get() + base, d_ld.get() + base, d_na.get() + base, d_nb.get() + base,
                           op.near_scale.get() + base, reinterpret_cast<_Float16*>(op.nearT.get()));
    }
    check_launch("pack near tiles");
    if (!keep) HDM_HIP(hipStreamSynchronize(s));
}

// offsets of the near tiles in the float64 layout (one entry per near pair)
static void near_ranges(const Op& op, std::vector<int64_t>& noff, std::vector<int64_t>& ncnt) {
    const int64_t L = op.L;
    noff.clear();
    ncnt.clear();
    for (int64_t a = 0; a < L; ++a)
        for (int32_t t = op.near_off[a]; t < op.near_off[a + 1]; ++t) {
            noff.push_back(op.near_tile_off[t]);
            ncnt.push_back(static_cast<int64_t>(op.near_ld[a]) * op.size[L + op.near_idx[t]]);
        }
}

// offsets of the packed float16 near tiles (ld_a x |b| rounded up to 8 per pair)
void packed_near_offsets(Op& op) {
    op.near_tile_off_mma.assign(op.near_idx.size(), 0);
    int64_t off = 0;
    for (int64_t a = 0; a < op.L; ++a)
        for (int32_t t = op.near_off[a]; t < op.near_off[a + 1]; ++t) {
            op.near_tile_off_mma[t] = off;
            off += static_cast<int64_t>(op.near_ld[a]) * ((op.size[op.L + op.near_idx[t]] + 7) / 8 * 8);
        }
    op.near_elems_mma = off;
}

void convert_near_tiles(Op& op, hipStream_t s) {
    if (op.prm.near_prec == HDM_F64 || op.near_converted) return;
    op.conv_keep.reset(new Op::ConvKeep());
    Op::ConvKeep* keep = op.conv_keep.get();
    std::vector<int64_t> noff, ncnt;
    near_ranges(op, noff, ncnt);
    switch (op.prm.near_prec) {
        case HDM_F32: convert_tiles<float>(op.near64, noff, ncnt, false, op.nearT, op.near_scale, op.near_elems, s, keep); break;
        case HDM_BF16: convert_tiles<bf16_t>(op.near64, noff, ncnt, true, op.nearT, op.near_scale, op.near_elems, s, keep); break;
        case HDM_F16: packed_near_offsets(op); pack_near(op, noff, ncnt, s, keep); break;
        default: fail(HDM_EINVAL, "bad tile precision");
    }
    op.near_converted = true;
}

void convert_eval_precision(Op& op, hipStream_t s) {
    if (op.prm.near_prec == HDM_F64 && op.prm.far_prec == HDM_F64) return;
    HDM_CHECK(op.prm.near_prec != HDM_F64 && op.prm.far_prec != HDM_F64, HDM_EINVAL,
              "float64 tiles cannot be mixed with reduced-precision tiles");
    // the index arrays of the conversions stay alive until finish_operator has
    // waited for s
    if (!op.conv_keep) op.conv_keep.reset(new Op::ConvKeep());
    Op::ConvKeep* keep = op.conv_keep.get();
    // near: one scale per tile (pair)
    std::vector<int64_t> noff, ncnt;
    near_ranges(op, noff, ncnt);
    // far: one scale per node block (indexed by heap id)
    std::vector<int64_t> foff(op.nnodes, 0), fcnt(op.nnodes, 0);
    for (int64_t h = 0; h < op.nnodes; ++h) {
        foff[h] = op.far_block_off[h];
        fcnt[h] = static_cast<int64_t>(op.rank[h]) * op.far_cols[h];
    }
    auto go = [&](int prec, const DevBuf<double>& src, const std::vector<int64_t>& off, const std::vector<int64_t>& cnt,
                  DevBuf<char>& dst, DevBuf<float>& scale, int64_t elems) {
        switch (prec) {
            case HDM_F32: convert_tiles<float>(src, off, cnt, false, dst, scale, elems, s, keep); break;
            case HDM_BF16: convert_tiles<bf16_t>(src, off, cnt, true, dst, scale, elems, s, keep); break;
            case HDM_F16: convert_tiles<f16_t>(src, off, cnt, true, dst, scale, elems, s, keep); break;
            default: fail(HDM_EINVAL, "bad tile precision");
        }
    };
    if (op.near_converted) {
        // converted on the side stream while the operator was built; s has waited for it
    } else if (op.packed) {
        pack_near(op, noff, ncnt, s, keep);
    } else {
        go(op.prm.near_prec, op.near64, noff, ncnt, op.nearT, op.near_scale, op.near_elems);
    }
    go(op.prm.far_prec, op.far64, foff, fcnt, op.farT, op.far_scale, op.far_elems);
    op.P32.alloc(std::max<int64_t>(op.np, 1));
    if (op.np > 0)
        hipLaunchKernelGGL(k_to_f32, dim3(ceil_div(op.np, kBlock)), dim3(kBlock), 0, s, op.P64.get(), op.P32.get(), op.np);
    check_launch("P to f32");
}

void finish_operator(Op& op, hipStream_t s) {
    // the near tiles' conversion may still run on the side stream
    if (op.lane.side) HDM_HIP(hipStreamSynchronize(op.lane.side));
    HDM_HIP(hipStreamSynchronize(s));
    op.near_pairs.release();
    op.part_ones.release();
    op.build_keep.reset();
    op.conv_keep.reset();
    if (!(op.prm.near_prec == HDM_F64 && op.prm.far_prec == HDM_F64)) {
        // the float64 tiles were only needed for the degrees
        op.near64.release();
        op.far64.release();
    }
    publish_descriptors(op, s);
}

}  // namespace hdm
