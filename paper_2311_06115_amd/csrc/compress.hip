// Geometry-oblivious compression on the GPU: kernel-space ball tree,
// randomized-tree neighbours, near/far interaction lists, nested skeletons by a
// sampled-row interpolative decomposition, and the kernel tiles of Eq. (3).
//
// Every decision (argmin, median cut, neighbour order, pivot) is taken in
// float64 with a total order (value, index); this file is compiled with
// -ffp-contract=off so each product and sum is one IEEE operation in the order
// written, which keeps the tree and the neighbour lists reproducible.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <type_traits>

#include "op.hpp"

namespace hdm {

namespace {

constexpr int kSample = 64;     // points sampled per node for the centroid
constexpr int kMaxCand = 2048;  // candidates of one node (leaf points or children's skeletons)
constexpr int kBlock = 256;
constexpr int kWave = 64;

struct Pts {
    const double* xf;
    const uint8_t* xu;
    const int32_t* nu;   // u8 codes: sum of squared codes per point (exact integer)
    int dim;
    int is_u8;
    double eps;
};

// ||x_i - x_j||^2 summed over coordinates in increasing order; for u8 codes the
// exact integer sum (a - b)^2 = a.a + b.b - 2 a.b, then divided by 255^2
__device__ inline double sqd(const Pts& P, int64_t i, int64_t j) {
    if (P.is_u8 && P.nu) {
        const uint32_t* a = reinterpret_cast<const uint32_t*>(P.xu + i * P.dim);
        const uint32_t* b = reinterpret_cast<const uint32_t*>(P.xu + j * P.dim);
        uint32_t g = 0;
        for (int d = 0; d < P.dim / 4; ++d) g = __builtin_amdgcn_udot4(a[d], b[d], g, false);
        const int32_t s2 = P.nu[i] + P.nu[j] - 2 * static_cast<int32_t>(g);
        return static_cast<double>(s2) / 65025.0;
    }
    if (P.is_u8) {
        const uint8_t* a = P.xu + i * P.dim;
        const uint8_t* b = P.xu + j * P.dim;
        int acc = 0;
        for (int d = 0; d < P.dim; ++d) {
            const int t = static_cast<int>(a[d]) - static_cast<int>(b[d]);
            acc += t * t;
        }
        return static_cast<double>(acc) / 65025.0;
    }
    const double* a = P.xf + i * P.dim;
    const double* b = P.xf + j * P.dim;
    double acc = 0.0;
    for (int d = 0; d < P.dim; ++d) {
        const double t = a[d] - b[d];
        acc = acc + t * t;
    }
    return acc;
}

// e^x for the kernel values.  The tree, neighbour and skeleton decisions are
// taken on kernel values, and the library exponentials of the device and of a
// CPU are not correctly rounded, so e^x is evaluated here by one fixed sequence
// of IEEE operations (this file is built with -ffp-contract=off): Cody and
// Waite's reduction x = n ln2 + r with n = floor(x / ln2 + 1/2) and ln2 split
// into a 32-bit high part (n times it is exact) and the rest; e^r by its Taylor
// polynomial of degree 13 (|r| <= ln2 / 2, omitted terms below 1e-17 relative) in
// Horner form with fused multiply-adds; the product with 2^n, through two exact
// powers of two when it is subnormal.  x <= -745.2 gives 0.  Within 1-2 ulp of
// e^x.  Constants: the doubles nearest ln2's high part, ln2 - high, 1/ln2 and 1/k!.
// Kernels whose kernel values decide nothing (the float64 degree products'
// near field, the tile scales) use the device's faster exp instead.
__device__ inline double det_exp(double x) {
    constexpr double kLn2Hi = 0x1.62e42fee00000p-1, kLn2Lo = 0x1.a39ef35793c76p-33, kInvLn2 = 0x1.71547652b82fep+0;
    if (!(x > -745.2)) return 0.0;
    const double n = floor(x * kInvLn2 + 0.5);
    const double r = (x - n * kLn2Hi) - n * kLn2Lo;
    double p = 0x1.6124613a86d09p-33;   // 1/13!
    p = fma(p, r, 0x1.1eed8eff8d898p-29);   // 1/12!
    p = fma(p, r, 0x1.ae64567f544e4p-26);   // 1/11!
    p = fma(p, r, 0x1.27e4fb7789f5cp-22);   // 1/10!
    p = fma(p, r, 0x1.71de3a556c734p-19);   // 1/9!
    p = fma(p, r, 0x1.a01a01a01a01ap-16);   // 1/8!
    p = fma(p, r, 0x1.a01a01a01a01ap-13);   // 1/7!
    p = fma(p, r, 0x1.6c16c16c16c17p-10);   // 1/6!
    p = fma(p, r, 0x1.1111111111111p-7);    // 1/5!
    p = fma(p, r, 0x1.5555555555555p-5);    // 1/4!
    p = fma(p, r, 0x1.5555555555555p-3);    // 1/3!
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    const int e = static_cast<int>(n);
    if (e >= -1021) return p * ldexp(1.0, e);
    return (p * ldexp(1.0, e + 600)) * ldexp(1.0, -600);
}

// Eq. (2): exp(-||x_i - x_j||^2 / eps)
__device__ inline double kval(const Pts& P, int64_t i, int64_t j) { return det_exp(-(sqd(P, i, j) / P.eps)); }

// ---------------------------------------------------------------------------
// u8 codes: exact squared distances of whole blocks with int8 matrix cores.
// With a = code - 128 (an int8), ||a - b||^2 = |a|^2 + |b|^2 - 2 a.b exactly;
// a.b comes from v_mfma_i32_16x16x64_i8 over 64-byte slices of the codes.
// ---------------------------------------------------------------------------
typedef int v4i __attribute__((ext_vector_type(4)));

struct GramBlock {
    const int32_t* ridx;   // row points (original indices)
    const int32_t* cidx;   // column points
    int32_t nr, nc;
    int64_t off;           // output offset (elements)
    int32_t ld;            // leading dimension of the output
    int32_t colmajor;      // 1: out[off + c * ld + r]; 0: out[off + r * ld + c]
};

__global__ void k_code_norms(const uint8_t* x, int64_t n, int dim, int32_t* nu, int32_t* ns) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    const uint32_t* a = reinterpret_cast<const uint32_t*>(x + i * dim);
    uint32_t g = 0;
    int32_t t = 0;
    for (int d = 0; d < dim / 4; ++d) {
        g = __builtin_amdgcn_udot4(a[d], a[d], g, false);
        const uint32_t w = a[d] ^ 0x80808080u;
        t = __builtin_amdgcn_sdot4(static_cast<int32_t>(w), static_cast<int32_t>(w), t, false);
    }
    nu[i] = static_cast<int32_t>(g);
    ns[i] = t;
}

// 16 code bytes of point idx at byte k, offset to int8 (zero outside)
__device__ inline v4i codes16(const uint8_t* x, int32_t idx, int k, int dim) {
    if (idx < 0 || k >= dim) return v4i{0, 0, 0, 0};
    const uint4 u = *reinterpret_cast<const uint4*>(x + static_cast<int64_t>(idx) * dim + k);
    return v4i{static_cast<int>(u.x ^ 0x80808080u), static_cast<int>(u.y ^ 0x80808080u),
               static_cast<int>(u.z ^ 0x80808080u), static_cast<int>(u.w ^ 0x80808080u)};
}

// one 64 x 64 output tile per workgroup (blockIdx.x: tile, blockIdx.y: block);
// mode 0 writes the integer 255^2 ||x - y||^2, mode 1 the float64 kernel value
__global__ void __launch_bounds__(256) k_gram_u8(const GramBlock* blocks, const uint8_t* x, const int32_t* ns, int dim,
                                                 double eps, int mode, void* out) {
    const GramBlock B = blocks[blockIdx.y];
    if (B.nr <= 0 || B.nc <= 0) return;
    const int tiles_c = (B.nc + 63) / 64;
    const int tr = blockIdx.x / tiles_c, tc = blockIdx.x % tiles_c;
    if (tr * 64 >= B.nr) return;
    const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int g = lane / 16, li = lane % 16;
    const int r0 = tr * 64 + wv * 16, c0 = tc * 64;
    const int32_t ia = r0 + li < B.nr ? B.ridx[r0 + li] : -1;
    int32_t ib[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) ib[t] = c0 + 16 * t + li < B.nc ? B.cidx[c0 + 16 * t + li] : -1;
    v4i acc[4] = {};
    for (int k0 = 0; k0 < dim; k0 += 64) {
        const int kk = k0 + 16 * g;
        const v4i a = codes16(x, ia, kk, dim);
#pragma unroll
        for (int t = 0; t < 4; ++t)
            acc[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, codes16(x, ib[t], kk, dim), acc[t], 0, 0, 0);
    }
    // acc[t][q] holds row r0 + 4 g + q, column c0 + 16 t + li
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int c = c0 + 16 * t + li;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = r0 + 4 * g + q;
            if (r >= B.nr || c >= B.nc) continue;
            const int32_t s2 = ns[B.ridx[r]] + ns[B.cidx[c]] - 2 * acc[t][q];
            const int64_t e = B.off + (B.colmajor ? static_cast<int64_t>(c) * B.ld + r : static_cast<int64_t>(r) * B.ld + c);
            if (mode == 0) static_cast<int32_t*>(out)[e] = s2;
            else static_cast<double*>(out)[e] = det_exp(-((static_cast<double>(s2) / 65025.0) / eps));
        }
    }
}

// sequential sum of each row of a row-major matrix (the order the sample sum uses)
__global__ void k_row_sums(const double* v, int64_t rows, const int32_t* ncols, int ld, int lvl,
                           const int64_t* start, double* out) {
    const int64_t pos = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (pos >= rows) return;
    int64_t h = 1;
    for (int l = 0; l < lvl; ++l) h = (pos < start[2 * h + 1]) ? 2 * h : 2 * h + 1;
    const int nc = ncols[h - (int64_t(1) << lvl)];
    double acc = 0.0;
    for (int q = 0; q < nc; ++q) acc = acc + v[pos * ld + q];
    out[pos] = acc;
}

// original indices of each node's sample (the Gram blocks' column lists)
__global__ void k_sample_ids(const int32_t* samp, const int32_t* nsamp, const int32_t* perm, int nodes, int32_t* ids) {
    const int t = blockIdx.x;
    if (t >= nodes) return;
    for (int q = threadIdx.x; q < nsamp[t]; q += blockDim.x) ids[t * 64 + q] = perm[samp[t * 64 + q]];
}

// heap id of the level-lvl node holding tree position pos
__device__ inline int64_t node_of(int64_t pos, int lvl, const int64_t* start) {
    int64_t h = 1;
    for (int l = 0; l < lvl; ++l) h = (pos < start[2 * h + 1]) ? 2 * h : 2 * h + 1;
    return h;
}

// ---------------------------------------------------------------------------
// tree construction
// ---------------------------------------------------------------------------
// identity permutation, one copy of n entries per tree (blockIdx.y)
__global__ void k_iota(int32_t* p, int64_t n) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i < n) p[blockIdx.y * n + i] = static_cast<int32_t>(i);
}

// Floyd's sampling of min(n, 64) distinct positions of each node, ascending.
// One wave per node: draws stay sequential (Floyd's rule depends on earlier
// picks); lane q holds pick q, membership is a ballot, and the final order is
// each pick's rank among the 64.
__global__ void __launch_bounds__(64) k_tree_sample(int lvl, const int64_t* start, const int64_t* size, uint64_t seed,
                                                    int32_t* samp, int32_t* nsamp) {
    const int64_t t = blockIdx.x;
    const int64_t h = (int64_t(1) << lvl) + t;
    const int64_t n = size[h];
    const int lane = threadIdx.x;
    int32_t* out = samp + t * kSample;
    if (n <= kSample) {
        if (lane < n) out[lane] = static_cast<int32_t>(start[h] + lane);
        if (lane == 0) nsamp[t] = static_cast<int32_t>(n);
        return;
    }
    int32_t mine = -1;   // pick number `lane`
    for (int q = 0; q < kSample; ++q) {
        const int64_t j = n - kSample + q;
        const int32_t r = static_cast<int32_t>(
            below(philox_draw(seed, kTreeSample, static_cast<uint32_t>(h), 0, static_cast<uint32_t>(j)),
                  static_cast<uint32_t>(j + 1)));
        const bool present = __ballot(lane < q && mine == r) != 0;
        if (lane == q) mine = present ? static_cast<int32_t>(j) : r;
    }
    int rank = 0;
    for (int q = 0; q < kSample; ++q) rank += __shfl(mine, q, 64) < mine;
    out[rank] = static_cast<int32_t>(start[h] + mine);
    if (lane == 0) nsamp[t] = kSample;
}

// sum over the node's sample of K(x_i, x_j), in ascending sample position.
// When the workgroup's positions lie in at most two nodes (float64 points of
// at most kTreeDim coordinates), the nodes' sample points are staged in shared
// memory and every term is formed from registers and shared memory with the
// operations of kval in the same order.
constexpr int kTreeDim = 16;
__global__ void __launch_bounds__(kBlock) k_tree_sumk(int lvl, int64_t n, const int64_t* start,
                                                       const int32_t* perm, const int32_t* samp,
                                                       const int32_t* nsamp, Pts P, double* sumk) {
    __shared__ double xs[2][kSample][kTreeDim];
    const int64_t b0 = blockIdx.x * static_cast<int64_t>(blockDim.x);
    const int64_t b1 = min(n, b0 + static_cast<int64_t>(blockDim.x)) - 1;
    const int64_t base = int64_t(1) << lvl;
    const int64_t t0 = node_of(b0, lvl, start) - base, t1 = node_of(b1, lvl, start) - base;
    const int64_t pos = b0 + threadIdx.x;
    if (P.is_u8 || P.dim > kTreeDim || t1 - t0 > 1) {   // uniform over the workgroup
        if (pos >= n) return;
        const int64_t t = node_of(pos, lvl, start) - base;
        const int32_t i = perm[pos];
        double acc = 0.0;
        const int ns = nsamp[t];
        for (int q = 0; q < ns; ++q) acc = acc + kval(P, i, perm[samp[t * kSample + q]]);
        sumk[pos] = acc;
        return;
    }
    const int dim = P.dim;
    for (int e = threadIdx.x; e < 2 * kSample * dim; e += blockDim.x) {
        const int k = e / (kSample * dim), q = (e / dim) % kSample, d = e % dim;
        const int64_t t = k == 0 ? t0 : t1;
        xs[k][q][d] = q < nsamp[t] ? P.xf[static_cast<int64_t>(perm[samp[t * kSample + q]]) * dim + d] : 0.0;
    }
    __syncthreads();
    if (pos >= n) return;
    const int k = (t1 != t0 && pos >= start[base + t1]) ? 1 : 0;
    const int ns = nsamp[k == 0 ? t0 : t1];
    const double* xi = P.xf + static_cast<int64_t>(perm[pos]) * dim;
    double a[kTreeDim];
#pragma unroll
    for (int d = 0; d < kTreeDim; ++d) a[d] = d < dim ? xi[d] : 0.0;
    double acc = 0.0;
    for (int q = 0; q < ns; ++q) {
        double sq = 0.0;
#pragma unroll
        for (int d = 0; d < kTreeDim; ++d)
            if (d < dim) {
                const double t = a[d] - xs[k][q][d];
                sq = sq + t * t;
            }
        acc = acc + det_exp(-(sq / P.eps));
    }
    sumk[pos] = acc;
}

// lexicographic block reduction helpers: (value, position), smaller wins / larger wins
__device__ inline void block_argbest(double& v, int64_t& p, bool want_min, double* sv, int64_t* sp) {
    const int tid = threadIdx.x;
    sv[tid] = v;
    sp[tid] = p;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (tid < w) {
            const double ov = sv[tid + w];
            const int64_t op = sp[tid + w];
            const bool better = want_min ? (ov < sv[tid] || (ov == sv[tid] && op < sp[tid]))
                                         : (ov > sv[tid] || (ov == sv[tid] && op < sp[tid]));
            if (better) { sv[tid] = ov; sp[tid] = op; }
        }
        __syncthreads();
    }
    v = sv[0];
    p = sp[0];
    __syncthreads();
}

// p = argmin sumk (the point farthest from the sample centroid in feature space),
// q = argmax ||x - x_p||^2; ties go to the lower position.  Each thread scans
// its positions in increasing order, eight loads in flight.
constexpr int kPqBlock = 1024;
__global__ void __launch_bounds__(kPqBlock) k_tree_pq(int lvl, const int64_t* start, const int64_t* size,
                                                      const int32_t* perm, const double* sumk, Pts P, int32_t* pq) {
    __shared__ double sv[kPqBlock];
    __shared__ int64_t sp[kPqBlock];
    const int64_t t = blockIdx.x;
    const int64_t h = (int64_t(1) << lvl) + t;
    const int64_t s0 = start[h], n = size[h], s1 = s0 + n;
    const int64_t B = blockDim.x;
    double best = INFINITY;
    int64_t bpos = INT64_MAX;
    for (int64_t p0 = s0 + threadIdx.x; p0 < s1; p0 += 8 * B) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p0 + u * B < s1 ? sumk[p0 + u * B] : INFINITY;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t pos = p0 + u * B;
            if (pos < s1 && (v[u] < best || (v[u] == best && pos < bpos))) { best = v[u]; bpos = pos; }
        }
    }
    block_argbest(best, bpos, true, sv, sp);
    if (bpos < s0 || bpos >= s1) bpos = s0;   // only reachable with non-finite sums
    const int32_t ip = perm[bpos];
    double far = -1.0;
    int64_t fpos = INT64_MAX;
    for (int64_t p0 = s0 + threadIdx.x; p0 < s1; p0 += 8 * B) {
        int32_t ii[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) ii[u] = perm[min(p0 + u * B, s1 - 1)];
        double d[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) d[u] = sqd(P, ii[u], ip);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t pos = p0 + u * B;
            if (pos < s1 && (d[u] > far || (d[u] == far && pos < fpos))) { far = d[u]; fpos = pos; }
        }
    }
    block_argbest(far, fpos, false, sv, sp);
    if (fpos < s0 || fpos >= s1) fpos = s0;
    if (threadIdx.x == 0) {
        pq[2 * t] = ip;
        pq[2 * t + 1] = perm[fpos];
    }
}

// random pivots p != q of each node of a neighbour-search tree
// random pivots of the neighbour trees; tree it + blockIdx.y uses its own
// permutation (stride n) and pivot slots (stride pq_stride)
__global__ void k_knn_pq(int lvl, const int64_t* start, const int64_t* size, const int32_t* perm_all, int64_t n_all,
                         uint64_t seed, int it0, int32_t* pq_all, int64_t pq_stride) {
    const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    const int64_t nodes = int64_t(1) << lvl;
    if (t >= nodes) return;
    const int it = it0 + static_cast<int>(blockIdx.y);
    const int32_t* perm = perm_all + blockIdx.y * n_all;
    int32_t* pq = pq_all + blockIdx.y * pq_stride;
    const int64_t h = nodes + t;
    const uint32_t n = static_cast<uint32_t>(size[h]);
    const uint32_t a = below(philox_draw(seed, kKnnPivot, static_cast<uint32_t>(h), static_cast<uint32_t>(it), 0), n);
    uint32_t b = below(philox_draw(seed, kKnnPivot, static_cast<uint32_t>(h), static_cast<uint32_t>(it), 1), n - 1);
    if (b >= a) ++b;
    pq[2 * t] = perm[start[h] + a];
    pq[2 * t + 1] = perm[start[h] + b];
}

// split key: mode 0 (ball tree) K(x,q) - K(x,p); mode 1 (neighbour trees) |x-p|^2 - |x-q|^2
__global__ void k_tree_key(int lvl, int64_t n, const int64_t* start, const int32_t* perm_all, const int32_t* pq_all,
                           int64_t pq_stride, Pts P, int mode, double* key_all) {
    const int64_t pos = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (pos >= n) return;
    const int32_t* perm = perm_all + blockIdx.y * n;     // tree blockIdx.y
    const int32_t* pq = pq_all + blockIdx.y * pq_stride;
    double* key = key_all + blockIdx.y * n;
    const int64_t t = node_of(pos, lvl, start) - (int64_t(1) << lvl);
    const int32_t i = perm[pos], p = pq[2 * t], q = pq[2 * t + 1];
    key[pos] = mode == 0 ? kval(P, i, q) - kval(P, i, p) : sqd(P, i, p) - sqd(P, i, q);
}

// Exclusive prefix count of a 0/1 flag over the workgroup in thread order
// (wave ballots + one shared-memory pass); *total receives the workgroup's count.
__device__ inline int wg_flag_scan(bool f, int* wsum, int* total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint64_t bal = __ballot(f);
    const int in_wave = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wv] = __popcll(bal);
    __syncthreads();
    int before = 0, tot = 0;
    for (int w = 0; w < nw; ++w) {
        const int c = wsum[w];
        before += w < wv ? c : 0;
        tot += c;
    }
    __syncthreads();
    *total = tot;
    return before + in_wave;
}

// Exclusive prefix sum of an int over the workgroup in thread order (wave
// shuffles + one shared-memory pass); *total receives the workgroup's sum.
__device__ inline int wg_scan_excl(int v, int* wsum, int* total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int incl = v;
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int before = 0, tot = 0;
    for (int w = 0; w < nw; ++w) {
        const int c = wsum[w];
        before += w < wv ? c : 0;
        tot += c;
    }
    __syncthreads();
    *total = tot;
    return before + incl - v;
}

// order-preserving image of a float64 key as an unsigned integer (+0 for zero)
__device__ inline uint64_t orderable(double x) {
    if (x == 0.0) x = 0.0;
    const uint64_t u = static_cast<uint64_t>(__double_as_longlong(x));
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// Median cut of every node, one workgroup per node.  The floor(n/2) members
// with the smallest (key, position) go left; positions follow ascending
// original index, so this is the (key, index) order.  The threshold is found by
// radix selection (eight 8-bit digits of the key image, ties by position), then
// the node is partitioned stably: both halves keep ascending original index.
// Each thread owns a contiguous run of positions for the partition; with at
// most kSplitReg per thread the run's key images stay in registers for all
// passes (else the histograms read the keys strided over the node).  Histogram
// counts of a wave whose active lanes share a bin (the common case for the
// leading digits) go in as one atomic.
constexpr int kSplitBlock = 1024;
constexpr int kSplitReg = 32;

__device__ inline void hist_add(int* hist, bool act, uint32_t bin) {
    const uint64_t am = __ballot(act);
    if (!am) return;
    const int lead = __ffsll(static_cast<long long>(am)) - 1;
    const uint32_t b0 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(bin), lead));
    const uint64_t same = __ballot(act && bin == b0);
    if (same == am) {
        if ((threadIdx.x & 63) == lead) atomicAdd(&hist[b0], __popcll(am));
    } else if (act) {
        atomicAdd(&hist[bin], 1);
    }
}

template <bool kReg>
__global__ void __launch_bounds__(kSplitBlock) k_tree_split(int lvl, const int64_t* start, const int64_t* size,
                                                            const int32_t* perm_all, const double* key_all,
                                                            int32_t* out_all, int64_t tstride) {
    // tree blockIdx.y: its permutation, keys and output at offset blockIdx.y * tstride
    const int32_t* perm = perm_all + blockIdx.y * tstride;
    const double* key = key_all + blockIdx.y * tstride;
    int32_t* out = out_all + blockIdx.y * tstride;
    __shared__ int hist[256];
    __shared__ int wsum[kSplitBlock / 64];
    __shared__ uint64_t s_prefix;
    __shared__ int s_k;
    const int64_t h = (int64_t(1) << lvl) + blockIdx.x;
    const int64_t s0 = start[h];
    const int n = static_cast<int>(size[h]);
    const int nl = n / 2;
    const int per = (n + static_cast<int>(blockDim.x) - 1) / static_cast<int>(blockDim.x);
    const int a0 = min(n, static_cast<int>(threadIdx.x) * per), a1 = min(n, a0 + per);
    constexpr int R = kReg ? kSplitReg : 1;
    uint64_t ur[R];
    if constexpr (kReg) {
#pragma unroll
        for (int r = 0; r < R; ++r) ur[r] = a0 + r < a1 ? orderable(key[s0 + a0 + r]) : 0;
    }
    auto img = [&](int r) -> uint64_t {   // key image of position a0 + r
        if constexpr (kReg) return ur[r];
        else return orderable(key[s0 + a0 + r]);
    };
    const int cnt = a1 - a0;
    constexpr int RU = kReg ? kSplitReg : 1;
    if (threadIdx.x == 0) { s_prefix = 0; s_k = nl; }
    uint64_t mask = 0;
    for (int shift = 56; shift >= 0; shift -= 8) {
        for (int b = threadIdx.x; b < 256; b += blockDim.x) hist[b] = 0;
        __syncthreads();
        const uint64_t prefix = s_prefix;
        if constexpr (kReg) {
#pragma unroll
            for (int r = 0; r < RU; ++r) {
                const bool in = r < cnt;
                const uint64_t u = ur[r];
                hist_add(hist, in && (u & mask) == prefix, static_cast<uint32_t>((u >> shift) & 255u));
            }
        } else {
            // strided over the node (coalesced), eight loads in flight per thread;
            // every wave runs the same rounds
            for (int q0 = 0; q0 < per; q0 += 8) {
                uint64_t u8[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int a = static_cast<int>(threadIdx.x) + (q0 + t) * static_cast<int>(blockDim.x);
                    u8[t] = orderable(key[s0 + min(a, n - 1)]);
                }
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int a = static_cast<int>(threadIdx.x) + (q0 + t) * static_cast<int>(blockDim.x);
                    const bool in = q0 + t < per && a < n;
                    hist_add(hist, in && (u8[t] & mask) == prefix, static_cast<uint32_t>((u8[t] >> shift) & 255u));
                }
            }
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            // lane l owns bins 4l..4l+3; an inclusive scan of their sums locates the bin of rank k
            const int lane = threadIdx.x;
            const int h0 = hist[4 * lane], h1 = hist[4 * lane + 1], h2 = hist[4 * lane + 2], h3 = hist[4 * lane + 3];
            const int mine = h0 + h1 + h2 + h3;
            int incl = mine;
            for (int off = 1; off < 64; off <<= 1) {
                const int o = __shfl_up(incl, off, 64);
                if (lane >= off) incl += o;
            }
            const int excl = incl - mine;
            const int k = s_k;
            if (excl <= k && k < incl) {
                int kk = k - excl, b = 4 * lane;
                if (kk >= h0) { kk -= h0; ++b;
                    if (kk >= h1) { kk -= h1; ++b;
                        if (kk >= h2) { kk -= h2; ++b; } } }
                s_k = kk;
                s_prefix = prefix | (static_cast<uint64_t>(b) << shift);
            }
        }
        mask |= 0xFFull << shift;
        __syncthreads();
    }
    // the threshold is the (s_k)-th member (position order) whose key image
    // equals s_prefix: two workgroup scans of per-thread counts give every
    // member its place
    const uint64_t ustar = s_prefix;
    const int kstar = s_k;
    int neq = 0;
#pragma unroll
    for (int r = 0; r < (kReg ? R : 1); ++r)
        if constexpr (kReg) neq += (r < cnt && img(r) == ustar);
    // (without registers: the thread's run read eight keys at a time, in order)
    auto run8 = [&](auto&& body) {
        for (int r0 = 0; r0 < cnt; r0 += 8) {
            uint64_t u8[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) u8[t] = orderable(key[s0 + a0 + min(r0 + t, cnt - 1)]);
#pragma unroll
            for (int t = 0; t < 8; ++t)
                if (r0 + t < cnt) body(r0 + t, u8[t]);
        }
    };
    if constexpr (!kReg) run8([&](int, uint64_t u) { neq += u == ustar; });
    int tot = 0;
    const int eq_base = wg_scan_excl(neq, wsum, &tot);
    int nleft = 0, e = eq_base;
    auto count_left = [&](int, uint64_t u) {
        const bool eq = u == ustar;
        nleft += u < ustar || (eq && e < kstar);
        e += eq;
    };
    if constexpr (kReg) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (r < cnt) count_left(r, img(r));
    } else {
        run8(count_left);
    }
    const int l_base = wg_scan_excl(nleft, wsum, &tot);
    int li = l_base, ri = a0 - l_base;
    e = eq_base;
    auto place = [&](int r, uint64_t u) {
        const bool eq = u == ustar;
        const bool left = u < ustar || (eq && e < kstar);
        e += eq;
        out[left ? s0 + li++ : s0 + nl + ri++] = perm[s0 + a0 + r];
    };
    if constexpr (kReg) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (r < cnt) place(r, img(r));
    } else {
        run8(place);
    }
}

// ---------------------------------------------------------------------------
// neighbours
// ---------------------------------------------------------------------------
__global__ void k_knn_init(int32_t* idx, double* d2, int64_t cnt) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i < cnt) { idx[i] = -1; d2[i] = INFINITY; }
}


// All pairs inside every leaf, merged into each point's running list of the k
// smallest (d2, index).  One wave per point: the list lives across lanes 0..k-1
// (ascending), each lane evaluates a share of the leaf's candidates, and the
// candidates that beat the current k-th entry are inserted one at a time
// (duplicate check and insert position by ballot, shift by one lane); an empty
// list takes a chunk's k smallest by their ranks in the chunk.  The result is
// the unique k smallest entries, whatever the insertion order.
constexpr int kLeafStageDim = 8;
constexpr int kLeafStageMax = 2048;
constexpr int kKnnBlock = 1024;
__device__ inline bool knn_less(double da, int32_t ia, double db, int32_t ib) {
    // empty slots (index < 0) compare greater than every candidate
    if (ib < 0) return ia >= 0;
    if (ia < 0) return false;
    return da < db || (da == db && ia < ib);
}

// Wave-wide lane moves without shared memory: the value of a lane chosen by a
// wave-uniform index (readlane), and the value of the next lower lane (DPP
// wave shift right by one; lane 0 keeps its own).
__device__ inline double lane_value(double v, int src) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane(static_cast<int>(b & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), src);
    return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ inline int32_t lane_value(int32_t v, int src) { return __builtin_amdgcn_readlane(v, src); }
__device__ inline int32_t from_lower_lane(int32_t v) { return __builtin_amdgcn_update_dpp(v, v, 0x138, 0xF, 0xF, false); }
__device__ inline double from_lower_lane(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = from_lower_lane(static_cast<int32_t>(b & 0xffffffffll));
    const int hi = from_lower_lane(static_cast<int32_t>(b >> 32));
    return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

__global__ void __launch_bounds__(kKnnBlock) k_knn_leaf(int depth, const int64_t* start, const int64_t* size,
                                                        const int32_t* perm, Pts P, int k, int stage, int splits,
                                                        const int32_t* leafd2, int leafmax, int32_t* kidx,
                                                        double* kd2) {
    extern __shared__ double xs[];          // staged coordinates (n x dim) when stage != 0
    __shared__ int32_t ids[kLeafStageMax];  // staged original indices
    __shared__ double sd[kKnnBlock];        // per wave: a list placed by rank
    __shared__ int32_t sj[kKnnBlock];
    const int64_t h = (int64_t(1) << depth) + blockIdx.x / splits;
    const int part = blockIdx.x % splits;
    const int64_t s0 = start[h], n = size[h];
    for (int64_t e = threadIdx.x; e < n && e < kLeafStageMax; e += blockDim.x) ids[e] = perm[s0 + e];
    if (stage)
        for (int64_t e = threadIdx.x; e < n * P.dim; e += blockDim.x)
            xs[e] = P.xf[static_cast<int64_t>(perm[s0 + e / P.dim]) * P.dim + e % P.dim];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int64_t a = static_cast<int64_t>(part) * nw + wv; a < n; a += static_cast<int64_t>(splits) * nw) {
        const int32_t i = n <= kLeafStageMax ? ids[a] : perm[s0 + a];
        double ld = INFINITY;
        int32_t li = -1;
        if (lane < k) {
            ld = kd2[static_cast<int64_t>(i) * k + lane];
            li = kidx[static_cast<int64_t>(i) * k + lane];
        }
        for (int64_t b0 = 0; b0 < n; b0 += 64) {
            const int64_t b = b0 + lane;
            double d = INFINITY;
            int32_t j = -1;
            if (b < n && b != a) {
                j = n <= kLeafStageMax ? ids[b] : perm[s0 + b];
                if (leafd2) {
                    const int64_t lf = blockIdx.x / splits;
                    d = static_cast<double>(leafd2[(lf * leafmax + a) * leafmax + b]) / 65025.0;
                } else if (stage) {
                    const double* xa = xs + a * P.dim;
                    const double* xb = xs + b * P.dim;
                    double acc = 0.0;
                    for (int q = 0; q < P.dim; ++q) {
                        const double tq = xa[q] - xb[q];
                        acc = acc + tq * tq;
                    }
                    d = acc;
                } else {
                    d = sqd(P, i, j);
                }
            }
            if (lane_value(li, 0) < 0) {
                // an empty list takes the chunk's k smallest: each candidate's rank
                // among the chunk (a strict order: the indices differ) is its slot
                int rank = 0;
                for (int m = 0; m < 64; ++m) {
                    const double dm = lane_value(d, m);
                    const int32_t jm = lane_value(j, m);
                    rank += jm >= 0 && knn_less(dm, jm, d, j);
                }
                double* wd = sd + wv * 64;
                int32_t* wj = sj + wv * 64;
                wd[lane] = INFINITY;
                wj[lane] = -1;
                __builtin_amdgcn_wave_barrier();
                if (j >= 0 && rank < k) {
                    wd[rank] = d;
                    wj[rank] = j;
                }
                __builtin_amdgcn_wave_barrier();
                if (lane < k) {
                    ld = wd[lane];
                    li = wj[lane];
                }
                __builtin_amdgcn_wave_barrier();
                continue;
            }
            // candidates that beat the current k-th entry
            const double dk = lane_value(ld, k - 1);
            const int32_t ik = lane_value(li, k - 1);
            uint64_t pend = __ballot(j >= 0 && knn_less(d, j, dk, ik));
            while (pend) {
                const int src = __ffsll(static_cast<long long>(pend)) - 1;
                pend &= pend - 1;
                const double dc = lane_value(d, src);
                const int32_t jc = lane_value(j, src);
                const bool dup = __ballot(lane < k && li == jc) != 0;
                if (dup) continue;
                const int pos = __popcll(__ballot(lane < k && knn_less(ld, li, dc, jc)));
                if (pos >= k) continue;
                const double up_d = from_lower_lane(ld);
                const int32_t up_i = from_lower_lane(li);
                if (lane == pos) { ld = dc; li = jc; }
                else if (lane > pos && lane < k) { ld = up_d; li = up_i; }
            }
        }
        if (lane < k) {
            kd2[static_cast<int64_t>(i) * k + lane] = ld;
            kidx[static_cast<int64_t>(i) * k + lane] = li;
        }
    }
}

// ---------------------------------------------------------------------------
// interaction lists
// ---------------------------------------------------------------------------
__global__ void k_inverse_perm(const int32_t* perm, int32_t* iperm, int64_t n) {
    const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (t < n) iperm[perm[t]] = static_cast<int32_t>(t);
}

// leaf index of every tree position (one workgroup per leaf)
__global__ void k_leaf_of(int depth, const int64_t* start, const int64_t* size, int32_t* leaf_of) {
    const int64_t a = blockIdx.x, h = (int64_t(1) << depth) + a;
    for (int64_t p = start[h] + threadIdx.x; p < start[h] + size[h]; p += blockDim.x)
        leaf_of[p] = static_cast<int32_t>(a);
}

// votes[a][b] = number of (point in leaf a, neighbour in leaf b) pairs: one
// workgroup per leaf a counts its row in shared memory (L bins) and writes it;
// with kGlobal (too many leaves for shared memory) it counts straight into the
// zeroed row
template <bool kGlobal>
__global__ void k_votes(int depth, const int64_t* start, const int64_t* size, const int32_t* perm,
                        const int32_t* iperm, const int32_t* kidx, int k, const int32_t* leaf_of, int32_t* votes) {
    extern __shared__ int32_t vh[];
    const int64_t L = int64_t(1) << depth;
    const int64_t a = blockIdx.x, h = L + a;
    const int64_t s0 = start[h], cnt = size[h] * k;
    int32_t* row = kGlobal ? votes + a * L : vh;
    if (!kGlobal) {
        for (int64_t b = threadIdx.x; b < L; b += blockDim.x) vh[b] = 0;
        __syncthreads();
    }
    for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) {
        const int32_t i = perm[s0 + e / k];
        const int32_t j = kidx[static_cast<int64_t>(i) * k + e % k];
        if (j >= 0) atomicAdd(&row[leaf_of[iperm[j]]], 1);
    }
    if (!kGlobal) {
        __syncthreads();
        for (int64_t b = threadIdx.x; b < L; b += blockDim.x) votes[a * L + b] = vh[b];
    }
}

// ---------------------------------------------------------------------------
// skeletonisation
// ---------------------------------------------------------------------------
struct LevelArgs {
    int lvl, depth;
    int64_t n;
    int k, s, cmax, rmax;
    uint64_t seed;
    double tau;
    const int64_t* start;
    const int64_t* size;
    const int32_t* perm;
    const int32_t* iperm;
    const int32_t* kidx;
    const int32_t* skel_fix;    // skeletons of every node, heap id h at h * s (levels below filled)
    const int32_t* rank;        // per heap id (levels below filled)
    int32_t* cand;              // per node cmax
    int32_t* ncand;             // per node
    int32_t* cnt;               // per node n
    uint32_t* bits;             // per node ceil(n/32)
    int32_t* uniq;              // per node cmax*k: unique outside neighbours, ascending
    int32_t* vts;               // per node cmax*k: their votes (sorted row selection)
    int32_t* rows;              // per node rmax
    int32_t* nrows;             // per node
    double* B;                  // per node rmax x cmax
    int32_t* cp;                // per node cmax
    double* Pfix;               // P of every node, heap id h at h * s * cmax (rank x ncand, row-major)
    int32_t* rk;                // per heap id: rank
    int32_t* status;            // per node: 0 ok, 1 row fill failed
    int64_t lds_b;              // ID: elements of B a workgroup keeps in shared memory
    int32_t* rows_fix;          // sampled rows of every node, heap id h at h * rmax
    int32_t* nc_all;            // per heap id: candidates
    int32_t* nr_all;            // per heap id: sampled rows
    int32_t* st_all;            // per heap id: row fill status
    int node0;                  // ID launches: first node of this launch
};

// the node's candidates: its points at the leaves, else its children's skeletons
__device__ inline void node_cand(const LevelArgs& A, int64_t t) {
    const int64_t h = (int64_t(1) << A.lvl) + t;
    int32_t* c = A.cand + t * A.cmax;
    if (A.lvl == A.depth) {
        const int64_t n = A.size[h];
        for (int64_t u = threadIdx.x; u < n; u += blockDim.x) c[u] = A.perm[A.start[h] + u];
        if (threadIdx.x == 0) A.ncand[t] = static_cast<int32_t>(n);
    } else {
        const int rl = A.rank[2 * h], rr = A.rank[2 * h + 1];
        const int32_t* sl = A.skel_fix + 2 * h * A.s;
        const int32_t* sr = A.skel_fix + (2 * h + 1) * A.s;
        for (int u = threadIdx.x; u < rl + rr; u += blockDim.x) c[u] = u < rl ? sl[u] : sr[u - rl];
        if (threadIdx.x == 0) A.ncand[t] = rl + rr;
    }
}

__global__ void k_cand(LevelArgs A) { node_cand(A, blockIdx.x); }

// neighbour votes of the candidates, for points outside the node
__global__ void k_row_count(LevelArgs A) {
    const int64_t t = blockIdx.y;
    const int64_t h = (int64_t(1) << A.lvl) + t;
    const int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    const int nc = A.ncand[t];
    if (e >= static_cast<int64_t>(nc) * A.k) return;
    const int32_t j = A.cand[t * A.cmax + e / A.k];
    const int32_t i = A.kidx[static_cast<int64_t>(j) * A.k + e % A.k];
    if (i < 0) return;
    const int64_t pi = A.iperm[i];
    if (pi >= A.start[h] && pi < A.start[h] + A.size[h]) return;
    atomicAdd(&A.cnt[t * A.n + i], 1);
}

// up to half of the rows: most-voted outside neighbours (ties: lower index);
// the rest: uniform draws from outside the node (or every outside point when
// that is all there is).  The draws are taken 64 at a time by one wave and
// accepted in draw order, exactly as a sequential rejection loop would.
constexpr int kMaxRows = 2048;   // sampled rows per node (2 max_rank_s)
constexpr int kVoteShared = 144 * 1024;   // shared memory for the bitmap vote counting (bytes)

// kSorted: the candidates' outside neighbours are marked in a bitmap over the
// points in shared memory, which lists them in ascending order, and their votes
// are counted at their ranks; otherwise k_row_count has counted them into a
// dense per-node array that is scanned in index order.  Both give the same
// ascending list and votes.
template <bool kSorted>
__global__ void k_row_select(LevelArgs A) {
    __shared__ int wsum[kBlock / 64];
    __shared__ int32_t hist[kMaxCand + 1];   // votes are at most the number of candidates
    __shared__ int32_t selv[kMaxRows / 2], selc[kMaxRows / 2];
    __shared__ int32_t s_t, s_need;
    __shared__ int32_t batch[64];
    const int64_t t = blockIdx.x;
    const int64_t h = (int64_t(1) << A.lvl) + t;
    const int64_t lo = A.start[h], hi = A.start[h] + A.size[h];
    int32_t* cnt = A.cnt + t * A.n;
    int32_t* uq = A.uniq + t * static_cast<int64_t>(A.cmax) * A.k;
    int32_t* rows = A.rows + t * A.rmax;
    uint32_t* bits = A.bits + t * ((A.n + 31) / 32);
    int64_t want = A.n - A.size[h];
    if (want > 2 * static_cast<int64_t>(A.s)) want = 2 * static_cast<int64_t>(A.s);
    const int64_t want_nb = want / 2;
    // votes of the u-th unique outside neighbour (uq ascending)
    int32_t* vt = A.vts + t * static_cast<int64_t>(A.cmax) * A.k;
    auto votes = [&](int64_t u) { return kSorted ? vt[u] : cnt[uq[u]]; };
    int64_t nu = 0;
    if constexpr (kSorted) {
        // the candidates are listed here (the dense variant's vote count needs them
        // before it, from k_cand); the workgroup reads them after the barrier
        node_cand(A, t);
        __syncthreads();
        // an n-bit map of the outside neighbours, the running popcount of its
        // words, and the votes at each neighbour's rank in index order
        extern __shared__ uint32_t dsh[];
        const int nw = static_cast<int>((A.n + 31) / 32);
        uint32_t* bm = dsh;
        int32_t* pre = reinterpret_cast<int32_t*>(dsh + nw);
        int32_t* sv = pre + nw;
        const int nc = A.ncand[t];
        const int32_t* cd = A.cand + t * A.cmax;
        const int64_t ntot = static_cast<int64_t>(nc) * A.k;
        for (int w = threadIdx.x; w < nw; w += blockDim.x) bm[w] = 0u;
        for (int64_t e = threadIdx.x; e < ntot; e += blockDim.x) sv[e] = 0;
        __syncthreads();
        // the neighbours of entries e0 + kBlock q (q < 8) that lie outside the
        // node (-1 otherwise), each chain of dependent loads issued for all
        // eight entries at once
        auto outside8 = [&](int64_t e0, int32_t* o) {
            int32_t c[8], i[8];
            int64_t pi[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int64_t e = min(e0 + q * kBlock, ntot - 1);
                c[q] = cd[e / A.k];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int64_t e = min(e0 + q * kBlock, ntot - 1);
                i[q] = A.kidx[static_cast<int64_t>(c[q]) * A.k + e % A.k];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) pi[q] = A.iperm[max(i[q], 0)];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                o[q] = (e0 + q * kBlock >= ntot || i[q] < 0 || (pi[q] >= lo && pi[q] < hi)) ? -1 : i[q];
        };
        for (int64_t e0 = threadIdx.x; e0 < ntot; e0 += 8 * kBlock) {
            int32_t o[8];
            outside8(e0, o);
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (o[q] >= 0) atomicOr(&bm[o[q] >> 5], 1u << (o[q] & 31));
        }
        __syncthreads();
        // words in contiguous ranges per thread: exclusive popcount prefix, then
        // the set bits in ascending order
        const int per = (nw + kBlock - 1) / kBlock;
        const int w0 = min(nw, static_cast<int>(threadIdx.x) * per), w1 = min(nw, w0 + per);
        int mine = 0;
        for (int w = w0; w < w1; ++w) mine += __popc(bm[w]);
        int tot = 0;
        int r = wg_scan_excl(mine, wsum, &tot);
        for (int w = w0; w < w1; ++w) {
            pre[w] = r;
            uint32_t m = bm[w];
            while (m) {
                const int bit = __ffs(m) - 1;
                m &= m - 1;
                uq[r++] = w * 32 + bit;
            }
        }
        nu = tot;
        __syncthreads();
        for (int64_t e0 = threadIdx.x; e0 < ntot; e0 += 8 * kBlock) {
            int32_t o[8];
            outside8(e0, o);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int32_t i = o[q];
                if (i >= 0) atomicAdd(&sv[pre[i >> 5] + __popc(bm[i >> 5] & ((1u << (i & 31)) - 1u))], 1);
            }
        }
        __syncthreads();
        for (int64_t u = threadIdx.x; u < nu; u += blockDim.x) vt[u] = sv[u];
        __syncthreads();
    } else {
        // compaction of {i : cnt[i] > 0} in index order: a contiguous range per
        // thread, one workgroup scan of the per-thread counts
        const int64_t per = (A.n + kBlock - 1) / kBlock;
        const int64_t i0 = min(A.n, static_cast<int64_t>(threadIdx.x) * per), i1 = min(A.n, i0 + per);
        int mine = 0;
        for (int64_t i = i0; i < i1; i += 16) {   // 16 loads in flight
            int32_t v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = cnt[min(i + u, i1 - 1)];   // clamped: unguarded loads
#pragma unroll
            for (int u = 0; u < 16; ++u) mine += (i + u < i1) && v[u] > 0;
        }
        int tot = 0;
        int w = wg_scan_excl(mine, wsum, &tot);
        for (int64_t i = i0; i < i1; i += 16) {
            int32_t v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = cnt[min(i + u, i1 - 1)];
#pragma unroll
            for (int u = 0; u < 16; ++u)
                if (i + u < i1 && v[u] > 0) uq[w++] = static_cast<int32_t>(i + u);
        }
        nu = tot;
    }
    for (int c = threadIdx.x; c <= kMaxCand; c += blockDim.x) hist[c] = 0;
    __syncthreads();
    // rank by (votes desc, index asc) and keep the first want_nb: the vote
    // threshold from a histogram, the ties at it in index order, then the
    // (at most want_nb) kept entries ordered among themselves
    for (int64_t u = threadIdx.x; u < nu; u += blockDim.x) atomicAdd(&hist[min(votes(u), kMaxCand)], 1);
    __syncthreads();
    // the threshold: the highest vote count c at which the entries with at least
    // c votes reach want_nb.  Thread t owns the kBins bins kMaxCand - kBins t
    // downwards; an exclusive scan gives the entries above its range.
    {
        constexpr int kBins = kMaxCand / kBlock;
        static_assert(kBins * kBlock == kMaxCand, "bins per thread");
        const int top = kMaxCand - kBins * static_cast<int>(threadIdx.x);
        int mine = 0;
        for (int c = top; c > top - kBins; --c) mine += hist[c];
        int tot = 0;
        int64_t above = wg_scan_excl(mine, wsum, &tot);
        if (threadIdx.x == 0) {
            s_t = 0;        // 0: every entry is kept
            s_need = 0;
        }
        __syncthreads();
        if (nu > want_nb && above < want_nb && above + mine >= want_nb)
            for (int c = top; c > top - kBins; --c) {
                if (above + hist[c] >= want_nb) {
                    s_t = c;
                    s_need = static_cast<int>(want_nb - above);
                    break;
                }
                above += hist[c];
            }
    }
    __syncthreads();
    const int tcut = s_t, need = s_need;
    int64_t m = 0;   // kept entries, collected in index order
    {
        const int64_t per = (nu + kBlock - 1) / kBlock;
        const int64_t u0 = min(nu, static_cast<int64_t>(threadIdx.x) * per), u1 = min(nu, u0 + per);
        int ties = 0;
        for (int64_t u = u0; u < u1; u += 16) {   // batched loads (clamped addresses)
            int32_t v[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = votes(min(u + q, u1 - 1));
#pragma unroll
            for (int q = 0; q < 16; ++q) ties += (u + q < u1) && v[q] == tcut;
        }
        int tt = 0;
        int tie_rank = wg_scan_excl(ties, wsum, &tt);
        int keep = 0;
        for (int64_t u = u0; u < u1; ++u) {
            const int32_t c = votes(u);
            keep += c > tcut || (c == tcut && tie_rank++ < need);
        }
        int tk = 0;
        int w = wg_scan_excl(keep, wsum, &tk);
        tie_rank -= ties;   // back to this thread's first tie rank
        for (int64_t u = u0; u < u1; ++u) {
            const int32_t c = votes(u);
            if (c > tcut || (c == tcut && tie_rank++ < need)) {
                selv[w] = uq[u];
                selc[w] = c;
                ++w;
            }
        }
        m = tk;
    }
    __syncthreads();
    for (int64_t e = threadIdx.x; e < m; e += blockDim.x) {
        const int32_t iu = selv[e], cu = selc[e];
        int64_t r = 0;
        for (int64_t v = 0; v < m; ++v) r += (selc[v] > cu) || (selc[v] == cu && v < e);
        rows[r] = iu;
        atomicOr(&bits[iu >> 5], 1u << (iu & 31));
    }
    __syncthreads();
    int64_t nr = nu < want_nb ? nu : want_nb;
    int32_t st = 0;
    if (nr < want && want == A.n - A.size[h]) {
        // every outside point not chosen yet, ascending index
        for (int64_t base = 0; base < A.n; base += blockDim.x) {
            const int64_t i = base + threadIdx.x;
            bool f = false;
            if (i < A.n) {
                const int64_t pi = A.iperm[i];
                f = !(pi >= lo && pi < hi) && !(bits[i >> 5] & (1u << (i & 31)));
            }
            int tot = 0;
            const int pre = wg_flag_scan(f, wsum, &tot);
            if (f && nr + pre < want) rows[nr + pre] = static_cast<int32_t>(i);
            nr = min<int64_t>(want, nr + tot);
        }
    } else if (nr < want && threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const uint64_t cap = 64ull * static_cast<uint64_t>(A.n) + 1024ull;
        uint64_t d = 0;
        while (nr < want) {
            if (d > cap) { st = 1; break; }
            const int32_t c = static_cast<int32_t>(below(
                philox_draw(A.seed, kRowFill, static_cast<uint32_t>(h), 0, static_cast<uint32_t>(d + lane)),
                static_cast<uint32_t>(A.n)));
            const int64_t pc = A.iperm[c];
            const bool valid = !(pc >= lo && pc < hi) && !(bits[c >> 5] & (1u << (c & 31)));
            batch[lane] = valid ? c : -1;
            __builtin_amdgcn_wave_barrier();
            bool dup = false;   // an earlier draw of this batch has the same point
#pragma unroll
            for (int l = 0; l < 64; ++l) dup = dup || (l < lane && batch[l] == c);
            const bool acc = valid && !dup;
            const uint64_t bal = __ballot(acc);
            const int pre = __popcll(bal & ((1ull << lane) - 1ull));
            if (acc && nr + pre < want) {
                rows[nr + pre] = c;
                atomicOr(&bits[c >> 5], 1u << (c & 31));
            }
            nr = min<int64_t>(want, nr + __popcll(bal));
            d += 64;
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (threadIdx.x == 0) {
        A.nrows[t] = static_cast<int32_t>(nr);
        A.status[t] = st;
    }
    // leave the node's bitmap clear for the next level (which uses a prefix of
    // these node slots)
    __syncthreads();
    for (int64_t w = threadIdx.x; w < (A.n + 31) / 32; w += blockDim.x) bits[w] = 0u;
}

// B = K(rows, cand) for float64 points of at most kDimReg coordinates: a thread
// keeps one candidate point in registers and walks a slice of the rows (the
// same row point for every thread at a time); the same operations in the same
// order as kval(P, row, candidate)
constexpr int kDimReg = 16;
constexpr int kBlockSlices = 4;   // row slices (workgroups) per node
__global__ void k_block_reg(LevelArgs A, Pts P) {
    const int64_t t = blockIdx.y;
    const int nc = A.ncand[t], nr = A.nrows[t];
    const int per = (nr + kBlockSlices - 1) / kBlockSlices;
    const int r0 = static_cast<int>(blockIdx.x) * per, r1 = min(nr, r0 + per);
    double* B = A.B + t * static_cast<int64_t>(A.rmax) * A.cmax;
    const int32_t* rows = A.rows + t * A.rmax;
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        const double* xj = P.xf + static_cast<int64_t>(A.cand[t * A.cmax + c]) * P.dim;
        double xc[kDimReg];
#pragma unroll
        for (int d = 0; d < kDimReg; ++d) xc[d] = d < P.dim ? xj[d] : 0.0;
        for (int r = r0; r < r1; ++r) {
            const double* xi = P.xf + static_cast<int64_t>(rows[r]) * P.dim;
            double acc = 0.0;
#pragma unroll
            for (int d = 0; d < kDimReg; ++d)
                if (d < P.dim) {
                    const double tq = xi[d] - xc[d];
                    acc = acc + tq * tq;
                }
            B[static_cast<int64_t>(r) * nc + c] = det_exp(-(acc / P.eps));
        }
    }
}

// B = K(rows, cand), row-major with leading dimension ncand
__global__ void k_block(LevelArgs A, Pts P) {
    const int64_t t = blockIdx.y;
    const int nc = A.ncand[t], nr = A.nrows[t];
    const int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (e >= static_cast<int64_t>(nr) * nc) return;
    const int r = static_cast<int>(e / nc), c = static_cast<int>(e % nc);
    A.B[t * static_cast<int64_t>(A.rmax) * A.cmax + e] = kval(P, A.rows[t * A.rmax + r], A.cand[t * A.cmax + c]);
}

// ---- interpolative decomposition --------------------------------------------
// Every column norm, reflector norm and reflector-column inner product of the
// ID is a sum over rows [i0, i1) taken in one fixed order: the term of row i
// goes to partial sum (i - i0) mod 8 in increasing i, and the partials combine
// as ((p0 + p1) + (p2 + p3)) + ((p4 + p5) + (p6 + p7)).  The eight chains are
// independent, so up to eight lanes share one column.

// The rows of a node's block B (nr x nc, row-major) below R are kept in shared
// memory (sB, odd leading dimension ldS against bank conflicts), the rest stay
// in global memory (gB, leading dimension nc).
typedef __attribute__((address_space(3))) double lds_f64;   // a float64 in shared memory

// B of one node: rows [T0, T0 + R) = [T0, nr) staged in shared memory (the
// trailing rows, which every reflector touches), the leading rows in global
// memory.
struct QrBlock {
    lds_f64* sB;
    double* gB;
    int nc, ldS, R, T0;
    __device__ double ld(int i, int c) const {
        return i >= T0 ? sB[(i - T0) * ldS + c] : gB[static_cast<int64_t>(i) * nc + c];
    }
    __device__ void st(int i, int c, double x) const {
        if (i >= T0) sB[(i - T0) * ldS + c] = x;
        else gB[static_cast<int64_t>(i) * nc + c] = x;
    }
};

// Rows [i0, i1) of column c, shared by the L lanes of a lane group (L = 1, 2,
// 4 or 8 consecutive lanes of one wave).  Row i has phase (i - i0) mod 8; lane
// `lane` owns phases lane + L m (m < 8 / L) and visits its rows in increasing
// order, in batches whose loads are all issued first.  body(m, i, x) sees the
// phase slot m as a compile-time constant; with kWrite the modified x is stored.
template <int L, bool kWrite, typename Body>
__device__ inline void group_rows(const QrBlock& Q, int lane, int c, int i0, int i1, Body&& body) {
    constexpr int PH = 8 / L, KB = L == 1 ? 2 : 8 / PH, SPAN = 8 * KB;   // 16 or 8 loads per lane and batch
    int i = i0;
    const int gl = min(Q.T0, i1);
    for (; i + SPAN <= gl; i += SPAN) {   // rows in global memory (i < T0)
        double x[KB][PH];
#pragma unroll
        for (int k = 0; k < KB; ++k)
#pragma unroll
            for (int m = 0; m < PH; ++m) x[k][m] = Q.gB[static_cast<int64_t>(i + 8 * k + lane + L * m) * Q.nc + c];
#pragma unroll
        for (int k = 0; k < KB; ++k)
#pragma unroll
            for (int m = 0; m < PH; ++m) {
                const int r = i + 8 * k + lane + L * m;
                body(m, r, x[k][m]);
                if (kWrite) Q.gB[static_cast<int64_t>(r) * Q.nc + c] = x[k][m];
            }
    }
    if (i < Q.T0 && i + SPAN <= i1) {   // the batch across T0
        double x[KB][PH];
#pragma unroll
        for (int k = 0; k < KB; ++k)
#pragma unroll
            for (int m = 0; m < PH; ++m) x[k][m] = Q.ld(i + 8 * k + lane + L * m, c);
#pragma unroll
        for (int k = 0; k < KB; ++k)
#pragma unroll
            for (int m = 0; m < PH; ++m) {
                const int r = i + 8 * k + lane + L * m;
                body(m, r, x[k][m]);
                if (kWrite) Q.st(r, c, x[k][m]);
            }
        i += SPAN;
    }
    for (; i + SPAN <= i1; i += SPAN) {   // rows in shared memory (i >= T0)
        double x[KB][PH];
#pragma unroll
        for (int k = 0; k < KB; ++k)
#pragma unroll
            for (int m = 0; m < PH; ++m) x[k][m] = Q.sB[(i - Q.T0 + 8 * k + lane + L * m) * Q.ldS + c];
#pragma unroll
        for (int k = 0; k < KB; ++k)
#pragma unroll
            for (int m = 0; m < PH; ++m) {
                const int r = i + 8 * k + lane + L * m;
                body(m, r, x[k][m]);
                if (kWrite) Q.sB[(r - Q.T0) * Q.ldS + c] = x[k][m];
            }
    }
    if (i < i1) {   // last partial batch; (i - i0) is a multiple of 8 here
        double x[KB][PH];
#pragma unroll
        for (int k = 0; k < KB; ++k)
#pragma unroll
            for (int m = 0; m < PH; ++m) {
                const int r = i + 8 * k + lane + L * m;
                x[k][m] = r < i1 ? Q.ld(r, c) : 0.0;
            }
#pragma unroll
        for (int k = 0; k < KB; ++k)
#pragma unroll
            for (int m = 0; m < PH; ++m) {
                const int r = i + 8 * k + lane + L * m;
                if (r < i1) {
                    body(m, r, x[k][m]);
                    if (kWrite) Q.st(r, c, x[k][m]);
                }
            }
    }
}

// The eight phase sums of a lane group, combined as
// ((p0 + p1) + (p2 + p3)) + ((p4 + p5) + (p6 + p7)); every lane of the group
// gets the total.  Lane l holds phases l + L m in p[m].  The shuffles add the
// partner lane's partial first (lanes l and l ^ d hold phases that are
// siblings in the tree), then the lane adds its own slots pairwise.
template <int L>
__device__ inline double group_total(double* p) {
    constexpr int PH = 8 / L;
#pragma unroll
    for (int d = 1; d < L; d <<= 1)
#pragma unroll
        for (int m = 0; m < PH; ++m) p[m] = p[m] + __shfl_xor(p[m], d, kWave);
    if (PH == 1) return p[0];
    if (PH == 2) return p[0] + p[1];
    if (PH == 4) return (p[0] + p[1]) + (p[2] + p[3]);
    return ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
}

// squared norms over rows [0, nr) of every column, L lanes per column
template <int L, int NT>
__device__ inline void id_norms(const QrBlock& Q, double* nsq, int nr, int nc) {
    constexpr int PH = 8 / L;
    const int lane = threadIdx.x % L;
    for (int c = threadIdx.x / L; c < nc; c += NT / L) {
        double p[PH];
#pragma unroll
        for (int m = 0; m < PH; ++m) p[m] = 0.0;
        group_rows<L, false>(Q, lane, c, 0, nr, [&](int m, int, double& x) { p[m] = p[m] + x * x; });
        const double t = group_total<L>(p);
        if (lane == 0) nsq[c] = t;
    }
}

// Apply the reflector (hv, rows [j, nr), hv^T hv = vtv) to the columns after j,
// L lanes per column, and leave their squared norms over rows [j + 1, nr) in
// nsq.  A column's lanes are in one wave and its dot product is complete (the
// shuffles consume every lane's loads) before any of its rows is stored.
template <int L, int NT>
__device__ inline void id_reflect(const QrBlock& Q, const double* hv, double* nsq, int j, int nr, int nc,
                                  double vtv) {
    constexpr int PH = 8 / L;
    const int lane = threadIdx.x % L;
    for (int c = j + 1 + threadIdx.x / L; c < nc; c += NT / L) {
        double p[PH];
#pragma unroll
        for (int m = 0; m < PH; ++m) p[m] = 0.0;
        double xj = 0.0;   // the pivot row's entry, seen by lane 0 (phase 0)
        group_rows<L, false>(Q, lane, c, j, nr, [&](int m, int i, double& x) {
            p[m] = p[m] + hv[i] * x;
            if (i == j) xj = x;
        });
        const double f = (2.0 * group_total<L>(p)) / vtv;
        // the pivot row first (its square is not part of the next norm), then the rest
        if (lane == 0) Q.st(j, c, xj - f * hv[j]);
#pragma unroll
        for (int m = 0; m < PH; ++m) p[m] = 0.0;
        group_rows<L, true>(Q, lane, c, j + 1, nr, [&](int m, int i, double& x) {
            x = x - f * hv[i];
            p[m] = p[m] + x * x;
        });
        const double t = group_total<L>(p);
        if (lane == 0) nsq[c] = t;
    }
}

// The reflector of step j formed and applied with each column's rows [j, nr)
// in registers, once every active row is staged in shared memory (j >= T0):
// every lane group builds hv from column j and its own v^T v.  The 8 lanes of a
// group share a column, lane l holding rows j + l + 8u (u < NPL), which it
// reads once and writes once; a group takes NCOL columns at a time (kBlock / 8
// apart) so that their dependent sums interleave.  The dot product's phase l
// sits on lane l (the order of group_total<8>).  The next norm is over rows
// [j + 1, nr), whose phase k = (i - j - 1) mod 8 sits on lane (k + 1) mod 8,
// so the partials move one lane down before the same combination.  A row slot
// past the end reads and writes the zero row kept after the staged rows, and a
// column slot past nc the zero padding column: their terms are exact zeros (a
// sum that starts at +0 is never -0, so adding +-0 leaves it unchanged, and
// 0 - f * 0 stores +0 back).
template <int NPL, int NCOL>
__device__ inline void id_reflect_regs(const QrBlock& Q, double* nsq, int j, int nr, int nc, double v0) {
    constexpr int kGroups = kBlock / 8;
    const int l = threadIdx.x % 8;
    const int gbase = (threadIdx.x % kWave) & ~7;
    const int first = (j + l - Q.T0) * Q.ldS;   // staged offset of the lane's first row (column 0)
    const int step = 8 * Q.ldS;
    const int zrow = Q.R * Q.ldS;                 // the zero row (logical row nr)
    // hv = column j below row j with v0 = x0 - alpha in row j, and v^T v
    // summed by the same phases (lane l: rows j + l + 8u)
    double hreg[NPL];
#pragma unroll
    for (int u = 0; u < NPL; ++u) hreg[u] = Q.sB[min(first + u * step, zrow) + j];
    if (l == 0) hreg[0] = v0;
    double pv = 0.0;
#pragma unroll
    for (int u = 0; u < NPL; ++u) pv = pv + hreg[u] * hreg[u];
    const double vtv = group_total<8>(&pv);
    for (int c0 = j + 1 + threadIdx.x / 8; c0 < nc; c0 += NCOL * kGroups) {
        int lim = zrow;
        asm volatile("" : "+v"(lim));   // row offsets clamped per column, not held in registers
        int cc[NCOL];
#pragma unroll
        for (int v = 0; v < NCOL; ++v) cc[v] = min(c0 + v * kGroups, nc);   // nc: the zero column
        double x[NCOL][NPL];
#pragma unroll
        for (int u = 0; u < NPL; ++u)
#pragma unroll
            for (int v = 0; v < NCOL; ++v) x[v][u] = Q.sB[min(first + u * step, lim) + cc[v]];
        double p[NCOL];
#pragma unroll
        for (int v = 0; v < NCOL; ++v) p[v] = 0.0;
#pragma unroll
        for (int u = 0; u < NPL; ++u)
#pragma unroll
            for (int v = 0; v < NCOL; ++v) p[v] = p[v] + hreg[u] * x[v][u];
        double f[NCOL], q[NCOL];
#pragma unroll
        for (int v = 0; v < NCOL; ++v) f[v] = (2.0 * group_total<8>(&p[v])) / vtv;
#pragma unroll
        for (int u = 0; u < NPL; ++u) {
            const int off = min(first + u * step, lim);
#pragma unroll
            for (int v = 0; v < NCOL; ++v) {
                const double xu = x[v][u] - f[v] * hreg[u];
                if (u == 0) q[v] = l > 0 ? xu * xu : 0.0;   // row j is not part of the next norm
                else q[v] = q[v] + xu * xu;
                Q.sB[off + cc[v]] = xu;
            }
        }
#pragma unroll
        for (int v = 0; v < NCOL; ++v) {
            double r = __shfl(q[v], gbase + ((l + 1) & 7), kWave);   // phase l of the norm
            const double t = group_total<8>(&r);
            if (l == 0 && c0 + v * kGroups < nc) nsq[c0 + v * kGroups] = t;
        }
    }
}

// Columns c >= rank of P = R11^-1 R12 by back substitution, one thread per
// column, each entry a sequential sum in q: acc = R[i][c] - sum_q R[i][q] X[q].
// With kLds the solution column is kept in the last rank staged rows (rows
// [nr - rank, nr), free once nr >= 2 rank) and copied to P at the end;
// otherwise it is built in P directly.
template <bool kLds>
__device__ inline void id_back_subst(const QrBlock& Q, double* Pm, const int32_t* cp, int rank, int nc) {
    const int x0 = Q.R - rank;   // staged slot of X[0]
    for (int c = rank + threadIdx.x; c < nc; c += blockDim.x) {
        const int pc = cp[c];
        auto xld = [&](int q) -> double {
            if constexpr (kLds) return Q.sB[(x0 + q) * Q.ldS + c];
            else return Pm[static_cast<int64_t>(q) * nc + pc];
        };
        auto xst = [&](int q, double v) {
            if constexpr (kLds) Q.sB[(x0 + q) * Q.ldS + c] = v;
            else Pm[static_cast<int64_t>(q) * nc + pc] = v;
        };
        for (int i = rank - 1; i >= 0; --i) {
            double acc = Q.ld(i, c);
            int q = i + 1;
            for (; q + 8 <= rank; q += 8) {
                double a[8], b[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    a[k] = Q.ld(i, q + k);
                    b[k] = xld(q + k);
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) acc = acc - a[k] * b[k];
            }
            for (; q < rank; ++q) acc = acc - Q.ld(i, q) * xld(q);
            xst(i, acc / Q.ld(i, i));
        }
        if (kLds)
            for (int i = 0; i < rank; ++i) Pm[static_cast<int64_t>(i) * nc + pc] = xld(i);
    }
}

// lanes per column for k remaining columns: as many as keep the workgroup's NT threads busy
template <int NT>
__device__ inline int id_lanes(int k) { return k * 8 <= NT ? 8 : k * 4 <= NT ? 4 : k * 2 <= NT ? 2 : 1; }

// workgroup argmax of (v, column) with ties to the lower column; every thread gets the result
template <int NT>
__device__ inline void wg_argmax(double& v, int& c, double* sv, int* sc) {
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const double ov = __shfl_xor(v, off, kWave);
        const int oc = __shfl_xor(c, off, kWave);
        if (ov > v || (ov == v && oc < c)) { v = ov; c = oc; }
    }
    const int w = threadIdx.x / kWave;
    if (threadIdx.x % kWave == 0) { sv[w] = v; sc[w] = c; }
    __syncthreads();
    v = sv[0];
    c = sc[0];
    for (int k = 1; k < NT / kWave; ++k)
        if (sv[k] > v || (sv[k] == v && sc[k] < c)) { v = sv[k]; c = sc[k]; }
    __syncthreads();
}

// rows x nc values from global memory (row stride nc) into staged rows
// (stride ldS), eight loads in flight per thread
template <int NT>
__device__ inline void stage_rows(lds_f64* dst, int ldS, const double* src, int nc, int rows) {
    const int n = rows * nc;
    for (int e0 = threadIdx.x; e0 < n; e0 += 8 * NT) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int e = e0 + k * NT;
            v[k] = e < n ? src[e] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int e = e0 + k * NT;
            if (e < n) dst[(e / nc) * ldS + e % nc] = v[k];
        }
    }
}

// Levels that sample more than kIdWideRows rows run the ID in workgroups of
// kIdWide threads.  The register path of the 256-thread kernel (nodes of at most
// 256 rows, once their rows are staged) does not fit the wider workgroup's
// registers, so the wide kernel leaves it out; both paths and both sizes sum in
// the same phase order, so the result does not depend on the choice.  Measured
// at N = 100000 (s = 256): 16.2 -> 15.2 ms per compression (1024 threads: 17.6,
// with register spills); MNIST-shaped N = 65536: 217 -> 195 ms.
constexpr int kIdWide = 512;
constexpr int kIdWideRows = 256;
// leaves per ID launch (with 512-thread workgroups at N = 100000, 256 leaves:
// 128 per launch 15.2 ms per compression, 256 14.8)
constexpr int kIdNodes = 256;

// Householder QR with column pivoting of B (nr x nc) and the interpolation
// matrix P = [I, R11^-1 R12] in candidate order.  One workgroup per node, one
// thread per column for the column sums (each a fixed-order sum, see above).
// The trailing rows of B are staged in shared memory (as many as fit, A.lds_b
// elements); the squared norms that choose the next pivot are accumulated
// while the reflector is applied.
template <int NT>
__global__ void __launch_bounds__(NT) k_pivoted_id(LevelArgs A) {
    extern __shared__ double dyn[];
    __shared__ double sv[NT / kWave];
    __shared__ int sc[NT / kWave];
    __shared__ double s_vtv, s_alpha;
    const int64_t t = A.node0 + blockIdx.x;
    const int nc = A.ncand[t], nr = A.nrows[t];
    double* hv = dyn;                 // Householder vector (A.rmax)
    double* nsq = dyn + A.rmax;       // remaining squared column norms (A.cmax)
    QrBlock Q;
    Q.sB = (lds_f64*)(nsq + A.cmax);   // address-space cast: dyn is shared memory
    Q.gB = A.B + t * static_cast<int64_t>(A.rmax) * A.cmax;
    Q.nc = nc;
    Q.ldS = (nc + 1) | 1;   // at least one padding column, kept zero
    // staged rows, then one zero row
    Q.R = nc > 0 ? max(0, min(nr, static_cast<int>(A.lds_b / Q.ldS) - 1)) : 0;
    Q.T0 = nr - Q.R;
    int32_t* cp = A.cp + t * A.cmax;
    const int64_t h = (int64_t(1) << A.lvl) + t;
    double* Pm = A.Pfix + h * A.s * A.cmax;
    stage_rows<NT>(Q.sB, Q.ldS, Q.gB + static_cast<int64_t>(Q.T0) * nc, nc, Q.R);
    if (nc > 0) {
        // the padding columns of every staged row and the whole zero row
        const int pad = Q.ldS - nc;
        for (int e = threadIdx.x; e < Q.R * pad; e += blockDim.x) Q.sB[(e / pad) * Q.ldS + nc + e % pad] = 0.0;
        for (int c = threadIdx.x; c < Q.ldS; c += blockDim.x) Q.sB[Q.R * Q.ldS + c] = 0.0;
    }
    for (int c = threadIdx.x; c < nc; c += blockDim.x) cp[c] = c;
    __syncthreads();
    switch (id_lanes<NT>(nc)) {
        case 8: id_norms<8, NT>(Q, nsq, nr, nc); break;
        case 4: id_norms<4, NT>(Q, nsq, nr, nc); break;
        case 2: id_norms<2, NT>(Q, nsq, nr, nc); break;
        default: id_norms<1, NT>(Q, nsq, nr, nc); break;
    }
    int kmax = nr < nc ? nr : nc;
    if (kmax > A.s) kmax = A.s;
    int rank = 0;
    double r11 = 0.0;
    __syncthreads();
    for (int j = 0; j < kmax; ++j) {
        // pivot: largest remaining column norm (ties: lowest column)
        double best = -1.0;
        int bc = INT32_MAX;
        for (int c = j + threadIdx.x; c < nc; c += blockDim.x) {
            const double nrm = sqrt(nsq[c]);
            if (nrm > best || (nrm == best && c < bc)) { best = nrm; bc = c; }
        }
        wg_argmax<NT>(best, bc, sv, sc);
        const int piv = (bc >= j && bc < nc) ? bc : j;
        if (piv != j) {
            for (int i = threadIdx.x; i < nr; i += blockDim.x) {
                const double x = Q.ld(i, j);
                Q.st(i, j, Q.ld(i, piv));
                Q.st(i, piv, x);
            }
            if (threadIdx.x == 0) {
                const int32_t x = cp[j]; cp[j] = cp[piv]; cp[piv] = x;
                const double y = nsq[j]; nsq[j] = nsq[piv]; nsq[piv] = y;
            }
            __syncthreads();
        }
        if (j == 0) r11 = best;
        if (!(best > A.tau * r11)) break;   // uniform: every thread holds the same best and r11
        if (NT == kBlock && j >= Q.T0 && nr <= 8 * 32) {
            // rows [j, nr) all staged: the reflector lives in registers
            const double x0 = Q.sB[(j - Q.T0) * Q.ldS + j];
            const double alpha = x0 >= 0.0 ? -best : best;
            id_reflect_regs<32, 1>(Q, nsq, j, nr, nc, x0 - alpha);
            __syncthreads();
            for (int i = j + threadIdx.x; i < nr; i += blockDim.x) Q.sB[(i - Q.T0) * Q.ldS + j] = (i == j) ? alpha : 0.0;
            rank = j + 1;
            __syncthreads();
            continue;
        }
        for (int i = j + threadIdx.x; i < nr; i += blockDim.x) hv[i] = Q.ld(i, j);
        __syncthreads();
        if (threadIdx.x < 8) {
            // v = x - alpha e_j; v^T v by phases: lane u sums rows j + u, j + u + 8, ...
            const int u = threadIdx.x;
            const double x0 = hv[j];
            const double alpha = x0 >= 0.0 ? -best : best;
            double acc = 0.0;
            int i = j + u;
            for (; i + 56 < nr; i += 64) {
                double v[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) v[k] = hv[i + 8 * k];
                if (i == j) v[0] = x0 - alpha;
#pragma unroll
                for (int k = 0; k < 8; ++k) acc = acc + v[k] * v[k];
            }
            for (; i < nr; i += 8) {
                const double vi = i == j ? x0 - alpha : hv[i];
                acc = acc + vi * vi;
            }
            // ((p0 + p1) + (p2 + p3)) + ((p4 + p5) + (p6 + p7)) across lanes 0..7
            acc = acc + __shfl_xor(acc, 1, 8);
            acc = acc + __shfl_xor(acc, 2, 8);
            acc = acc + __shfl_xor(acc, 4, 8);
            if (u == 0) {
                s_vtv = acc;
                s_alpha = alpha;
                hv[j] = x0 - alpha;
            }
        }
        __syncthreads();
        const double vtv = s_vtv;
        switch (id_lanes<NT>(nc - j - 1)) {
            case 8: id_reflect<8, NT>(Q, hv, nsq, j, nr, nc, vtv); break;
            case 4: id_reflect<4, NT>(Q, hv, nsq, j, nr, nc, vtv); break;
            case 2: id_reflect<2, NT>(Q, hv, nsq, j, nr, nc, vtv); break;
            default: id_reflect<1, NT>(Q, hv, nsq, j, nr, nc, vtv); break;
        }
        __syncthreads();
        for (int i = j + threadIdx.x; i < nr; i += blockDim.x) Q.st(i, j, (i == j) ? s_alpha : 0.0);
        rank = j + 1;
        __syncthreads();
    }
    __syncthreads();
    // P[:, cp[j]] = e_j for j < rank; P[:, cp[c]] = R11^-1 R12[:, c] (back substitution)
    for (int64_t e = threadIdx.x; e < static_cast<int64_t>(rank) * nc; e += blockDim.x) Pm[e] = 0.0;
    __syncthreads();
    for (int j = threadIdx.x; j < rank; j += blockDim.x) Pm[static_cast<int64_t>(j) * nc + cp[j]] = 1.0;
    if (Q.T0 >= rank && 2 * rank <= Q.R) {
        // the rows of R are all in global memory and the staged rows are free
        // (they hold rows >= T0 >= rank): stage R at the front for the solve
        stage_rows<NT>(Q.sB, Q.ldS, Q.gB, nc, rank);
        Q.T0 = 0;
        __syncthreads();
    }
    if (rank <= Q.R && 2 * rank <= nr) id_back_subst<true>(Q, Pm, cp, rank, nc);
    else id_back_subst<false>(Q, Pm, cp, rank, nc);
    // this level's skeletons, sampled rows and sizes into the per-node slots
    int32_t* skel_save = const_cast<int32_t*>(A.skel_fix) + h * A.s;
    for (int u = threadIdx.x; u < rank; u += blockDim.x) skel_save[u] = A.cand[t * A.cmax + cp[u]];
    for (int u = threadIdx.x; u < nr; u += blockDim.x) A.rows_fix[h * A.rmax + u] = A.rows[t * A.rmax + u];
    if (threadIdx.x == 0) {
        A.rk[h] = rank;
        A.nc_all[h] = nc;
        A.nr_all[h] = nr;
        A.st_all[h] = A.status[t];
    }
}

// move every node's skeletons, P and rows into the compact operator arrays
__global__ void k_compact(const int32_t* skel_fix, const int32_t* rows_fix, const double* Pfix, const int32_t* rank,
                          const int32_t* nc_all, const int32_t* nr_all, const int64_t* skoff, const int64_t* poff,
                          const int64_t* rowoff, int s, int cmax, int rmax, int32_t* skel_out, double* P_out,
                          int32_t* rows_out) {
    const int64_t h = 2 + blockIdx.x;
    const int rk = rank[h], nc = nc_all[h], nr = nr_all[h];
    for (int u = threadIdx.x; u < rk; u += blockDim.x) skel_out[skoff[h] + u] = skel_fix[h * s + u];
    const double* src = Pfix + h * s * cmax;
    for (int64_t e = threadIdx.x; e < static_cast<int64_t>(rk) * nc; e += blockDim.x) P_out[poff[h] + e] = src[e];
    for (int u = threadIdx.x; u < nr; u += blockDim.x) rows_out[rowoff[h] + u] = rows_fix[h * rmax + u];
}

// ---------------------------------------------------------------------------
// kernel tiles
// ---------------------------------------------------------------------------
struct NearPair {
    int64_t off;       // element offset of the tile (column-major, leading dim ld)
    int32_t ld, a0, na, b0, nb, pad;   // a0/b0: tree positions of row 0 / column 0
};

// float64 near tiles; with out32 also their float32 copy (the unscaled
// round-to-nearest conversion of the evaluation tiles, written at the same offsets)
// (a tile has at most 2048 x 2048 entries, so its element index fits 32 bits)
__global__ void k_near_tiles(const NearPair* pairs, const int32_t* perm, Pts P, double* out, float* out32) {
    const NearPair pr = pairs[blockIdx.y];
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= static_cast<uint32_t>(pr.ld) * static_cast<uint32_t>(pr.nb)) return;
    const int i = static_cast<int>(e % static_cast<uint32_t>(pr.ld)), j = static_cast<int>(e / static_cast<uint32_t>(pr.ld));
    const double v = i < pr.na ? kval(P, perm[pr.a0 + i], perm[pr.b0 + j]) : 0.0;
    if (out) out[pr.off + e] = v;
    if (out32) out32[pr.off + e] = static_cast<float>(v);
}

// ---------------------------------------------------------------------------
// Near tiles written directly in the evaluation precision (float64 points of at
// most kDimReg coordinates): no float64 copy is kept, and the two float64 degree
// products evaluate the kernel values on the fly (k_near_otf).
// ---------------------------------------------------------------------------
constexpr int kDirectDim = 16;

// The coordinates of point i in registers.  The kernels below are compiled per
// point dimension D (1..8, and 16 for 9..16 with the unused slots zero), so a
// thread keeps only the registers its points need.
template <int D>
__device__ inline void load_point(const Pts& P, int32_t i, double (&x)[D]) {
    const double* p = P.xf + static_cast<int64_t>(i) * P.dim;
#pragma unroll
    for (int d = 0; d < D; ++d) x[d] = d < P.dim ? p[d] : 0.0;
}

// squared distance, coordinates in increasing order, one rounding per operation
// (zero slots past the point's dimension add exact zeros)
template <int D>
__device__ inline double sqd_regs(const double (&x)[D], const double (&y)[D]) {
    double acc = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const double t = x[d] - y[d];
        acc = acc + t * t;
    }
    return acc;
}

// Per tile (one workgroup): a bound on its largest kernel value, used as the
// float scale of the reduced-precision tile (values K / scale <= 1).  The
// kernel decreases with the distance, and every pair of points of leaves a and
// b is at least g = max(0, |c_a - c_b| - r_a - r_b) apart, c the centre of a
// leaf's bounding box and r its largest distance from it; so exp(-g^2 / eps) is
// at least the tile's largest value (1 for a leaf with itself; 1 where the bound
// underflows, since then every value does).  Two passes over the tile's 2 x 390
// points instead of its 390 x 390 distances: the scale only keeps a tile of
// small values clear of the half-precision subnormals, and any value between
// the largest entry and 1 does that.
template <int D>
__device__ inline void wg_reduce(double (&v)[D], bool is_max, double* sm) {
    // every thread's D values combined over the workgroup (min or max); result in every thread
#pragma unroll
    for (int d = 0; d < D; ++d) {
        double x = v[d];
        for (int off = 32; off > 0; off >>= 1) {
            const double y = __shfl_xor(x, off, 64);
            x = is_max ? fmax(x, y) : fmin(x, y);
        }
        v[d] = x;
    }
    __syncthreads();
    const int wv = threadIdx.x / 64, nw = blockDim.x / 64;
    if (threadIdx.x % 64 == 0)
#pragma unroll
        for (int d = 0; d < D; ++d) sm[wv * D + d] = v[d];
    __syncthreads();
#pragma unroll
    for (int d = 0; d < D; ++d) {
        double x = sm[d];
        for (int w = 1; w < nw; ++w) x = is_max ? fmax(x, sm[w * D + d]) : fmin(x, sm[w * D + d]);
        v[d] = x;
    }
}

template <int D>
__device__ inline void leaf_ball(const Pts& P, const int32_t* perm, int p0, int np, double (&c)[D], double& r,
                                 double* sm) {
    double lo[D], hi[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = INFINITY;
        hi[d] = -INFINITY;
    }
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        double x[D];
        load_point<D>(P, perm[p0 + i], x);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            lo[d] = fmin(lo[d], x[d]);
            hi[d] = fmax(hi[d], x[d]);
        }
    }
    wg_reduce<D>(lo, false, sm);
    wg_reduce<D>(hi, true, sm);
#pragma unroll
    for (int d = 0; d < D; ++d) c[d] = 0.5 * (lo[d] + hi[d]);
    double r2[1] = {0.0};
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        double x[D];
        load_point<D>(P, perm[p0 + i], x);
        r2[0] = fmax(r2[0], sqd_regs<D>(x, c));
    }
    wg_reduce<1>(r2, true, sm);
    r = sqrt(r2[0]);
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_near_scale(const NearPair* pairs, const int32_t* perm, Pts P,
                                                       float* scale) {
    __shared__ double sm[(kBlock / 64) * D];
    const NearPair pr = pairs[blockIdx.x];
    double ca[D], cb[D], ra, rb;
    leaf_ball<D>(P, perm, pr.a0, pr.na, ca, ra, sm);
    leaf_ball<D>(P, perm, pr.b0, pr.nb, cb, rb, sm);
    if (threadIdx.x == 0) {
        const double g = fmax(0.0, sqrt(sqd_regs<D>(ca, cb)) - ra - rb);
        const double m = exp(-(g * g / P.eps));
        scale[blockIdx.x] = m > 0.0 ? static_cast<float>(m) : 1.0f;
    }
}

typedef _Float16 direct_h8 __attribute__((ext_vector_type(8)));

// K / scale for a reduced-precision tile: the squared distance in float64 (the
// coordinates' differences would lose digits in float32), the exponential in
// float32.  Its relative error, about |d2 / eps| 2^-24 with |d2 / eps| < 104
// before the value underflows, stays below 1e-5 of the value: far under half an
// ulp of float16 (2^-12) or bfloat16 (2^-9).
template <int D>
__device__ inline float kval_scaled_f32(const double (&x)[D], const double (&y)[D], float neg_inv_eps,
                                        float inv_scale) {
    return __expf(static_cast<float>(sqd_regs<D>(x, y)) * neg_inv_eps) * inv_scale;
}

// Column points of a near tile in shared memory, kColStage at a time: slot c
// holds column c0 + c (clamped to the last column), its D coordinates together.
constexpr int kColStage = 256;

template <int D>
__device__ inline void stage_cols(const Pts& P, const int32_t* perm, int b0, int c0, int nb, double* cs) {
    for (int e = threadIdx.x; e < kColStage * D; e += blockDim.x) {
        const int c = e / D, d = e % D;
        const int32_t idx = perm[b0 + min(c0 + c, nb - 1)];
        cs[e] = d < P.dim ? P.xf[static_cast<int64_t>(idx) * P.dim + d] : 0.0;
    }
}

// float16 tiles packed for the matrix cores: tile t is ld x kc (kc = nb rounded
// up to 8, zero padded) with element (r, k) at ((k / 8) ld + r) 8 + k mod 8.
// Grid: (row blocks of kBlock rows, tiles).  A thread owns one row (its point in
// registers) and writes the 8 consecutive columns of each group (16 bytes;
// consecutive threads, consecutive rows); the column points come from shared
// memory as broadcasts.
template <int D>
__global__ void __launch_bounds__(kBlock) k_near_direct_f16(const NearPair* pairs, const int64_t* offp,
                                                            const int32_t* perm, Pts P, const float* scale,
                                                            _Float16* dst) {
    __shared__ double cs[kColStage * D];
    const NearPair pr = pairs[blockIdx.y];
    const int r = static_cast<int>(blockIdx.x) * kBlock + static_cast<int>(threadIdx.x);
    if (static_cast<int>(blockIdx.x) * kBlock >= pr.ld) return;   // the whole workgroup
    const float inv = 1.0f / scale[blockIdx.y];
    const float nie = static_cast<float>(-1.0 / P.eps);
    double xr[D];
    load_point<D>(P, perm[pr.a0 + min(r, pr.na - 1)], xr);
    const int kc = (pr.nb + 7) / 8 * 8;
    _Float16* out = dst + offp[blockIdx.y] + static_cast<int64_t>(r) * 8;
    const int64_t gstride = static_cast<int64_t>(pr.ld) * 8;
    for (int c0 = 0; c0 < kc; c0 += kColStage) {
        __syncthreads();   // the previous chunk is read
        stage_cols<D>(P, perm, pr.b0, c0, pr.nb, cs);
        __syncthreads();
        if (r >= pr.ld) continue;
        const int cend = min(kc, c0 + kColStage);
        for (int c = c0; c < cend; c += 8) {
            direct_h8 v;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                double xc[D];
#pragma unroll
                for (int d = 0; d < D; ++d) xc[d] = cs[(c - c0 + q) * D + d];
                const bool in = r < pr.na && c + q < pr.nb;
                v[q] = static_cast<_Float16>(in ? kval_scaled_f32<D>(xr, xc, nie, inv) : 0.0f);
            }
            *reinterpret_cast<direct_h8*>(out + (c / 8) * gstride) = v;
        }
    }
}

// bfloat16 tiles (column-major ld x nb, padded rows zero): round-to-nearest-even
// of K / scale in float32; one thread per row as above, one column at a time
template <int D>
__global__ void __launch_bounds__(kBlock) k_near_direct_bf16(const NearPair* pairs, const int32_t* perm, Pts P,
                                                             const float* scale, uint16_t* dst) {
    __shared__ double cs[kColStage * D];
    const NearPair pr = pairs[blockIdx.y];
    const int r = static_cast<int>(blockIdx.x) * kBlock + static_cast<int>(threadIdx.x);
    if (static_cast<int>(blockIdx.x) * kBlock >= pr.ld) return;   // the whole workgroup
    const float inv = 1.0f / scale[blockIdx.y];
    const float nie = static_cast<float>(-1.0 / P.eps);
    double xr[D];
    load_point<D>(P, perm[pr.a0 + min(r, pr.na - 1)], xr);
    uint16_t* out = dst + pr.off + r;
    for (int c0 = 0; c0 < pr.nb; c0 += kColStage) {
        __syncthreads();   // the previous chunk is read
        stage_cols<D>(P, perm, pr.b0, c0, pr.nb, cs);
        __syncthreads();
        if (r >= pr.ld) continue;
        const int cend = min(pr.nb, c0 + kColStage);
        for (int c = c0; c < cend; ++c) {
            double xc[D];
#pragma unroll
            for (int d = 0; d < D; ++d) xc[d] = cs[(c - c0) * D + d];
            const float x = r < pr.na ? kval_scaled_f32<D>(xr, xc, nie, inv) : 0.0f;
            const uint32_t u = __float_as_uint(x);
            out[static_cast<int64_t>(c) * pr.ld] = static_cast<uint16_t>((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
        }
    }
}

// exp(x) for x <= 0 by Tang's table-driven method (P. T. P. Tang, ACM TOMS 15(2),
// 1989): x = (64 k + j) ln2/64 + r with |r| <= ln2/128, so exp(x) = 2^k 2^(j/64) e^r,
// 2^(j/64) from a 64-entry table (each entry within an ulp) and e^r from its Taylor
// polynomial of degree 5 (remainder below 4e-17 of the value); 0 below -745.2.  The
// reduction splits ln2/64 as in det_exp (its head times the integer is exact).
// Within a few ulp of exp: used for kernel values that only enter products (the
// degree pass's near field), never for a decision of the compression.
__device__ inline double exp_neg_tab(double x, const double* tab) {
    constexpr double kInv64 = 0x1.71547652b82fep+6;         // 64 / ln 2
    constexpr double kHi = 0x1.62e42fee00000p-7;            // ln2/64, head
    constexpr double kLo = 0x1.a39ef35793c76p-39;           // ln2/64, tail
    const bool live = x > -745.2;
    x = live ? x : -745.2;   // branch-free: the value is dropped below
    const double t = rint(x * kInv64);
    const int n = static_cast<int>(t);
    const double r = fma(-t, kLo, fma(-t, kHi, x));
    double p = fma(r, 1.0 / 120.0, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    const double v = ldexp(tab[n & 63] * p, n >> 6);   // n = 64 k + j, j = n mod 64 in [0, 64)
    return live ? v : 0.0;
}

// The float64 near field of one column with the kernel evaluated on the fly:
// the waves take the work items of the plain plan in turn (as the stored-tile
// kernel takes them, one item per wave on a full grid), lane l
// owning rows row0 + 2 l and row0 + 2 l + 1 of each 128-row pass.  The item's
// (at most 64) column points and weights are loaded once, one per lane, and
// broadcast from their lane column by column; part[part_off + row] = sum over the
// columns in increasing order of K(row, col) w[col], K in float64 with one
// rounding per operation (the exponent's argument d2 times 1/eps: within an ulp
// of the oracle's d2 / eps).
// one run of consecutive items of a leaf and row group: each lane takes two
// rows at a time and accumulates them over every column of the run's items in
// item order (w = nullptr: all ones); the run writes one partial-sum slot
template <int D>
__device__ inline void near_otf_run(const NearItem* items, const OtfRun R, const int32_t* perm, const Pts& P,
                                    const double* w, double* part, const double* tab) {
    const int lane = threadIdx.x % kWave;
    const NearItem I0 = items[R.item];
    const double ie = 1.0 / P.eps;
    const int rend = min(I0.ld, I0.row0 + I0.nrows);
    for (int r0 = I0.row0; r0 < rend; r0 += 2 * kWave) {
        const int row = r0 + 2 * lane;
        double x0[D], x1[D];
        const bool v0 = row < I0.row_n, v1 = row + 1 < I0.row_n;
        load_point<D>(P, perm[I0.row_pos + min(row, I0.row_n - 1)], x0);
        load_point<D>(P, perm[I0.row_pos + min(row + 1, I0.row_n - 1)], x1);
        double a0 = 0.0, a1 = 0.0;
        for (int q = 0; q < R.count; ++q) {
            const NearItem I = items[R.item + q];
            double xc[D];
            load_point<D>(P, perm[I.col_pos + min(lane, I.ncols - 1)], xc);
            const double wl = w ? w[I.col_pos + min(lane, I.ncols - 1)] : 1.0;
            for (int j = 0; j < I.ncols; ++j) {
                double y[D];
#pragma unroll
                for (int d = 0; d < D; ++d) y[d] = lane_value(xc[d], j);
                const double wj = lane_value(wl, j);
                const double k0 = exp_neg_tab(-(sqd_regs<D>(x0, y) * ie), tab);   // values only
                const double k1 = exp_neg_tab(-(sqd_regs<D>(x1, y) * ie), tab);
                a0 = a0 + (v0 ? k0 : 0.0) * wj;
                a1 = a1 + (v1 ? k1 : 0.0) * wj;
            }
        }
        if (row < rend) {
            double* out = part + R.part_off + row;
            out[0] = a0;
            if (row + 1 < rend) out[1] = a1;
        }
    }
}


template <int D>
__global__ void __launch_bounds__(kBlock) k_near_otf(const NearItem* items, const OtfRun* runs, int64_t nruns,
                                                    const int32_t* perm, Pts P, const double* w, double* part) {
    __shared__ double tab[64];   // 2^(j/64)
    if (threadIdx.x < 64) tab[threadIdx.x] = exp2(static_cast<double>(threadIdx.x) / 64.0);
    __syncthreads();
    const int64_t waves = static_cast<int64_t>(gridDim.x) * (blockDim.x / kWave);
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x / kWave) + threadIdx.x / kWave; u < nruns;
         u += waves)
        near_otf_run<D>(items, runs[u], perm, P, w, part, tab);
}

// launches a kernel template specialised on the point dimension
#define HDM_DIM_DISPATCH(dim, KERNEL, ...)                                                          \
    do {                                                                                           \
        switch (dim) {                                                                             \
            case 1: hipLaunchKernelGGL(KERNEL<1>, __VA_ARGS__); break;                              \
            case 2: hipLaunchKernelGGL(KERNEL<2>, __VA_ARGS__); break;                              \
            case 3: hipLaunchKernelGGL(KERNEL<3>, __VA_ARGS__); break;                              \
            case 4: hipLaunchKernelGGL(KERNEL<4>, __VA_ARGS__); break;                              \
            case 5: hipLaunchKernelGGL(KERNEL<5>, __VA_ARGS__); break;                              \
            case 6: hipLaunchKernelGGL(KERNEL<6>, __VA_ARGS__); break;                              \
            case 7: hipLaunchKernelGGL(KERNEL<7>, __VA_ARGS__); break;                              \
            case 8: hipLaunchKernelGGL(KERNEL<8>, __VA_ARGS__); break;                              \
            default: hipLaunchKernelGGL(KERNEL<kDirectDim>, __VA_ARGS__); break;                    \
        }                                                                                          \
    } while (0)

struct FarBlock {
    int64_t off;       // element offset (row-major rank x cols)
    int64_t col0;      // first column in the global column map
    int32_t rows, cols;
    int64_t sk0;       // skeleton offset of the row node
};

__global__ void k_far_tiles(const FarBlock* blocks, const int32_t* colmap, const int32_t* skel, Pts P, double* out) {
    const FarBlock fb = blocks[blockIdx.y];
    const int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (e >= static_cast<int64_t>(fb.rows) * fb.cols) return;
    const int i = static_cast<int>(e / fb.cols), c = static_cast<int>(e % fb.cols);
    out[fb.off + e] = kval(P, skel[fb.sk0 + i], skel[colmap[fb.col0 + c]]);
}

__global__ void k_check_points(const double* x, int64_t cnt, int* bad) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i < cnt && !isfinite(x[i])) atomicOr(bad, 1);
}

template <typename T>
T* ptr(DevBuf<T>& b) { return b.get(); }

}  // namespace

// ---------------------------------------------------------------------------
// host orchestration
// ---------------------------------------------------------------------------
// Points as the kernels see them, plus the integer-code helpers when the
// matrix-core path applies (u8 codes whose dimension is a multiple of 16).
struct Geo {
    Pts P{};
    bool gram = false;
    DevBuf<int32_t> nu, ns;   // sum of squared codes, unsigned and offset by 128
};

// exact u8 distance blocks with matrix cores (see k_gram_u8); blocks must stay
// alive until the launches complete, so this synchronises the stream
// and checks every block against the output's extent before the launch
template <typename T>
static void gram_launch(const Geo& G, const std::vector<GramBlock>& blocks, int mode, DevBuf<T>& out, hipStream_t s) {
    static_assert(sizeof(T) == (std::is_same<T, double>::value ? 8 : 4), "output is int32 or float64");
    HDM_CHECK(((mode == 0) == std::is_same<T, int32_t>::value), HDM_EINTERNAL, "distance block output type");
    if (blocks.empty()) return;
    int64_t maxt = 0;
    for (const GramBlock& b : blocks) {
        HDM_CHECK(b.nr >= 0 && b.nc >= 0 && b.off >= 0, HDM_EINTERNAL, "distance block with a negative extent");
        if (b.nr == 0 || b.nc == 0) continue;
        const int64_t last = b.colmajor ? b.off + int64_t(b.nc - 1) * b.ld + (b.nr - 1)
                                        : b.off + int64_t(b.nr - 1) * b.ld + (b.nc - 1);
        HDM_CHECK(b.ld >= (b.colmajor ? b.nr : b.nc) && last < static_cast<int64_t>(out.n), HDM_EINTERNAL,
                  "distance block outside its output");
        maxt = std::max<int64_t>(maxt, int64_t((b.nr + 63) / 64) * ((b.nc + 63) / 64));
    }
    DevBuf<GramBlock> d = to_device(blocks, s);
    if (maxt == 0) return;
    for (size_t base = 0; base < blocks.size(); base += 65535) {
        const int cnt = static_cast<int>(std::min<size_t>(65535, blocks.size() - base));
        hipLaunchKernelGGL(k_gram_u8, dim3(static_cast<unsigned>(maxt), cnt), dim3(256), 0, s, d.get() + base, G.P.xu,
                           G.ns.get(), G.P.dim, G.P.eps, mode, static_cast<void*>(out.get()));
    }
    check_launch("u8 distance blocks");
    HDM_HIP(hipStreamSynchronize(s));
}
static void tree_ranges(int64_t n, int depth, std::vector<int64_t>& start, std::vector<int64_t>& size) {
    const int64_t nn = int64_t(1) << (depth + 1);
    start.assign(nn, 0);
    size.assign(nn, 0);
    size[1] = n;
    for (int64_t h = 1; h < (int64_t(1) << depth); ++h) {
        const int64_t nl = size[h] / 2;
        start[2 * h] = start[h];
        size[2 * h] = nl;
        start[2 * h + 1] = start[h] + nl;
        size[2 * h + 1] = size[h] - nl;
    }
}

// one perfect tree of the given depth: ball tree (mode 0) or random-pivot tree (mode 1)
// mode 0: the ball tree (ntrees = 1); mode 1: ntrees neighbour trees at once
// (trees it0 .. it0 + ntrees - 1, each level of all of them in one launch);
// perm, tmp and key hold ntrees x n entries, pq ntrees x 2L.
// One or several trees built level by level on a stream; the caller can
// interleave the levels of two builds on two streams.
struct TreeBuild {
    Op& op;
    int mode, it0, ntrees;
    DevBuf<int32_t>& perm;
    DevBuf<int32_t>& tmp;
    const Geo& G;
    hipStream_t s;
    DevBuf<int32_t>& samp;
    DevBuf<int32_t>& nsamp;
    DevBuf<int32_t>& pq;
    DevBuf<double>& sumk;
    DevBuf<double>& key;
    DevBuf<int32_t> sample_ids;
    DevBuf<double> kvals;

    TreeBuild(Op& op_, int mode_, int it0_, int ntrees_, DevBuf<int32_t>& perm_, DevBuf<int32_t>& tmp_, const Geo& G_,
              hipStream_t s_, DevBuf<int32_t>& samp_, DevBuf<int32_t>& nsamp_, DevBuf<int32_t>& pq_,
              DevBuf<double>& sumk_, DevBuf<double>& key_)
        : op(op_), mode(mode_), it0(it0_), ntrees(ntrees_), perm(perm_), tmp(tmp_), G(G_), s(s_), samp(samp_),
          nsamp(nsamp_), pq(pq_), sumk(sumk_), key(key_) {
        HDM_CHECK(mode == 1 || ntrees == 1, HDM_EINTERNAL, "one ball tree at a time");
        HDM_CHECK(perm.n >= static_cast<size_t>(ntrees) * op.n && tmp.n >= static_cast<size_t>(ntrees) * op.n &&
                      key.n >= static_cast<size_t>(ntrees) * op.n &&
                      pq.n >= static_cast<size_t>(ntrees) * 2 * op.L,
                  HDM_EINTERNAL, "tree buffers too small");
        if (mode == 0 && G.gram) {
            sample_ids.alloc(static_cast<size_t>(op.L) * kSample);
            kvals.alloc(static_cast<size_t>(op.n) * kSample);
        }
        hipLaunchKernelGGL(k_iota, dim3(ceil_div(op.n, kBlock), ntrees), dim3(kBlock), 0, s, perm.get(), op.n);
    }

    void level(int lvl) {
        const int64_t pq_stride = 2 * static_cast<int64_t>(op.L);
        const Pts& P = G.P;
        const int64_t n = op.n;
        const int gN = ceil_div(n, kBlock);
        const int nodes = 1 << lvl;
        if (mode == 0) {
            hipLaunchKernelGGL(k_tree_sample, dim3(nodes), dim3(64), 0, s, lvl, op.d_start.get(), op.d_size.get(),
                               op.prm.seed, samp.get(), nsamp.get());
            if (G.gram) {
                // kernel values point x sample by matrix cores, then the sample sums in order
                hipLaunchKernelGGL(k_sample_ids, dim3(nodes), dim3(64), 0, s, samp.get(), nsamp.get(), perm.get(), nodes,
                                   sample_ids.get());
                std::vector<GramBlock> blocks;
                for (int t = 0; t < nodes; ++t) {
                    const int64_t h = nodes + t;
                    blocks.push_back(GramBlock{perm.get() + op.start[h], sample_ids.get() + int64_t(t) * kSample,
                                               static_cast<int32_t>(op.size[h]),
                                               static_cast<int32_t>(std::min<int64_t>(op.size[h], kSample)),
                                               op.start[h] * kSample, kSample, 0});
                }
                gram_launch(G, blocks, 1, kvals, s);
                hipLaunchKernelGGL(k_row_sums, dim3(gN), dim3(kBlock), 0, s, kvals.get(), n, nsamp.get(), kSample, lvl,
                                   op.d_start.get(), sumk.get());
            } else {
                hipLaunchKernelGGL(k_tree_sumk, dim3(gN), dim3(kBlock), 0, s, lvl, n, op.d_start.get(), perm.get(),
                                   samp.get(), nsamp.get(), P, sumk.get());
            }
            hipLaunchKernelGGL(k_tree_pq, dim3(nodes), dim3(kPqBlock), 0, s, lvl, op.d_start.get(), op.d_size.get(),
                               perm.get(), sumk.get(), P, pq.get());
        } else {
            hipLaunchKernelGGL(k_knn_pq, dim3(ceil_div(nodes, 64), ntrees), dim3(64), 0, s, lvl, op.d_start.get(),
                               op.d_size.get(), perm.get(), n, op.prm.seed, it0, pq.get(), pq_stride);
        }
        hipLaunchKernelGGL(k_tree_key, dim3(gN, ntrees), dim3(kBlock), 0, s, lvl, n, op.d_start.get(), perm.get(),
                           pq.get(), pq_stride, P, mode, key.get());
        // a node has at most ceil(n / 2^lvl) members: keys in registers when a
        // thread's run fits (and is long enough to be worth it)
        const int64_t maxnode = (n + nodes - 1) / nodes;
        const int64_t per = (maxnode + kSplitBlock - 1) / kSplitBlock;
        if (per > 4 && per <= kSplitReg)
            hipLaunchKernelGGL(k_tree_split<true>, dim3(nodes, ntrees), dim3(kSplitBlock), 0, s, lvl, op.d_start.get(),
                               op.d_size.get(), perm.get(), key.get(), tmp.get(), n);
        else
            hipLaunchKernelGGL(k_tree_split<false>, dim3(nodes, ntrees), dim3(kSplitBlock), 0, s, lvl,
                               op.d_start.get(), op.d_size.get(), perm.get(), key.get(), tmp.get(), n);
        check_launch("tree level");
        std::swap(perm, tmp);
    }

    // the sample buffers are freed on return while the last level's kernels may
    // still be queued on s: wait for them first (hipFree's implicit
    // synchronisation is not relied on, e.g. for non-blocking streams)
    ~TreeBuild() {
        if (sample_ids.n || kvals.n) (void)hipStreamSynchronize(s);
    }
};

// near lists: self plus ceil(budget * L) other leaves by (votes desc, id asc), symmetrised
static void build_near_lists(Op& op, const std::vector<int32_t>& votes) {
    const int64_t L = op.L;
    std::vector<uint8_t> rel(static_cast<size_t>(L * L), 0);
    const int64_t extra = static_cast<int64_t>(std::ceil(op.prm.budget * static_cast<double>(L)));
    std::vector<int32_t> order(L);
    for (int64_t a = 0; a < L; ++a) {
        rel[a * L + a] = 1;
        int cnt = 0;
        for (int64_t b = 0; b < L; ++b)
            if (b != a) order[cnt++] = static_cast<int32_t>(b);
        // the first `extra` by (votes desc, id asc), a strict order: only they are sorted
        const int64_t top = std::min<int64_t>(extra, cnt);
        std::partial_sort(order.begin(), order.begin() + top, order.begin() + cnt, [&](int32_t x, int32_t y) {
            const int32_t vx = votes[a * L + x], vy = votes[a * L + y];
            return vx != vy ? vx > vy : x < y;
        });
        for (int64_t t = 0; t < top; ++t) rel[a * L + order[t]] = 1;
    }
    for (int64_t a = 0; a < L; ++a)
        for (int64_t b = 0; b < L; ++b)
            if (rel[a * L + b]) rel[b * L + a] = 1;
    op.near_off.assign(L + 1, 0);
    op.near_idx.clear();
    for (int64_t a = 0; a < L; ++a) {
        op.near_off[a] = static_cast<int32_t>(op.near_idx.size());
        for (int64_t b = 0; b < L; ++b)
            if (rel[a * L + b]) op.near_idx.push_back(static_cast<int32_t>(b));
    }
    op.near_off[L] = static_cast<int32_t>(op.near_idx.size());
}

// far lists: dual traversal from (root, root); a same-level pair without any
// near leaf pair beneath it is far, otherwise its four child pairs are visited
static void build_far_lists(Op& op) {
    const int64_t L = op.L;
    const int depth = op.depth;
    // near leaf relation as bit rows for quick subtree queries
    std::vector<uint8_t> rel(static_cast<size_t>(L * L), 0);
    for (int64_t a = 0; a < L; ++a)
        for (int32_t t = op.near_off[a]; t < op.near_off[a + 1]; ++t) rel[a * L + op.near_idx[t]] = 1;
    // prefix sums over the relation matrix for O(1) rectangle queries
    std::vector<int64_t> ps(static_cast<size_t>((L + 1) * (L + 1)), 0);
    for (int64_t a = 0; a < L; ++a)
        for (int64_t b = 0; b < L; ++b)
            ps[(a + 1) * (L + 1) + (b + 1)] = rel[a * L + b] + ps[a * (L + 1) + (b + 1)] + ps[(a + 1) * (L + 1) + b] -
                                              ps[a * (L + 1) + b];
    auto related = [&](int64_t x, int64_t y, int lvl) {
        const int sh = depth - lvl;
        const int64_t x0 = (x << sh) - L, x1 = x0 + (int64_t(1) << sh);
        const int64_t y0 = (y << sh) - L, y1 = y0 + (int64_t(1) << sh);
        return ps[x1 * (L + 1) + y1] - ps[x0 * (L + 1) + y1] - ps[x1 * (L + 1) + y0] + ps[x0 * (L + 1) + y0] > 0;
    };
    std::vector<std::vector<int32_t>> far(static_cast<size_t>(op.nnodes));
    struct Item { int64_t x, y; int lvl; };
    std::vector<Item> stack{{1, 1, 0}};
    while (!stack.empty()) {
        const Item it = stack.back();
        stack.pop_back();
        if (!related(it.x, it.y, it.lvl)) { far[it.x].push_back(static_cast<int32_t>(it.y)); continue; }
        if (it.lvl == depth) continue;
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) stack.push_back({2 * it.x + i, 2 * it.y + j, it.lvl + 1});
    }
    op.far_off.assign(op.nnodes + 1, 0);
    op.far_idx.clear();
    for (int64_t h = 0; h < op.nnodes; ++h) {
        std::sort(far[h].begin(), far[h].end());
        op.far_off[h] = static_cast<int32_t>(op.far_idx.size());
        op.far_idx.insert(op.far_idx.end(), far[h].begin(), far[h].end());
    }
    op.far_off[op.nnodes] = static_cast<int32_t>(op.far_idx.size());
}

// Buffers of a skeletonisation in flight: the level loop is enqueued by
// skeletonize_levels and completed (sizes downloaded, outputs compacted) by
// skeletonize_finish, so the host can do other work while the levels run.
struct SkelRun {
    int cmax = 0, rmax = 0;
    DevBuf<int32_t> cand, ncand, rows, nrows, cp, status, uniq, cnt, vts, skel_fix, rows_fix, sizes;
    DevBuf<uint32_t> bits;
    DevBuf<double> B, Pfix;
    DevBuf<int64_t> offs;   // compaction offsets (skeletons, P, rows), read by k_compact
};

// The evaluation-precision near tiles and the near field of K~ 1 run on the side
// stream from the level with at most kSideGateNodes nodes on: the levels above
// are latency-bound (a few workgroups each) and leave the device mostly idle,
// while the leaf levels need its bandwidth (0: from the start).
// N = 100000, ms per compression: 0 -> 15.3, 32 -> 14.8, 8 -> 15.2, 2 -> 14.7 (with
// the shared-memory tile kernels; the spread is near the run-to-run noise)
constexpr int kSideGateNodes = 32;

static void skeletonize_levels(Op& op, const Geo& G, hipStream_t s, SkelRun& R, hipEvent_t gate) {
    const Pts& P = G.P;
    const int64_t n = op.n;
    const int k = op.prm.knn_k, smax = op.prm.max_rank_s;
    int64_t leafmax = 0;
    for (int64_t h = op.L; h < 2 * int64_t(op.L); ++h) leafmax = std::max(leafmax, op.size[h]);
    const int cmax = static_cast<int>(std::max<int64_t>(leafmax, 2 * static_cast<int64_t>(smax)));
    HDM_CHECK(cmax <= kMaxCand, HDM_EINVAL, "leaf size and 2 * max_rank_s must be <= 2048");
    const int rmax = 2 * smax;
    HDM_CHECK(rmax <= kMaxRows, HDM_EINVAL, "max_rank_s must be <= 1024");
    R.cmax = cmax;
    R.rmax = rmax;
    const int64_t NN = op.nnodes;
    // per-level workspaces, sized for the widest level
    const int64_t maxnodes = op.L;
    R.cand.alloc(maxnodes * cmax);
    R.ncand.alloc(maxnodes);
    R.rows.alloc(maxnodes * rmax);
    R.nrows.alloc(maxnodes);
    R.cp.alloc(maxnodes * cmax);
    R.status.alloc(maxnodes);
    R.uniq.alloc(static_cast<size_t>(maxnodes) * cmax * k);
    R.B.alloc(static_cast<size_t>(maxnodes) * rmax * cmax);
    const size_t vote_shmem = sizeof(int32_t) * (2 * static_cast<size_t>((n + 31) / 32) + static_cast<size_t>(cmax) * k);
    bool sorted_votes = vote_shmem <= static_cast<size_t>(kVoteShared);
    if (sorted_votes) {   // the kernel's own shared arrays plus the dynamic part within the 160 KB of a CU
        hipFuncAttributes fa{};
        HDM_HIP(hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(&k_row_select<true>)));
        sorted_votes = vote_shmem + fa.sharedSizeBytes <= 160 * 1024;
    }
    if (sorted_votes) R.vts.alloc(static_cast<size_t>(maxnodes) * cmax * k);
    else R.cnt.alloc(static_cast<size_t>(maxnodes) * n);
    R.bits.alloc(static_cast<size_t>(maxnodes) * ((n + 31) / 32));
    // per-node slots filled level by level (heap id h): skeletons, sampled rows, P, and
    // rank | candidates | rows | row-fill status; compacted once at the end, so the
    // levels run back to back without the host
    R.skel_fix.alloc(static_cast<size_t>(NN) * smax);
    R.rows_fix.alloc(static_cast<size_t>(NN) * rmax);
    R.Pfix.alloc(static_cast<size_t>(NN) * smax * cmax);
    R.sizes.alloc(4 * static_cast<size_t>(NN));
    auto& cand = R.cand;
    auto& ncand = R.ncand;
    auto& rows = R.rows;
    auto& nrows = R.nrows;
    auto& cp = R.cp;
    auto& status = R.status;
    auto& uniq = R.uniq;
    auto& B = R.B;
    auto& cnt = R.cnt;
    auto& bits = R.bits;
    auto& skel_fix = R.skel_fix;
    auto& rows_fix = R.rows_fix;
    auto& Pfix = R.Pfix;
    auto& sizes = R.sizes;
    int32_t* d_rank = sizes.get();
    int32_t* d_nc = d_rank + NN;
    int32_t* d_nr = d_rank + 2 * NN;
    int32_t* d_st = d_rank + 3 * NN;
    HDM_HIP(hipMemsetAsync(sizes.get(), 0, sizes.bytes(), s));
    // the ID's shared memory: Householder vector, column norms, then as many rows of B as fit
    size_t id_shmem = 0;
    int64_t id_lds = 0;
    {
        int dev = 0, max_shared = 0;
        HDM_HIP(hipGetDevice(&dev));
        HDM_HIP(hipDeviceGetAttribute(&max_shared, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        // both workgroup sizes stage the same rows (the larger static part decides)
        const void* id_fns[2] = {reinterpret_cast<const void*>(&k_pivoted_id<kBlock>),
                                 reinterpret_cast<const void*>(&k_pivoted_id<kIdWide>)};
        size_t stat = 0;
        for (const void* f : id_fns) {
            hipFuncAttributes fa{};
            HDM_HIP(hipFuncGetAttributes(&fa, f));
            stat = std::max(stat, fa.sharedSizeBytes);
        }
        const int64_t avail = (static_cast<int64_t>(max_shared) - static_cast<int64_t>(stat)) /
                              static_cast<int64_t>(sizeof(double));
        HDM_CHECK(avail >= rmax + cmax, HDM_EINTERNAL, "shared memory too small for the ID's vectors");
        id_lds = avail - rmax - cmax;
        id_shmem = sizeof(double) * static_cast<size_t>(rmax + cmax + id_lds);
        if (id_shmem > 65536)
            for (const void* f : id_fns)
                HDM_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(id_shmem)));
    }
    // row selection: the neighbour votes are counted through a bitmap over the
    // points in shared memory when it fits, else in a dense per-node array
    size_t sort_shmem = 0;
    if (sorted_votes) {
        sort_shmem = vote_shmem;
        HDM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_row_select<true>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(sort_shmem)));
    }
    std::vector<int32_t> h_nc(maxnodes), h_nr(maxnodes);
    // the row bitmaps start clear; each row selection clears its node's after use
    HDM_HIP(hipMemsetAsync(bits.get(), 0, sizeof(uint32_t) * static_cast<size_t>(1 << op.depth) * ((n + 31) / 32), s));
    bool gated = false;
    for (int lvl = op.depth; lvl >= 1; --lvl) {
        if (!gated && (kSideGateNodes <= 0 || (int64_t(1) << lvl) <= kSideGateNodes)) {
            HDM_HIP(hipEventRecord(gate, s));
            gated = true;
        }
        const int nodes = 1 << lvl;
        LevelArgs A{};
        A.lvl = lvl;
        A.depth = op.depth;
        A.n = n;
        A.k = k;
        A.s = smax;
        A.cmax = cmax;
        A.rmax = rmax;
        A.seed = op.prm.seed;
        A.tau = op.prm.tau;
        A.start = op.d_start.get();
        A.size = op.d_size.get();
        A.perm = op.perm.get();
        A.iperm = op.iperm.get();
        A.kidx = op.knn_idx.get();
        A.skel_fix = skel_fix.get();
        A.rank = d_rank;
        A.cand = cand.get();
        A.ncand = ncand.get();
        A.cnt = cnt.get();
        A.bits = bits.get();
        A.uniq = uniq.get();
        A.vts = R.vts.get();
        A.rows = rows.get();
        A.nrows = nrows.get();
        A.B = B.get();
        A.cp = cp.get();
        A.Pfix = Pfix.get();
        A.rk = d_rank;
        A.status = status.get();
        A.lds_b = id_lds;
        A.rows_fix = rows_fix.get();
        A.nc_all = d_nc;
        A.nr_all = d_nr;
        A.st_all = d_st;
        if (sorted_votes) {
            hipLaunchKernelGGL(k_row_select<true>, dim3(nodes), dim3(kBlock), sort_shmem, s, A);
        } else {
            hipLaunchKernelGGL(k_cand, dim3(nodes), dim3(kBlock), 0, s, A);
            HDM_HIP(hipMemsetAsync(cnt.get(), 0, sizeof(int32_t) * static_cast<size_t>(nodes) * n, s));
            hipLaunchKernelGGL(k_row_count, dim3(ceil_div(static_cast<int64_t>(cmax) * k, kBlock), nodes), dim3(kBlock), 0,
                               s, A);
            hipLaunchKernelGGL(k_row_select<false>, dim3(nodes), dim3(kBlock), 0, s, A);
        }
        if (G.gram) {
            // the Gram-form kernel blocks are planned on the host from the level's sizes
            ncand.download(h_nc.data(), nodes, s);
            nrows.download(h_nr.data(), nodes, s);
            HDM_HIP(hipStreamSynchronize(s));
            std::vector<GramBlock> blocks;
            for (int t = 0; t < nodes; ++t)
                blocks.push_back(GramBlock{rows.get() + int64_t(t) * rmax, cand.get() + int64_t(t) * cmax, h_nr[t],
                                           h_nc[t], int64_t(t) * rmax * cmax, h_nc[t], 0});
            gram_launch(G, blocks, 1, B, s);
        } else if (!P.is_u8 && P.dim <= kDimReg && lvl == op.depth) {
            // leaves: many candidates per node, one per thread (above the leaves the
            // element-per-thread kernel keeps more threads busy)
            hipLaunchKernelGGL(k_block_reg, dim3(kBlockSlices, nodes), dim3(kBlock), 0, s, A, P);
        } else {
            hipLaunchKernelGGL(k_block, dim3(ceil_div(static_cast<int64_t>(rmax) * cmax, kBlock), nodes), dim3(kBlock),
                               0, s, A, P);
        }
        // the leaves in launches of at most kIdNodes: their blocks B, which every
        // step of the QR reads and writes again, then fit the last-level cache
        const int per = lvl == op.depth ? std::min(kIdNodes, nodes) : nodes;
        for (int t0 = 0; t0 < nodes; t0 += per) {
            A.node0 = t0;
            if (rmax > kIdWideRows)
                hipLaunchKernelGGL(k_pivoted_id<kIdWide>, dim3(std::min(per, nodes - t0)), dim3(kIdWide), id_shmem, s, A);
            else
                hipLaunchKernelGGL(k_pivoted_id<kBlock>, dim3(std::min(per, nodes - t0)), dim3(kBlock), id_shmem, s, A);
        }
        A.node0 = 0;
        check_launch("skeletonisation");
    }
    if (!gated) HDM_HIP(hipEventRecord(gate, s));
}

static void skeletonize_finish(Op& op, hipStream_t s, SkelRun& R) {
    const int64_t NN = op.nnodes;
    const int smax = op.prm.max_rank_s;
    int32_t* d_rank = R.sizes.get();
    int32_t* d_nc = d_rank + NN;
    int32_t* d_nr = d_rank + 2 * NN;
    // sizes of every node, then offsets in level order (leaves first, heap order within a level)
    std::vector<int32_t> hs(4 * static_cast<size_t>(NN));
    R.sizes.download(hs.data(), hs.size(), s);
    HDM_HIP(hipStreamSynchronize(s));
    op.rank.assign(NN, 0);
    op.ncand.assign(NN, 0);
    op.nrows.assign(NN, 0);
    op.skoff.assign(NN, 0);
    op.poff.assign(NN, 0);
    op.rowoff.assign(NN, 0);
    int64_t sk_next = 0, row_next = 0, p_next = 0;
    for (int lvl = op.depth; lvl >= 1; --lvl)
        for (int64_t h = int64_t(1) << lvl; h < (int64_t(2) << lvl); ++h) {
            HDM_CHECK(hs[3 * NN + h] == 0, HDM_EINTERNAL, "row sampling did not terminate");
            op.rank[h] = hs[h];
            op.ncand[h] = hs[NN + h];
            op.nrows[h] = hs[2 * NN + h];
            op.skoff[h] = sk_next;
            sk_next += op.rank[h];
            op.rowoff[h] = row_next;
            row_next += op.nrows[h];
            op.poff[h] = p_next;
            p_next += static_cast<int64_t>(op.rank[h]) * op.ncand[h];
        }
    std::vector<int64_t> offs(3 * static_cast<size_t>(NN));
    std::copy(op.skoff.begin(), op.skoff.end(), offs.begin());
    std::copy(op.poff.begin(), op.poff.end(), offs.begin() + NN);
    std::copy(op.rowoff.begin(), op.rowoff.end(), offs.begin() + 2 * NN);
    R.offs = to_device(offs, s);
    const DevBuf<int64_t>& d_offs = R.offs;
    op.nskel = sk_next;
    op.skel.alloc(sk_next + 1);
    op.rows.alloc(row_next + 1);
    op.np = p_next;
    op.P64.alloc(p_next > 0 ? p_next : 1);
    if (NN > 2)
        hipLaunchKernelGGL(k_compact, dim3(NN - 2), dim3(kBlock), 0, s, R.skel_fix.get(), R.rows_fix.get(),
                           R.Pfix.get(), d_rank, d_nc, d_nr, d_offs.get(), d_offs.get() + NN, d_offs.get() + 2 * NN, smax,
                           R.cmax, R.rmax, op.skel.get(), op.P64.get(), op.rows.get());
    check_launch("compact");
    // no wait: R outlives the compaction (the far tiles wait for s before the
    // operator build goes on)
}

// near tiles; with float64 points the launch is left in flight on s (the pair
// descriptors stay alive in op.near_pairs until the operator is finished)
static void build_near_tiles(Op& op, const Geo& G, hipStream_t s) {
    const Pts& P = G.P;
    const int64_t L = op.L;
    // near blocks: per leaf, column-major ld x (sum of near leaf sizes), ld = rows rounded up to 8
    op.near_block_off.assign(L, 0);
    op.near_ld.assign(L, 0);
    op.near_tile_off.assign(op.near_idx.size(), 0);
    std::vector<NearPair> pairs;
    int64_t off = 0;
    for (int64_t a = 0; a < L; ++a) {
        const int64_t ha = L + a;
        const int32_t ld = static_cast<int32_t>((op.size[ha] + 7) / 8 * 8);
        op.near_ld[a] = ld;
        op.near_block_off[a] = off;
        for (int32_t t = op.near_off[a]; t < op.near_off[a + 1]; ++t) {
            const int64_t hb = L + op.near_idx[t];
            op.near_tile_off[t] = off;
            pairs.push_back(NearPair{off, ld, static_cast<int32_t>(op.start[ha]), static_cast<int32_t>(op.size[ha]),
                                     static_cast<int32_t>(op.start[hb]), static_cast<int32_t>(op.size[hb]), 0});
            off += static_cast<int64_t>(ld) * op.size[hb];
        }
    }
    op.near_elems = off;
    for (const NearPair& pr : pairs)
        HDM_CHECK(pr.na >= 1 && pr.na <= pr.ld && pr.a0 >= 0 && pr.a0 + pr.na <= op.n && pr.b0 >= 0 && pr.nb >= 1 &&
                      pr.b0 + pr.nb <= op.n && pr.off >= 0 && pr.off + static_cast<int64_t>(pr.ld) * pr.nb <= off,
                  HDM_EINTERNAL, "near tile descriptor outside its buffers");
    // float64 points of few coordinates: the tiles go straight to the evaluation
    // precision and the degree products evaluate the kernel on the fly
    const bool direct = !G.gram && !P.is_u8 && P.dim <= kDirectDim && op.prm.near_prec != HDM_F64;
    op.near_direct = direct;
    if (!direct) op.near64.alloc(off);
    if (direct) {
        op.near_pairs.alloc(pairs.size() * sizeof(NearPair));
        op.near_pairs.upload(reinterpret_cast<const char*>(pairs.data()), pairs.size() * sizeof(NearPair), s);
        const NearPair* pairs_dev = reinterpret_cast<const NearPair*>(op.near_pairs.get());
        const int64_t np = static_cast<int64_t>(pairs.size());
        int64_t maxe = 0;
        for (auto& p : pairs) maxe = std::max<int64_t>(maxe, static_cast<int64_t>(p.ld) * p.nb);
        if (op.prm.near_prec == HDM_F32) {
            // unscaled float32 values of the float64 kernel
            op.nearT.alloc(static_cast<size_t>(std::max<int64_t>(op.near_elems, 1)) * sizeof(float));
            for (int64_t base = 0; base < np; base += 65535) {
                const int cnt = static_cast<int>(std::min<int64_t>(65535, np - base));
                hipLaunchKernelGGL(k_near_tiles, dim3(ceil_div(maxe, kBlock), cnt), dim3(kBlock), 0, s, pairs_dev + base,
                                   op.perm.get(), P, nullptr, reinterpret_cast<float*>(op.nearT.get()));
            }
        } else {
            op.near_scale.alloc(static_cast<size_t>(np));
            HDM_DIM_DISPATCH(P.dim, k_near_scale, dim3(static_cast<unsigned>(np)), dim3(kBlock), 0, s, pairs_dev,
                             op.perm.get(), P, op.near_scale.get());
            int32_t maxld = 0;
            for (auto& p : pairs) maxld = std::max(maxld, p.ld);
            const unsigned gx = static_cast<unsigned>(ceil_div(static_cast<int64_t>(maxld), kBlock));
            if (op.prm.near_prec == HDM_BF16) {
                op.nearT.alloc(static_cast<size_t>(std::max<int64_t>(op.near_elems, 1)) * sizeof(uint16_t));
                for (int64_t base = 0; base < np; base += 65535) {
                    const int cnt = static_cast<int>(std::min<int64_t>(65535, np - base));
                    HDM_DIM_DISPATCH(P.dim, k_near_direct_bf16, dim3(std::max(gx, 1u), cnt), dim3(kBlock), 0, s,
                                     pairs_dev + base, op.perm.get(), P, op.near_scale.get() + base,
                                     reinterpret_cast<uint16_t*>(op.nearT.get()));
                }
            } else {   // float16, packed for the matrix cores
                packed_near_offsets(op);
                if (!op.conv_keep) op.conv_keep.reset(new Op::ConvKeep());
                op.conv_keep->h64.push_back(op.near_tile_off_mma);
                op.conv_keep->d64.push_back(to_device(op.conv_keep->h64.back(), s));
                const int64_t* offp = op.conv_keep->d64.back().get();
                op.nearT.alloc(static_cast<size_t>(std::max<int64_t>(op.near_elems_mma, 1)) * sizeof(_Float16));
                for (int64_t base = 0; base < np; base += 65535) {
                    const int cnt = static_cast<int>(std::min<int64_t>(65535, np - base));
                    HDM_DIM_DISPATCH(P.dim, k_near_direct_f16, dim3(std::max(gx, 1u), cnt), dim3(kBlock), 0, s,
                                     pairs_dev + base, offp + base, op.perm.get(), P, op.near_scale.get() + base,
                                     reinterpret_cast<_Float16*>(op.nearT.get()));
                }
            }
        }
        check_launch("near tiles (evaluation precision)");
        op.near_converted = true;
        return;
    }
    if (G.gram) {
        HDM_HIP(hipMemsetAsync(op.near64.get(), 0, op.near64.bytes(), s));   // padded rows stay zero
        std::vector<GramBlock> blocks;
        for (const NearPair& pr : pairs)
            blocks.push_back(GramBlock{op.perm.get() + pr.a0, op.perm.get() + pr.b0, pr.na, pr.nb, pr.off, pr.ld, 1});
        gram_launch(G, blocks, 1, op.near64, s);
    } else {
        op.near_pairs.alloc(pairs.size() * sizeof(NearPair));
        op.near_pairs.upload(reinterpret_cast<const char*>(pairs.data()), pairs.size() * sizeof(NearPair), s);
        const NearPair* pairs_dev = reinterpret_cast<const NearPair*>(op.near_pairs.get());
        HDM_HIP(hipStreamSynchronize(s));   // the host copy of the pairs goes out of scope
        int64_t maxe = 0;
        for (auto& p : pairs) maxe = std::max<int64_t>(maxe, static_cast<int64_t>(p.ld) * p.nb);
        // float32 evaluation tiles are written by the same launch
        float* out32 = nullptr;
        if (op.prm.near_prec == HDM_F32) {
            op.nearT.alloc(static_cast<size_t>(std::max<int64_t>(op.near_elems, 1)) * sizeof(float));
            out32 = reinterpret_cast<float*>(op.nearT.get());
            op.near_converted = true;
        }
        for (size_t base = 0; base < pairs.size(); base += 65535) {
            const int cnt = static_cast<int>(std::min<size_t>(65535, pairs.size() - base));
            hipLaunchKernelGGL(k_near_tiles, dim3(ceil_div(maxe, kBlock), cnt), dim3(kBlock), 0, s,
                               pairs_dev + base, op.perm.get(), P, op.near64.get(), out32);
        }
        check_launch("near tiles");
    }
}

// far tiles (after skeletonisation), left in flight on s; their block
// descriptors go to `keep` (alive until the operator is finished)
static void build_far_tiles(Op& op, const Geo& G, hipStream_t s, DevBuf<char>& keep) {
    const Pts& P = G.P;
    // far blocks: per node, row-major rank x (sum of far ranks)
    op.far_block_off.assign(op.nnodes, 0);
    op.far_cols.assign(op.nnodes, 0);
    op.far_colbase.assign(op.nnodes, 0);
    std::vector<FarBlock> blocks;
    std::vector<int32_t> colmap;
    int64_t foff = 0;
    for (int64_t h = 2; h < op.nnodes; ++h) {
        int32_t cols = 0;
        op.far_colbase[h] = static_cast<int64_t>(colmap.size());
        for (int32_t t = op.far_off[h]; t < op.far_off[h + 1]; ++t) {
            const int32_t g = op.far_idx[t];
            for (int32_t j = 0; j < op.rank[g]; ++j) colmap.push_back(static_cast<int32_t>(op.skoff[g] + j));
            cols += op.rank[g];
        }
        op.far_cols[h] = cols;
        op.far_block_off[h] = foff;
        if (cols > 0 && op.rank[h] > 0)
            blocks.push_back(FarBlock{foff, static_cast<int64_t>(colmap.size()) - cols, op.rank[h], cols, op.skoff[h]});
        foff += static_cast<int64_t>(op.rank[h]) * cols;
    }
    op.far_elems = foff;
    for (const FarBlock& b : blocks)
        HDM_CHECK(b.rows >= 1 && b.cols >= 1 && b.off >= 0 && b.off + static_cast<int64_t>(b.rows) * b.cols <= foff &&
                      b.col0 >= 0 && b.col0 + b.cols <= static_cast<int64_t>(colmap.size()) && b.sk0 >= 0 &&
                      b.sk0 + b.rows <= op.nskel,
                  HDM_EINTERNAL, "far tile descriptor outside its buffers");
    for (int32_t slot : colmap)
        HDM_CHECK(slot >= 0 && slot < op.nskel, HDM_EINTERNAL, "far column map entry outside the skeletons");
    op.far64.alloc(foff > 0 ? foff : 1);
    op.far_colmap = to_device(colmap, s);
    if (G.gram) {
        std::vector<GramBlock> gb;
        for (int64_t h = 2; h < op.nnodes; ++h) {
            if (op.rank[h] == 0) continue;
            int64_t col = 0;
            for (int32_t t = op.far_off[h]; t < op.far_off[h + 1]; ++t) {
                const int32_t g = op.far_idx[t];
                if (op.rank[g] > 0)
                    gb.push_back(GramBlock{op.skel.get() + op.skoff[h], op.skel.get() + op.skoff[g], op.rank[h],
                                           op.rank[g], op.far_block_off[h] + col, op.far_cols[h], 0});
                col += op.rank[g];
            }
        }
        gram_launch(G, gb, 1, op.far64, s);
    } else if (!blocks.empty()) {
        keep.alloc(blocks.size() * sizeof(FarBlock));
        keep.upload(reinterpret_cast<const char*>(blocks.data()), blocks.size() * sizeof(FarBlock), s);
        const FarBlock* db = reinterpret_cast<const FarBlock*>(keep.get());
        int64_t maxe = 0;
        for (auto& b : blocks) maxe = std::max<int64_t>(maxe, static_cast<int64_t>(b.rows) * b.cols);
        for (size_t base = 0; base < blocks.size(); base += 65535) {
            const int cnt = static_cast<int>(std::min<size_t>(65535, blocks.size() - base));
            hipLaunchKernelGGL(k_far_tiles, dim3(ceil_div(maxe, kBlock), cnt), dim3(kBlock), 0, s, db + base,
                               op.far_colmap.get(), op.skel.get(), P, op.far64.get());
        }
        check_launch("far tiles");
    }
}

void near_field_ones(Op& op, hipStream_t s) {
    op.part_ones.alloc(static_cast<size_t>(std::max<int64_t>(op.part_elems_otf, 1)));
    // beside the skeletonisation: at most kOtfSideWgs workgroups per compute unit,
    // so that the ID's workgroups of the levels it overlaps find room (N = 100000:
    // 14.68 -> 14.53 ms per compression; 4 per unit: 14.73)
    constexpr int kOtfSideWgs = 2;
    int dev = 0, ncu = 0;
    HDM_HIP(hipGetDevice(&dev));
    HDM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    near_field_otf(op, nullptr, op.part_ones.get(), s, kOtfSideWgs * ncu);
}

void near_field_otf(const Op& op, const double* w_tree, double* part, hipStream_t s, int max_wgs) {
    HDM_CHECK(op.near_direct && op.xf.get() && op.dim <= kDirectDim, HDM_EINTERNAL,
              "on-the-fly near field needs float64 points of few coordinates");
    Pts P{};
    P.xf = op.xf.get();
    P.dim = op.dim;
    P.is_u8 = 0;
    P.eps = op.prm.eps;
    const int64_t nr = static_cast<int64_t>(op.otf_runs.size());
    if (nr == 0) return;
    const int wpb = kBlock / kWave;
    int64_t grid = ceil_div(nr, wpb);
    if (max_wgs > 0) grid = std::min<int64_t>(grid, max_wgs);
    HDM_DIM_DISPATCH(P.dim, k_near_otf, dim3(static_cast<unsigned>(grid)), dim3(kBlock), 0, s, op.d_items.get(),
                     op.d_otf_runs.get(), nr, op.perm.get(), P, w_tree, part);
    check_launch("near field (kernel on the fly)");
}

// buffers of the build that queued kernels still read when compress_operator
// returns: the skeletonisation run (the compaction) and the far-tile descriptors
struct BuildKeep {
    SkelRun skel;
    DevBuf<char> far_blocks;
};

void compress_operator(Op& op, const void* X, int x_on_device, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const hdm_params& p = op.prm;
    op.n = p.n;
    op.dim = p.dim;
    int depth = 0;
    while ((op.n + (int64_t(1) << depth) - 1) / (int64_t(1) << depth) > p.leaf_m) ++depth;
    op.depth = depth;
    op.L = 1 << depth;
    op.nnodes = int64_t(2) * op.L;
    HDM_CHECK((op.n >> depth) > p.knn_k, HDM_EINVAL, "every leaf must hold more than knn_k points");
    tree_ranges(op.n, depth, op.start, op.size);
    op.d_start = to_device(op.start, s);
    op.d_size = to_device(op.size, s);
    // points
    const size_t xb = static_cast<size_t>(op.n) * op.dim * dtype_size(p.x_dtype);
    const hipMemcpyKind kind = x_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    Geo G;
    Pts& P = G.P;
    P.dim = op.dim;
    P.eps = p.eps;
    if (p.x_dtype == HDM_U8) {
        op.xu.alloc(xb);
        HDM_HIP(hipMemcpyAsync(op.xu.get(), X, xb, kind, s));
        P.xu = op.xu.get();
        P.is_u8 = 1;
        if (op.dim % 16 == 0) {
            G.gram = true;
            G.nu.alloc(op.n);
            G.ns.alloc(op.n);
            hipLaunchKernelGGL(k_code_norms, dim3(ceil_div(op.n, kBlock)), dim3(kBlock), 0, s, op.xu.get(), op.n, op.dim,
                               G.nu.get(), G.ns.get());
            check_launch("code norms");
            P.nu = G.nu.get();
        }
    } else {
        op.xf.alloc(static_cast<size_t>(op.n) * op.dim);
        HDM_HIP(hipMemcpyAsync(op.xf.get(), X, xb, kind, s));
        P.xf = op.xf.get();
        P.is_u8 = 0;
        DevBuf<int> bad(1);
        HDM_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int), s));
        hipLaunchKernelGGL(k_check_points, dim3(ceil_div(static_cast<int64_t>(op.n) * op.dim, kBlock)), dim3(kBlock), 0, s,
                           op.xf.get(), static_cast<int64_t>(op.n) * op.dim, bad.get());
        int hb = 0;
        bad.download(&hb, 1, s);
        HDM_HIP(hipStreamSynchronize(s));
        HDM_CHECK(hb == 0, HDM_EINVAL, "points contain NaN or Inf");
    }
    // trees: the ball tree on the side stream while the neighbour trees run on s
    const int64_t n = op.n;
    op.lane.init(op.ctx ? &op.ctx->lanes : nullptr);
    hipStream_t side = op.lane.side;
    HDM_HIP(hipEventRecord(op.lane.fork, s));
    HDM_HIP(hipStreamWaitEvent(side, op.lane.fork, 0));
    DevBuf<int32_t> perm(n), tmp(n), samp(static_cast<size_t>(op.L) * kSample), nsamp(op.L), pq(2 * op.L);
    DevBuf<double> sumk(n), key(n);
    op.iperm.alloc(n);
    // neighbours: random-pivot trees, all pairs inside leaves
    const int k = p.knn_k;
    op.knn_idx.alloc(static_cast<size_t>(n) * k);
    op.knn_d2.alloc(static_cast<size_t>(n) * k);
    hipLaunchKernelGGL(k_knn_init, dim3(ceil_div(n * k, kBlock)), dim3(kBlock), 0, s, op.knn_idx.get(), op.knn_d2.get(),
                       n * k);
    // all neighbour trees are built together (every level of every tree in one launch);
    // their levels and the ball tree's are issued alternately so both streams start at once
    const int T = p.knn_iters;
    DevBuf<int32_t> kperm(static_cast<size_t>(T) * n), ktmp(static_cast<size_t>(T) * n),
        kpq(static_cast<size_t>(T) * 2 * op.L);
    DevBuf<double> kkey(static_cast<size_t>(T) * n);
    {
        TreeBuild ball(op, 0, 0, 1, perm, tmp, G, side, samp, nsamp, pq, sumk, key);
        std::unique_ptr<TreeBuild> knn;
        if (T > 0) knn.reset(new TreeBuild(op, 1, 0, T, kperm, ktmp, G, s, samp, nsamp, kpq, sumk, kkey));
        for (int lvl = 0; lvl < op.depth; ++lvl) {
            if (knn) knn->level(lvl);
            ball.level(lvl);
        }
    }
    op.perm = std::move(perm);
    hipLaunchKernelGGL(k_inverse_perm, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, side, op.perm.get(),
                       op.iperm.get(), n);
    HDM_HIP(hipEventRecord(op.lane.join, side));
    int64_t leafmax = 0;
    for (int64_t h = op.L; h < 2 * int64_t(op.L); ++h) leafmax = std::max(leafmax, op.size[h]);
    const int stage = (!P.is_u8 && P.dim <= kLeafStageDim && leafmax * P.dim * 8 <= 48 * 1024) ? 1 : 0;
    DevBuf<int32_t> leafd2;
    if (G.gram) leafd2.alloc(static_cast<size_t>(op.L) * leafmax * leafmax);
    const size_t shm = stage ? sizeof(double) * leafmax * P.dim : 0;
    // enough workgroups to cover the device: split each leaf's points over several
    const int splits = std::max(1, std::min(static_cast<int>((leafmax + 15) / 16), 2048 / op.L));
    for (int it = 0; it < T; ++it) {
        const int32_t* tperm = kperm.get() + static_cast<int64_t>(it) * n;   // tree it's permutation
        if (G.gram) {
            std::vector<GramBlock> blocks;
            for (int64_t h = op.L; h < 2 * int64_t(op.L); ++h)
                blocks.push_back(GramBlock{tperm + op.start[h], tperm + op.start[h],
                                           static_cast<int32_t>(op.size[h]), static_cast<int32_t>(op.size[h]),
                                           (h - op.L) * leafmax * leafmax, static_cast<int32_t>(leafmax), 0});
            gram_launch(G, blocks, 0, leafd2, s);
        }
        hipLaunchKernelGGL(k_knn_leaf, dim3(op.L * splits), dim3(kKnnBlock), shm, s, op.depth, op.d_start.get(),
                           op.d_size.get(), tperm, P, k, stage, splits, G.gram ? leafd2.get() : nullptr,
                           static_cast<int>(leafmax), op.knn_idx.get(), op.knn_d2.get());
        check_launch("knn leaf");
    }
    // neighbour votes between leaves on the side stream (after the ball tree there
    // and the neighbours on s); the skeletonisation levels are enqueued on s, and
    // the host builds the interaction lists while they run
    HDM_HIP(hipEventRecord(op.lane.fork, s));
    HDM_HIP(hipStreamWaitEvent(s, op.lane.join, 0));   // the ball tree and its inverse permutation
    HDM_HIP(hipStreamWaitEvent(side, op.lane.fork, 0));
    DevBuf<int32_t> votes(static_cast<size_t>(op.L) * op.L), leaf_of(n);
    hipLaunchKernelGGL(k_leaf_of, dim3(op.L), dim3(kBlock), 0, side, op.depth, op.d_start.get(), op.d_size.get(),
                       leaf_of.get());
    if (op.L <= 8192) {
        hipLaunchKernelGGL(k_votes<false>, dim3(op.L), dim3(kBlock), sizeof(int32_t) * static_cast<size_t>(op.L), side,
                           op.depth, op.d_start.get(), op.d_size.get(), op.perm.get(), op.iperm.get(),
                           op.knn_idx.get(), k, leaf_of.get(), votes.get());
    } else {
        HDM_HIP(hipMemsetAsync(votes.get(), 0, votes.bytes(), side));
        hipLaunchKernelGGL(k_votes<true>, dim3(op.L), dim3(kBlock), 0, side, op.depth, op.d_start.get(),
                           op.d_size.get(), op.perm.get(), op.iperm.get(), op.knn_idx.get(), k, leaf_of.get(),
                           votes.get());
    }
    check_launch("votes");
    auto keep = std::make_shared<BuildKeep>();
    SkelRun& skr = keep->skel;
    hipEvent_t gate = nullptr;
    HDM_HIP(hipEventCreateWithFlags(&gate, hipEventDisableTiming));
    struct EventGuard {
        hipEvent_t e;
        ~EventGuard() { (void)hipEventDestroy(e); }
    } gate_guard{gate};
    skeletonize_levels(op, G, s, skr, gate);
    {
        // through pinned staging when there is some: a pageable download took
        // hundreds of microseconds longer to come back
        std::vector<int32_t> hv(static_cast<size_t>(op.L) * op.L);
        if (void* pin = host_stage(hv.size() * sizeof(int32_t))) {
            votes.download(static_cast<int32_t*>(pin), hv.size(), side);
            HDM_HIP(hipStreamSynchronize(side));
            std::memcpy(hv.data(), pin, hv.size() * sizeof(int32_t));
        } else {
            votes.download(hv.data(), hv.size(), side);
            HDM_HIP(hipStreamSynchronize(side));
        }
        build_near_lists(op, hv);
        build_far_lists(op);
    }
    // near tiles and their evaluation-precision copy on the side stream
    // the main stream waits for the float64 tiles and the near plan only (the
    // degree products need them); their conversion to the evaluation precision
    // runs on through the far tiles and the degrees, and finish_operator waits
    HDM_HIP(hipStreamWaitEvent(side, gate, 0));
    build_near_tiles(op, G, side);
    build_near_plan(op, side);
    if (op.near_direct) near_field_ones(op, side);   // the near part of K~ 1, beside the skeletonisation
    HDM_HIP(hipEventRecord(op.lane.ready, side));
    convert_near_tiles(op, side);
    skeletonize_finish(op, s, skr);
    HDM_HIP(hipStreamWaitEvent(s, op.lane.ready, 0));
    build_far_tiles(op, G, s, keep->far_blocks);
    op.build_keep = keep;   // released by finish_operator after it has waited for s
    op.seconds_compress = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace hdm
