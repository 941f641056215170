// The compressed operator resident in HBM, and the launch plans that apply it.
#pragma once

#include <chrono>
#include <memory>
#include <mutex>

#include <hip/hip_ext.h>

#include "common.hpp"

struct hdm_ctx_s;
struct hdm_op_s;

namespace hdm {

// HIP-event pairs around phase launches, accumulated per phase.
struct Profiler {
    bool on = false;
    uint32_t mask = ~0u;                         // phases recorded while on (bit 1 << hdm_phase)
    bool records(int phase) const { return on && ((mask >> phase) & 1u); }
    std::mutex mu;                               // several host threads may record
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Mark { int phase; size_t a, b; };
    std::vector<Mark> marks;   // phase with the pool indices of its start and end events
    hipEvent_t take();
    void begin(int phase, hipStream_t s, size_t& slot);
    void end(size_t slot, hipStream_t s) noexcept;
    // events for hipExtLaunchKernelGGL: they take the kernel's own start and end times
    void kernel_events(int phase, hipEvent_t& start, hipEvent_t& stop);
    void totals(int64_t* launches, double* ms);
    void reset() { used = 0; marks.clear(); }
    ~Profiler();
};

// Side streams with their fork/join events, kept by a context for its next
// operators: creating and destroying a stream costs ~60-80 us each.
struct LanePool {
    struct Entry {
        hipStream_t side;
        hipEvent_t fork, join, ready;
    };
    std::mutex mu;
    std::vector<Entry> free;
    ~LanePool();
};

struct Ctx {
    int device = 0;
    size_t budget = 0;      // bytes, 0 = unlimited
    size_t resident = 0;    // bytes held by live operators of this context
    bool graphs = false;    // hdm_matvec replays a HIP graph (hdm_ctx_graphs)
    Profiler prof;
    LanePool lanes;
};

// start/stop events of one profiled kernel launch (both null unless the context profiles)
struct KernelEvents {
    hipEvent_t start = nullptr, stop = nullptr;
    KernelEvents(Ctx* c, int phase) {
        if (c && c->prof.records(phase)) c->prof.kernel_events(phase, start, stop);
    }
};

// scoped phase interval on a stream (no-op unless the context profiles)
struct PhaseScope {
    Profiler* p;
    hipStream_t s;
    size_t slot = 0;
    PhaseScope(Ctx* c, int phase, hipStream_t st) : p(c && c->prof.records(phase) ? &c->prof : nullptr), s(st) {
        if (p) p->begin(phase, s, slot);
    }
    ~PhaseScope() {
        if (p) p->end(slot, s);
    }
};

// One streaming work item of the near-field product: ncols consecutive
// columns (one near tile) times the rows [row0, row0 + nrows) of leaf a's near
// block.  Column c of the item multiplies w at tree position col_pos + c.
struct NearItem {
    int64_t tile_off;   // element offset of the item's first column, row 0, in the near buffer
    int64_t part_off;   // offset of the item's partial sums (nrows_ld values)
    int32_t ld;         // leading dimension (padded rows) of the leaf's near block
    int32_t row0;       // first row of the item (multiple of the row group)
    int32_t ncols;
    int32_t col_pos;    // tree position of the first column's point
    int32_t tile;       // index of the near tile (for its scale)
    int32_t nrows;      // rows of the item: [row0, min(ld, row0 + nrows))
    int32_t leaf_b;     // column leaf (matrix-core items: index of its vector scales)
    int32_t row_pos;    // tree position of the row leaf's first point (plain items)
    int32_t row_n;      // points in the row leaf (rows at or past it are padding)
    int32_t ntiles;     // matrix-core items: consecutive near tiles from `tile` on (one per tile record)
    int32_t kbeg;       // matrix-core segments: first column taken of the first tile (a multiple of 32)
    int32_t kend;       // matrix-core segments: end of the columns taken of the last tile
};

// float64 products of operators whose near tiles are made directly in the
// evaluation precision evaluate the near field on the fly; each wave takes a
// run of consecutive plain items of one leaf and row group and writes one
// partial-sum slot for the run (fewer slots for the combine to add)
struct OtfRun {
    int64_t part_off;   // the run's partial-sum slot (ld rows of its leaf)
    int32_t item;       // its first plain item
    int32_t count;      // consecutive plain items of the same leaf and row group
};

// Per leaf: where its partial sums live and how many items feed each row group.
struct LeafPlan {
    int64_t part_off;   // first partial of the leaf
    int32_t nitems;     // items per row group of this leaf (same for each group)
    int32_t ld;
    int32_t start;      // tree position of row 0
    int32_t rows;       // points in the leaf
    int32_t heap;       // heap id
    int32_t ngroups;    // row groups
    int64_t wpad;       // matrix-core plans: offset of the leaf in the padded half-precision vectors
    int32_t gstep;      // products of several columns: its partial sums pre-added in groups of gstep items
};

// partial sums of a leaf with more than kReduceAbove near-field items are
// pre-added in groups of kReduceGroup (products of several columns)
constexpr int kReduceAbove = 16;
constexpr int kReduceGroup = 8;

// one skeleton row: heap id and row index
struct RowTask {
    int32_t h, i;
};

constexpr int kMaxLevels = 17;   // tree depth <= 16
constexpr int kMaxRhs = 16;      // right-hand sides per pass of a product (more are taken in passes)

// Everything a product kernel needs about one operator, resident in device
// memory next to it.  Two copies exist per operator: one for the float64 tiles
// (the degree products) and one for the evaluation precision.
struct OpDev {
    int64_t n;
    int32_t depth, L;
    const int32_t* perm;
    const double* c;              // alpha = 1 scale, tree order
    const int64_t* start;
    const int32_t* rank;
    const int32_t* ncand;
    const int64_t* skoff;
    const int64_t* poff;
    const void* P;
    const RowTask* rows;          // skeleton rows grouped by level (leaves first)
    int64_t row_begin[kMaxLevels];
    int64_t row_count[kMaxLevels];
    int64_t row_total;
    const int64_t* far_off;
    const int32_t* far_cols;
    const int64_t* far_colbase;
    const int32_t* far_colmap;
    const void* far;
    const float* fscale;
    const NearItem* items;        // work items and per-leaf plans of products of several columns
    int64_t nitems;
    const LeafPlan* leaves;
    int64_t ldp;                  // column stride of the partial sums
    const NearItem* items1;       // the same for one column (the plain plan: the same arrays)
    int64_t nitems1;
    const LeafPlan* leaves1;
    int64_t ldp1;
    const NearItem* tiles;        // matrix-core plans: one record per near tile (items take runs of them)
    const int32_t* wseg;          // matrix-core plans: first segment of each workgroup (several columns)
    const int32_t* wseg1;         // the same for one column
    const void* near;
    const float* nscale;
    void* w;                      // workspaces (nrhs columns each)
    void* skw;
    void* sku;
    void* part;
    int64_t ldsk;
    // half-precision near field on matrix cores: the staged vectors (hi and lo
    // halves, 16 right-hand sides, leaves padded to 8 points) and their per
    // leaf, per column scales
    void* wh;
    float* wsc;
    int64_t ldw;
    const void* comp;             // composites of the nested bases (nullptr: level by level)
    int32_t s2n_levels;           // 1: the downward pass runs level by level before the combine
    int32_t s2n_multi;            // the same for products with several right-hand sides
    int32_t s2n_comp;             // several right-hand sides: the combine forms each leaf's potentials
                                  // from its ancestors' far fields through the composites
    int32_t s2n_comp1;            // the same for one right-hand side
    const int64_t* coff;
};

// A side stream with its fork/join events: the upward pass and the far field
// run there while the near field streams on the caller's stream.
struct Lane {
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    hipEvent_t ready = nullptr;   // operator build: float64 near tiles and near plan on the side stream
    LanePool* pool = nullptr;   // where the stream and events go back to (null: destroyed)
    void init(LanePool* from = nullptr);
    Lane() = default;
    Lane(const Lane&) = delete;
    Lane& operator=(const Lane&) = delete;
    ~Lane();
};

struct Op {
    Ctx* ctx = nullptr;
    hdm_params prm{};
    int64_t n = 0;
    int dim = 0, depth = 0, L = 0;
    int64_t nnodes = 0;                  // 2L heap slots (slot 0 unused)
    std::vector<int64_t> start, size;    // per heap id
    DevBuf<int64_t> d_start, d_size;
    DevBuf<double> xf;                   // points, original order (float64)
    DevBuf<uint8_t> xu;                  // points, original order (u8 codes)
    DevBuf<int32_t> perm, iperm;         // tree position -> original index, and back
    DevBuf<int32_t> knn_idx;             // n x k (original order)
    DevBuf<double> knn_d2;
    // interaction lists (host copies are the source of truth for planning)
    std::vector<int32_t> near_off, near_idx, far_off, far_idx;
    // skeletons
    std::vector<int32_t> rank, ncand, nrows;   // per heap id
    std::vector<int64_t> skoff;                // per heap id: offset into skeleton arrays (children adjacent)
    int64_t nskel = 0;
    DevBuf<int32_t> skel;                      // original indices, by skoff
    std::vector<int64_t> poff;                 // per heap id: offset of P (rank x ncand, row-major)
    int64_t np = 0;
    DevBuf<double> P64;
    DevBuf<float> P32;
    std::vector<int64_t> rowoff;               // per heap id: offset of sampled rows
    DevBuf<int32_t> rows;
    // near field: per leaf a column-major block ld x (sum of near leaf sizes)
    std::vector<int64_t> near_block_off;       // per leaf (elements)
    std::vector<int32_t> near_ld;              // per leaf
    std::vector<int64_t> near_tile_off;        // per near pair (elements; same order as near_idx)
    int64_t near_elems = 0;
    mutable unsigned near_calls = 0;           // near-field products so far (their tile order alternates)
    DevBuf<char> near_pairs;                   // pair descriptors of the near-tile launch, until finish_operator
    std::shared_ptr<void> build_keep;          // build buffers read by work still queued, until finish_operator
    DevBuf<double> near64;
    DevBuf<char> nearT;                        // eval precision copy (near_prec)
    DevBuf<float> near_scale;                  // per near pair
    // far field: per node a row-major block rank x (sum of far ranks)
    std::vector<int64_t> far_block_off;        // per heap id
    std::vector<int32_t> far_cols;             // per heap id
    int64_t far_elems = 0;
    DevBuf<double> far64;
    DevBuf<char> farT;
    DevBuf<float> far_scale;                   // per heap id (one scale per block)
    DevBuf<int32_t> far_colmap;                // per block column: skeleton slot of the weight it multiplies
    std::vector<int64_t> far_colbase;          // per heap id: first column of its block in far_colmap
    const int64_t* d_far_colbase = nullptr;     // in plan_blob
    // plans
    std::vector<NearItem> items;
    DevBuf<NearItem> d_items;
    std::vector<LeafPlan> leaves;
    DevBuf<LeafPlan> d_leaves;
    int64_t part_elems = 0;
    // runs of the on-the-fly float64 near field and their leaf plans
    std::vector<OtfRun> otf_runs;
    DevBuf<OtfRun> d_otf_runs;
    std::vector<LeafPlan> leaves_otf;
    DevBuf<LeafPlan> d_leaves_otf;
    int64_t part_elems_otf = 0;
    int near_rows_per_group = 256;
    // half-precision near tiles are packed for the matrix cores (evaluate.hip):
    // their own tile offsets, items, leaf plans and partial-sum extent
    bool packed = false;
    std::vector<int64_t> near_tile_off_mma;
    // packed (matrix-core) plans, [0] for one right-hand side, [1] for several
    // (each a list of segments, every workgroup an equal share of the tile steps)
    int64_t near_elems_mma = 0, part_elems_mma[2] = {0, 0};
    int red_groups = 0, red_groups_mma[2] = {0, 0};   // most pre-added groups of one leaf (plain, packed plans)
    std::vector<NearItem> items_mma[2], tiles_mma;
    DevBuf<NearItem> d_items_mma[2], d_tiles_mma;
    std::vector<LeafPlan> leaves_mma[2];
    DevBuf<LeafPlan> d_leaves_mma[2];
    std::vector<int32_t> wseg_mma[2];   // per workgroup of the packed near field: its first segment (+ end)
    DevBuf<int32_t> d_wseg_mma[2];
    bool wseg_one[2] = {false, false};  // one segment per workgroup (the kernel takes no list)
    int64_t ldw = 0;
    DevBuf<char> wh;                           // 2 x 16 x ldw halves
    DevBuf<float> wsc;                         // L x 16
    // near tiles converted to the evaluation precision early (while the skeletons
    // are computed); the conversion's staging buffers live until it has completed
    bool near_converted = false;
    // near tiles written directly in the evaluation precision (no float64 copy);
    // the float64 degree products evaluate the kernel on the fly (compress.hip)
    bool near_direct = false;
    // with near_direct: the near field of K~ 1 (the first degree product), computed
    // on the side stream while the skeletons are found, and taken by that product
    DevBuf<double> part_ones;
    bool near_ones_next = false;
    struct ConvKeep {
        std::vector<DevBuf<int64_t>> d64;
        std::vector<DevBuf<int32_t>> d32;
        std::vector<std::vector<int64_t>> h64;
        std::vector<std::vector<int32_t>> h32;
    };
    std::unique_ptr<ConvKeep> conv_keep;
    // HIP graphs of the single-operator product, one per (precision path,
    // normalised, right-hand sides, profiled) (evaluate.hip)
    struct GraphCache;
    GraphCache* graphs = nullptr;
    // skeleton-dependent plan arrays, uploaded together into plan_blob
    DevBuf<char> plan_blob;
    const int32_t* d_rank = nullptr;
    const int32_t* d_ncand = nullptr;
    const int64_t* d_skoff = nullptr;
    const int64_t* d_poff = nullptr;
    const int64_t* d_far_block_off = nullptr;
    const int32_t* d_far_cols = nullptr;
    std::vector<int64_t> row_begin, row_count; // per level: skeleton-row tasks of the upward pass
    int64_t row_total = 0;
    const RowTask* d_row_tasks = nullptr;   // in plan_blob
    Lane lane;                                 // side stream of single-operator products
    OpDev host64{}, hostT{};                   // descriptors (host copies)
    DevBuf<OpDev> dev64, devT;                 // the same, in device memory
    // normalisation (tree order)
    DevBuf<double> q, d, c;
    // workspaces of the product
    int ws_nrhs = 0;
    DevBuf<char> w_tree, skw, sku, part;
    // composites of the nested bases: per inner node below the root, the
    // rank x (leaf skeletons under it) map from the leaves' skeleton weights to
    // its own; none where they would outweigh P (the upper levels then run level
    // by level)
    std::vector<int64_t> coff;                 // per heap id
    int64_t ncomp = 0;
    bool s2n_levels = false;   // downward pass in per-level launches (large ranks) instead of per leaf path
    bool s2n_multi = false;    // the same for several right-hand sides (every nested tree of depth >= 2)
    // several right-hand sides in evaluation precision: the leaf potentials through
    // the composites inside the combine (no per-level launches), where they fit
    bool s2n_comp = false;
    // the downward pass of a product runs in per-level launches
    bool s2n_by_levels(bool multi, bool f64) const { return multi ? s2n_multi && !(s2n_comp && !f64) : s2n_levels; }
    int max_leaf_rank = 0;
    // one right-hand side through the composites: the largest shared-memory staging
    // of any leaf (its ancestors' far fields and composite blocks, the per-level sums)
    int64_t comp1_stage = 0;
    std::vector<int32_t> lvl_max_nc, lvl_max_rank;   // per tree level: largest candidate count and rank
    DevBuf<double> C64;
    DevBuf<float> C32;
    const int64_t* d_coff = nullptr;           // in plan_blob
    double seconds_compress = 0.0;
    size_t footprint() const;
    Op() = default;
    Op(const Op&) = delete;
    Op& operator=(const Op&) = delete;
    ~Op();
};

// one operand of a batched product
struct ApplyReq {
    Op* op;
    const double* x;
    double* y;
    const OpDev* desc = nullptr;   // device descriptor to launch with (nullptr: the operator's own)
};

// One Lanczos eigensolve (Sec. 2.2) that advances a step at a time: the caller
// applies the normalised operator to current() into output() (possibly in a
// batch with other solves), then after_product() reorthogonalises and, every
// few steps, checks the Ritz pairs.  result() forms the Ritz vectors.
struct LanczosRun {
    Op* op = nullptr;
    int r = 0, max_basis = 0, check_every = 5;
    double tol = 0.0;
    uint64_t seed = 0;
    int64_t n = 0;
    int nb = 0, ldp = 0;
    DevBuf<double> V, y, part, h1, h2, np, alpha, beta, theta, bound, Y;
    DevBuf<unsigned> counters;   // arrival counters of the last-workgroup reductions (zero between launches)
    std::vector<double> h_theta, h_bound;
    int j = 0, m = 0, matvecs = 0;
    bool converged = false, finished = false;
    std::chrono::steady_clock::time_point t0;
    // thick restart (Sec. 2.2, implicitly restarted Lanczos with exact shifts):
    // when the basis is full and the pairs have not converged, the leading `keep`
    // Ritz vectors and the last Lanczos vector become the new basis (at most
    // max_restarts times; 0 = no restarts, the basis limit ends the solve)
    int max_restarts = 0, restarts = 0, keep = 0;
    bool restarted = false;                    // the projected matrix is no longer tridiagonal
    DevBuf<double> T, A, dd, ee, tau, tmp;     // projected matrix, its reduction, the new basis
    void restart(hipStream_t s);
    void solve_projected(int nvec, hipStream_t s);   // Ritz pairs of the restarted projected matrix
    void start(Op& op, int r, double tol, int max_basis, uint64_t seed, hipStream_t s);
    const double* current() const { return V.get() + static_cast<int64_t>(j) * n; }
    double* output() { return y.get(); }
    bool after_product(hipStream_t s);   // true once finished
    hdm_status result(double* evals, double* evecs, hdm_eig_info_t* info, hipStream_t s);
    size_t bytes() const;
};

// message of the last failure on the calling thread (hdm_last_error)
void set_last_error(const char* msg);

// builds a compressed, normalised operator (validation, compression, plan,
// degrees, precision conversion); the caller owns the result (api.cpp)
void validate_params(const hdm_params& p);
hdm_op_s* make_operator(Ctx* ctx, const void* X, int x_on_device, const hdm_params& p, hipStream_t s);
// upper bound of the device memory one request of the serving loop holds at its peak
size_t footprint_estimate(const hdm_params& p, int max_basis);

// compression (compress.hip)
void compress_operator(Op& op, const void* X, int x_on_device, hipStream_t s);
// float64 near field of one column with the kernel evaluated on the fly from the
// points (operators with near_direct): part[item] = K(rows, cols) w over the
// plain work items, w and part the product's float64 workspaces
void near_field_otf(const Op& op, const double* w_tree, double* part, hipStream_t s, int max_wgs = 0);
// the same with w = 1 into op.part_ones (launched on the side stream after the near plan)
void near_field_ones(Op& op, hipStream_t s);
// offsets of the packed half-precision near tiles (evaluate.hip)
void packed_near_offsets(Op& op);
// evaluation (evaluate.hip)
void build_near_plan(Op& op, hipStream_t s);
void build_eval_plan(Op& op, hipStream_t s);
void normalise_degrees(Op& op, hipStream_t s);
// evaluation-precision copies of the tiles and P, enqueued on s without waiting
void convert_eval_precision(Op& op, hipStream_t s);
// waits for s, releases the float64 tiles (unless they are the evaluation tiles)
// and publishes the descriptors
void finish_operator(Op& op, hipStream_t s);
// starts the conversion of the float64 near tiles to the evaluation precision
// on s without waiting (its index arrays live in conv_keep until finish_operator)
void convert_near_tiles(Op& op, hipStream_t s);
// graph_ok: the product may replay the operator's cached HIP graph (the caller's
// one-off products); iterations that interleave other kernels launch eagerly.
// tree_order: x and y are in the tree's point order (no gather or scatter; the
// block eigensolver keeps its basis that way)
void apply(Op& op, int normalised, bool exact64, const double* x, double* y, int nrhs, hipStream_t s,
           bool graph_ok = false, bool tree_order = false);
// One launch per phase for every operator of the batch (same tile precisions,
// at most kMaxBatch operators, one nrhs); each operator's result is the one a
// single-operator product gives.
constexpr int kMaxBatch = 8;
void apply_batch(const ApplyReq* reqs, int nops, int normalised, int nrhs, hipStream_t s, Lane& lane, Ctx* prof_ctx);
// Allocation-free products (evaluate.hip): a file-scope device array holds the
// product's workspaces and a copy of the descriptor.  scratch_init resolves its
// address on the current device (once per device, at context creation);
// scratch_for returns it (nullptr before scratch_init).
constexpr size_t kScratchBytes = size_t(64) << 20;
void scratch_init(int device);
void* scratch_for(int device);
// bytes of scratch a product of `per` right-hand sides per pass needs
size_t noalloc_bytes(const Op& op, int per);
void apply_noalloc(Op& op, int normalised, const double* x, double* y, int nrhs, hipStream_t s, void* scratch);
// eigensolver (lanczos.hip)
hdm_status lanczos_eigs(Op& op, int r, double tol, int block, int max_basis, uint64_t seed, double* evals,
                        double* evecs, hdm_eig_info_t* info, hipStream_t s);
// diffusion-map outputs from the eigenpairs of S~ (lanczos.hip)
hdm_status diffusion_map(Op& op, int r, const double* evals, const double* phi, int t, double delta, double* psi,
                         double* coords, double* evals_t, int32_t* dim_t, hipStream_t s);

}  // namespace hdm

// the opaque handles of the C ABI are the internal objects
struct hdm_ctx_s : hdm::Ctx {};
struct hdm_op_s : hdm::Op {};
