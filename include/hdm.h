/*
 * hdm.h -- C ABI of the MI355X hierarchical diffusion-maps library (libhdm.so).
 *
 * The library computes the leading eigenpairs of the diffusion-maps operator of
 * a point cloud (Sec. 2.1, Alg. 1 with alpha = 1) by Lanczos iteration (Sec. 2.2)
 * over a hierarchical approximation K~ = D + S + UV of the Gaussian kernel matrix
 * (Eq. (2), Eq. (3)), compressed once and applied once per iteration (Sec. 1.2).
 *
 * Conventions for every entry point:
 *  - The return value is an hdm_status; HDM_OK is 0.  On any other value the
 *    outputs are left untouched and hdm_last_error() describes the failure.
 *  - No C++ exception crosses this boundary.
 *  - Vectors at the boundary are float64, in the caller's original point order,
 *    column-major with leading dimension n when several right-hand sides are
 *    passed.  The tree permutation is internal.
 *  - "device" pointers are HIP device memory of the context's GPU; "host"
 *    pointers are ordinary host memory.  The caller owns every buffer it passes.
 *  - stream: a hipStream_t (NULL = the default stream).  Calls that return
 *    results in host memory synchronise that stream before returning.
 *  - One hdm_ctx and the operators made from it are used by one thread at a
 *    time.  The server calls are thread-safe.
 */
#ifndef HDM_H
#define HDM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HDM_OK = 0,
    HDM_EINVAL = 1,      /* bad argument, size or parameter; NaN/Inf in the points */
    HDM_ENOMEM = 2,      /* device or host allocation failed, or over the context budget */
    HDM_EDEVICE = 3,     /* a HIP call failed */
    HDM_ENOCONV = 4,     /* Lanczos stopped at max_basis before the tolerance was met */
    HDM_EBUSY = 5,       /* request still pending (hdm_poll) */
    HDM_ECANCELLED = 6,  /* request cancelled */
    HDM_EINTERNAL = 7,   /* internal invariant violated */
    HDM_ENUMERIC = 8     /* non-positive degree in the normalisation */
} hdm_status;

typedef enum { HDM_F64 = 0, HDM_F32 = 1, HDM_BF16 = 2, HDM_F16 = 3, HDM_U8 = 4 } hdm_dtype;

typedef struct hdm_ctx_s *hdm_ctx;
typedef struct hdm_op_s *hdm_op;
typedef struct hdm_server_s *hdm_server;

/* Problem statement: points X and bandwidth eps (Eq. (2), eps = sigma^2), the
 * density parameter alpha (Alg. 1; only 1 is supported), and the compression
 * parameters of Sec. 4.2.3: leaf size m, maximal off-diagonal rank s,
 * tolerance tau, neighbour count k. */
typedef struct {
    int64_t n;          /* number of points, >= 2 */
    int32_t dim;        /* coordinates per point, >= 1 */
    int32_t x_dtype;    /* HDM_F64 (n x dim row-major doubles) or HDM_U8 (codes k meaning k/255) */
    double eps;         /* > 0 */
    double alpha;       /* must be 1 */
    int32_t leaf_m;     /* leaf size bound: depth = min d with ceil(n / 2^d) <= m; every leaf must hold > knn_k points */
    int32_t max_rank_s; /* 1..1024; above 512 only with leaves of at most 512 points
                           (ceil(n / 2^depth) <= 512); with HDM_U8 points at most the
                           smallest leaf size (floor(n / 2^depth)): other values are
                           refused (HDM_EINVAL) */
    double tau;         /* >= 0, relative pivot threshold of the interpolative decomposition */
    int32_t knn_k;      /* neighbours per point, 1..64 */
    int32_t knn_iters;  /* random trees for the neighbour search, >= 1 (10) */
    double budget;      /* fraction of leaves added to each near list, in [0, 1] (0.05) */
    int32_t near_prec;  /* HDM_F64, HDM_F32, HDM_BF16 or HDM_F16: near-field tiles */
    int32_t far_prec;   /* HDM_F64, HDM_F32, HDM_BF16 or HDM_F16: skeleton tiles */
    uint64_t seed;      /* all random choices are Philox4x32-10 draws keyed by this seed */
} hdm_params;

/* Fills p with the defaults (alpha 1, knn_iters 10, budget 0.05, f32 tiles). */
void hdm_params_default(hdm_params *p);
/* The parameter checks of hdm_compress and hdm_submit alone (no device is
 * touched): HDM_OK, or HDM_EINVAL with hdm_last_error() naming the rule. */
hdm_status hdm_params_validate(const hdm_params *p);

typedef struct {
    int64_t n;
    int32_t dim, depth, leaves, knn_k;
    int32_t max_rank, min_leaf_rank;
    double mean_leaf_rank;
    int64_t near_pairs, far_pairs;
    int64_t bytes_near, bytes_far, bytes_p, bytes_total;  /* resident operator bytes in HBM */
    int64_t algo_bytes_matvec;   /* bytes one single-vector product must move (tiles once + vectors) */
    int64_t algo_bytes_near;     /* of which the near-field launch: unpadded near tiles, its input and output
                                    vectors, and the leaf level of the upward pass it carries (the leaves' P
                                    once, their skeleton weights written) */
    int64_t flops_matvec;        /* 2 x multiply-adds of one single-vector product */
    double seconds_compress;     /* wall time of hdm_compress */
    int64_t near_tile_bytes;     /* unpadded near tiles in the evaluation precision (read once per product pass) */
    int64_t near_elems;          /* unpadded near-tile elements (multiply-adds per right-hand side) */
} hdm_op_stats_t;

typedef struct {
    int32_t iters;        /* Lanczos steps (block steps when block > 1) */
    int32_t matvecs;      /* operator applications (vectors) */
    int32_t converged;    /* 1 when every requested pair met the tolerance */
    double max_rel_resid; /* max_i |beta_j y_{j,i}| / |theta_i| at exit */
    double seconds;
} hdm_eig_info_t;

/* Phases timed by the context profiler (hdm_ctx_profile). */
typedef enum {
    HDM_PHASE_PREP = 0,      /* gather + scale of the input vector into tree order */
    HDM_PHASE_N2S = 1,       /* upward pass: skeleton weights */
    HDM_PHASE_S2S = 2,       /* far field between skeletons */
    HDM_PHASE_S2N = 3,       /* downward pass over inner levels */
    HDM_PHASE_L2L = 4,       /* near field: streams the near tiles */
    HDM_PHASE_COMBINE = 5,   /* near partial sums + leaf downward pass + scatter */
    HDM_PHASE_ORTHO = 6,     /* Lanczos reorthogonalisation and norms */
    HDM_PHASE_TRIDIAG = 7,   /* tridiagonal eigensolve */
    HDM_PHASE_COMPRESS = 8,  /* whole compression (one interval per hdm_compress) */
    HDM_PHASE_COUNT = 9
} hdm_phase;

typedef struct {
    int64_t launches[HDM_PHASE_COUNT];  /* intervals recorded per phase */
    double ms[HDM_PHASE_COUNT];         /* summed GPU time per phase (HIP events on the launch stream) */
} hdm_phase_times_t;

/* ---- context -------------------------------------------------------------- */
/* device: HIP ordinal.  hbm_budget_bytes: cap on operator memory (0 = no cap). */
hdm_status hdm_ctx_create(int device, size_t hbm_budget_bytes, hdm_ctx *out);
hdm_status hdm_ctx_destroy(hdm_ctx ctx);
/* Message of the last failure on the calling thread (valid until its next call). */
const char *hdm_last_error(void);
/* Version string of the library. */
const char *hdm_version(void);
/* enable = 1 clears the per-phase totals and starts recording a pair of HIP
 * events around every phase launched through this context; enable = 0 stops. */
hdm_status hdm_ctx_profile(hdm_ctx ctx, int enable);
/* As hdm_ctx_profile(ctx, 1), but only the phases p with bit (1u << p) set in
 * phase_mask are timed (the others run without events); phase_mask = 0 stops. */
hdm_status hdm_ctx_profile_phases(hdm_ctx ctx, uint32_t phase_mask);
/* Synchronises the recorded events and returns the per-phase totals since the
 * last hdm_ctx_profile(ctx, 1). */
hdm_status hdm_ctx_phase_times(hdm_ctx ctx, hdm_phase_times_t *out);
/* enable = 1: hdm_matvec replays a HIP graph of the product's kernels, built on
 * the operator's first hdm_matvec of each kind (normalised, right-hand sides per
 * pass) and kept until the operator is destroyed; only the vector arguments
 * change between replays.  enable = 0 (the default), and any product while the
 * context profiles (hdm_ctx_profile), launches the kernels one by one, each
 * timed by its own start and end stamps.  The products inside hdm_eigs always
 * launch one by one.  Both give bit-identical results.  On MI355X the replay
 * (135 us per product at N = 32768) is slower than the direct launches
 * (127 us); it saves host work where the host is the bottleneck.  Takes effect
 * on the next product. */
hdm_status hdm_ctx_graphs(hdm_ctx ctx, int enable);

/* ---- compression (Sec. 1.2 "compressed once"; Eq. (3)) ---------------------
 * Builds the kernel-space ball tree, the randomized-tree neighbour lists, the
 * near and far interaction lists, the nested skeletons with their interpolation
 * matrices, the near and skeleton kernel tiles, and the alpha = 1 degrees of K~
 * (two float64 products), all on the GPU.  X: n x dim, row-major, host or device
 * memory (x_on_device).  X is copied; the caller may free it on return. */
hdm_status hdm_compress(hdm_ctx ctx, const void *X, int x_on_device, const hdm_params *params, void *stream,
                        hdm_op *out);
hdm_status hdm_op_destroy(hdm_op op);
hdm_status hdm_op_stats(hdm_op op, hdm_op_stats_t *out);

/* ---- inspection (host outputs) -------------------------------------------- */
/* perm[t] = original index of the point at tree position t (n entries). */
hdm_status hdm_op_perm(hdm_op op, int32_t *perm);
/* Neighbour lists in original order: idx n x k, d2 n x k (squared distances),
 * each row ascending by (d2, index).  Either pointer may be NULL. */
hdm_status hdm_op_knn(hdm_op op, int32_t *idx, double *d2);
/* Interaction lists.  Near: CSR over leaves 0..L-1 (near_off L+1 entries).
 * Far: CSR over heap ids 0..2L-1 (far_off 2L+1 entries; root 1, children 2h, 2h+1).
 * Call with NULL arrays to get the sizes in *near_nnz / *far_nnz. */
hdm_status hdm_op_lists(hdm_op op, int32_t *near_off, int32_t *near_idx, int64_t *near_nnz, int32_t *far_off,
                        int32_t *far_idx, int64_t *far_nnz);
/* Per heap id (2L entries): rank, candidate count and sampled-row count. */
hdm_status hdm_op_ranks(hdm_op op, int32_t *rank, int32_t *ncand, int32_t *nrows);
/* Skeleton of heap node h (rank original indices), its sampled rows (nrows
 * original indices) and its interpolation matrix P (rank x ncand row-major,
 * float64).  Any pointer may be NULL. */
hdm_status hdm_op_node(hdm_op op, int64_t h, int32_t *skel, int32_t *rows, double *P);
/* Degrees of the alpha = 1 normalisation in original order (host, n each):
 * q = K~ 1, d = Q^-1 K~ Q^-1 1, c = 1 / (q sqrt(d)).  Any pointer may be NULL. */
hdm_status hdm_op_degrees(hdm_op op, double *q, double *d, double *c);

/* ---- evaluation (Eq. (3); called once per Lanczos step) --------------------
 * y = K~ x (normalised = 0) or y = S~ x = c * K~ (c * x) (normalised = 1), the
 * symmetric conjugate of the Markov matrix of Alg. 1.  x, y: device float64,
 * n x nrhs column-major (ld = n), 1 <= nrhs <= 4096 (the scaling study of
 * Sec. 4.2.3 evaluates 512), x and y must not overlap.
 * Tiles are applied in the operator's near/far precision with float32
 * accumulation (float64 when the tiles are float64).  Columns are taken 16 at a
 * time, each tile read once per pass.  Float16 near tiles run on the matrix
 * cores: the vectors are staged per leaf and column as a power-of-two scale
 * times a float16 hi + lo pair (about 22 bits), the sums are float32. */
hdm_status hdm_matvec(hdm_op op, int normalised, const double *x, double *y, int32_t nrhs, void *stream);

/* ---- allocation-free evaluation -----------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the product of
 * hdm_matvec (same arguments, same kernels, bit-identical results) whose
 * workspaces -- the staged vector, skeleton weights and potentials, near-field
 * partial sums, half-precision staging and a copy of the operator's descriptor --
 * live in a 64 MiB device array that the library holds on every device it has
 * a context on until the process ends.  It calls no allocating routine; the
 * descriptor copy is a hipMemcpyAsync from pageable host memory (it returns
 * when the copy is done).
 * Limits and errors: a pass of min(nrhs, 16) columns needs about
 * 8 min(nrhs, 16) (n + 2 skeleton slots + near partial sums) bytes; an operator
 * above the 64 MiB gets HDM_ENOMEM and a message naming both sizes (fewer
 * columns per call may fit).  Every call on one GPU shares its array: calls
 * whose launches overlap on that GPU (other streams, other threads) race and
 * give wrong results; calls ordered on one stream are safe.  Nothing in the
 * array needs clearing between calls (every workspace is written before it is
 * read). */
hdm_status hdm_matvec_noalloc(hdm_op op, int normalised, const double *x, double *y, int32_t nrhs, void *stream);

/* ---- eigensolver (Alg. 1 eigendecomposition; Sec. 2.2 Lanczos) --------------
 * Leading r eigenpairs (largest algebraic) of S~ by Lanczos with full float64
 * reorthogonalisation.  block = 1: single-vector Lanczos, stops when every
 * pair i < r has |beta_j y_{j,i}| <= rel_resid_tol |theta_i|; when the basis
 * reaches max_basis vectors (r + 2 <= max_basis <= 512) before that, it is
 * thick-restarted (Sec. 2.2, the implicit restart with exact shifts): the
 * leading min(max_basis - 2, max(r + 1, (max_basis + r) / 2)) Ritz vectors and
 * the next Lanczos vector become the new basis, up to 100 times.  2 <= block <= 16:
 * block Lanczos with that many vectors per step (one product with block
 * right-hand sides, block QR by shifted Cholesky QR, banded projected matrix
 * solved after Householder tridiagonalisation); pair i is accepted when
 * ||B_j y_i[last block entries]|| <= rel_resid_tol |theta_i|, and max_basis is
 * at most 512 (default min(n, 512), rounded down to a multiple of block).
 * Either stops with HDM_ENOCONV, evals/info filled, when the basis reaches
 * max_basis vectors (block = 1: after the last restart); HDM_ENUMERIC if a
 * residual block loses rank.  info->iters: steps taken (block steps for block > 1).
 * evals: host, r entries, descending.  evecs: device float64 n x r (column-major,
 * phi: unit 2-norm, largest-magnitude entry positive) or NULL. */
hdm_status hdm_eigs(hdm_op op, int32_t r, double rel_resid_tol, int32_t block, int32_t max_basis, uint64_t seed,
                    double *evals, double *evecs, hdm_eig_info_t *info, void *stream);

/* ---- diffusion-map outputs (Alg. 1, last steps) -------------------------------
 * From the leading eigenpairs (lambda_k, phi_k) of S~ (hdm_eigs: evals on the
 * host, phi on the device, n x r column-major, original order):
 *  - psi_k = phi_k / sqrt(d), the right eigenvectors of the Markov matrix
 *    P = D^-1 Q^-1 K~ Q^-1 (the eigenvectors of Alg. 1's eigendecomposition step),
 *    d the alpha = 1 degrees of the operator;
 *  - evals_t[k] = lambda_k^t, the eigenvalues of P^t after t steps of the walk;
 *  - coords_k = lambda_k^t psi_k, the diffusion map at time t;
 *  - dim_t = max{l : |lambda_l|^t > delta |lambda_1|^t} (l from 1; 0 if none), the
 *    lower dimension of Alg. 1 (its printed inequality reads "<"; the intended
 *    reading, the largest l whose weight still exceeds delta times the first, is ">").
 * t >= 0 (an integer number of steps), delta >= 0.  psi, coords: device n x r or
 * NULL; evals_t: host r or NULL; dim_t: host or NULL.  phi may be NULL when psi and
 * coords are.  Synchronises the stream when it writes device outputs. */
hdm_status hdm_diffusion_map(hdm_op op, int32_t r, const double *evals, const double *phi, int32_t t, double delta,
                             double *psi, double *coords, double *evals_t, int32_t *dim_t, void *stream);

/* ---- serving --------------------------------------------------------------- */
typedef struct {
    int32_t max_slots;          /* requests on the GPU at once */
    size_t mem_budget_bytes;    /* admission limit on the sum of resident footprints */
    int32_t compressors;        /* threads building operators concurrently (0: 2) */
} hdm_server_cfg_t;

typedef struct {
    const void *X;          /* host points (params.x_dtype, n x dim); copied by hdm_submit, so the
                               caller may free X on return */
    hdm_params params;
    int32_t r;              /* eigenpairs */
    double rel_resid_tol;
    int32_t max_basis;
    double arrival_s;       /* arrival time on CLOCK_MONOTONIC in seconds (0: the submission time); latency = done - arrival */
} hdm_request_t;

typedef struct {
    int32_t status;         /* hdm_status of the solve */
    int32_t r;
    double evals[64];       /* leading eigenvalues, descending (first r valid) */
    double latency_s;       /* completion - arrival on the caller's clock */
    double service_s;       /* admission -> completion */
    int32_t iters;
    int32_t x_released;     /* 1 once the library has dropped its host copy of X (after the
                               operator is built, or when the request ends) */
} hdm_result_t;

typedef struct {
    int64_t submitted, admitted, completed, rejected, cancelled;
    double solves_per_s, p50_latency_s, p99_latency_s;
    int64_t peak_resident_bytes;
    int64_t shared_launches;  /* launches that served more than one request */
} hdm_server_stats_t;

/* Continuous batching of eigensolves (Alg. 1 + Sec. 2.2 per request): requests
 * are admitted first come, first served while a slot is free and the sum of
 * the admitted requests' device-memory footprints (an upper estimate until the
 * operator exists, then its size) stays within mem_budget_bytes (0 = no cap).
 * A compressor thread builds admitted operators; a solver thread advances every
 * running eigensolve by one Lanczos step per tick, issuing the products of all
 * running solves with equal tile precisions as one launch per phase.  Each
 * result equals the one hdm_compress + hdm_eigs give for the request alone. */
hdm_status hdm_server_create(hdm_ctx ctx, const hdm_server_cfg_t *cfg, hdm_server *out);
/* HDM_EINVAL for bad parameters or NaN/Inf points, HDM_ENOMEM when the
 * request's estimated footprint exceeds the whole budget (counted as rejected). */
hdm_status hdm_submit(hdm_server srv, const hdm_request_t *req, uint64_t *ticket);
/* HDM_EBUSY while the request is queued or running; its result otherwise.  A
 * result is handed out once: the library then forgets the ticket, and later
 * calls with it return HDM_EINVAL (unknown ticket). */
hdm_status hdm_poll(hdm_server srv, uint64_t ticket, hdm_result_t *out);
hdm_status hdm_cancel(hdm_server srv, uint64_t ticket);
hdm_status hdm_server_stats(hdm_server srv, hdm_server_stats_t *out);
/* Waits for running requests, cancels queued ones, frees everything. */
hdm_status hdm_server_destroy(hdm_server srv);

#ifdef __cplusplus
}
#endif
#endif /* HDM_H */
