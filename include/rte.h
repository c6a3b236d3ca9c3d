/*
 * rte.h -- C ABI of the MI355X (gfx950) library for the integral form of
 * radiative transfer with a planar reflective wall, compressed with
 * H-matrices (Pironneau & Tournier, "Reflective Conditions for Radiative
 * Transfer in Integral Form with H-Matrices", arXiv 2306.05789).
 *
 * Conventions shared by every call:
 *  - Every call returns rte_status_t.  No C++ exception or abort crosses the
 *    ABI.  On an error, rte_last_error() returns a thread-local message.
 *  - Handles (rte_mesh_t, rte_plan_t, rte_hmat_t) are opaque and owned by the
 *    library; *_destroy(NULL) is a no-op.  Handles are immutable after
 *    creation, so concurrent calls on different streams may share them.
 *  - Arrays documented "device" are HIP device pointers on the current
 *    device (for example torch tensors' data pointers); "host" arrays are
 *    ordinary host memory.  The caller owns every array it passes.
 *  - Vertex arrays are in natural order v = (i*n1 + j)*n2 + k of the grid
 *    index (i,j,k); the library permutes to its cluster order internally.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Device work is enqueued on it; calls that return host-visible results
 *    synchronise that stream before returning.
 *  - Validation of every argument happens before any device work.
 */
#ifndef RTE_H
#define RTE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RTE_OK = 0,
    RTE_E_INVALID_ARG = 1,   /* an argument failed validation; nothing was enqueued */
    RTE_E_OUT_OF_MEMORY = 2, /* a device allocation failed; no state leaks */
    RTE_E_BUDGET = 3,        /* the request does not fit the configured memory budget */
    RTE_E_DEVICE = 4,        /* a HIP runtime call failed */
    RTE_E_NOT_CONVERGED = 5, /* max_iter reached; outputs hold the last iterate */
    RTE_E_INTERNAL = 6
} rte_status_t;

typedef enum {
    RTE_FP64 = 0,        /* FP64 entries, ACA, storage and matvec */
    RTE_FP32 = 1,        /* FP32 entries, ACA, storage; FP32 accumulation */
    RTE_MIXED_BF16 = 2   /* FP32 entries and ACA; every stored element (low-rank factors
                            and dense leaves) as BF16 hi + lo, hi = bf16(x), lo =
                            bf16(x - hi); solves use BF16-hi sweeps with FP64 defect
                            correction */
} rte_precision_t;

typedef enum { RTE_VOLUME = 0, RTE_SURFACE = 1 } rte_kind_t;

typedef struct rte_mesh *rte_mesh_t;
typedef struct rte_plan *rte_plan_t;
typedef struct rte_hmat *rte_hmat_t;

/* ------------------------------------------------------------------ mesh
 * Section "FEM discretization": a tetrahedral mesh of the domain and a
 * triangular mesh of its boundary.  Here the domain is the box [lo,hi] with
 * n[a] >= 2 vertices per axis (fewer than 2^28 in all, else
 * RTE_E_INVALID_ARG); each cell is split into the six Kuhn
 * tetrahedra that share its (0,0,0)-(1,1,1) diagonal, and each boundary square
 * into the two triangles of its low-to-high diagonal.
 * reflect_axis in {-1,0,1,2}: -1 = no reflective wall; else the box face
 * x[reflect_axis] = (reflect_side ? hi : lo) reflects with coefficient
 * R in [0,1] (Corollary, planar wall, one reflection: Hypothesis 1 with M = 1).
 * reflect_faces: bit f (faces numbered as for emit_faces) marks further
 * reflective faces, face f with coefficient R_faces[f] in [0,1] (the several
 * reflective planes of Section "An Academic Test"); every wall adds the term
 * of its own mirror image and each ray reflects at most once (Hypothesis 1).
 * A face may be given once.
 * emit_faces: bit f (0..5 = x-,x+,y-,y+,z-,z+) marks a black emitting face
 * (boundary source Q = B_nu(T_wall), eq. SE1); a reflective face may not emit.
 * Non-convex domain (Remark rem1; the inner cube of Section "An Academic
 * Test"): when hole_lo[a] < hole_hi[a] on every axis, the cells
 * [hole_lo, hole_hi) (cell indices, 0 <= hole_lo[a] < hole_hi[a] <= n[a]-1)
 * are removed, kappa = +infinity there.  A path that runs a positive length
 * through the removed box, or over a part of a box face that the box covers,
 * is blocked (one grazing the hole's faces or edges is not); the hole's cells
 * belong to no vertex's star; vertices with no remaining cell keep zero rows
 * and columns (the iteration leaves them at J = 0, T = 0).  hole_emit: bit f
 * makes the hole's face on side f%2 of axis f/2 a black emitting face, which
 * must lie inside the box (hole_lo[a] > 0 for side 0, hole_hi[a] < n[a]-1 for
 * side 1).  The surface unknowns are the corners of the emitting face squares
 * (a box-face square under the hole does not emit), in ascending vertex id.
 * All-zero hole fields: the whole box. */
typedef struct {
    int32_t n[3];
    double lo[3], hi[3];
    int32_t reflect_axis;
    int32_t reflect_side;
    double R;
    uint32_t emit_faces;
    uint32_t reflect_faces;
    double R_faces[6];
    int32_t hole_lo[3];
    int32_t hole_hi[3];
    uint32_t hole_emit;
    uint32_t emission;   /* 0: isotropic black wall, Q = B_nu(T_wall) and the kernel [(x-y).n]_+ / |x-y|^3
                            of eq. SE1 (the default); 1: the cosine-weighted source of Section "Example",
                            Q = [omega.n]_- Q0, kernel ([(x-y).n]_+)^2 / |x-y|^4 (in the face's plane on the
                            diagonal theta_F / (8 pi)); the same for every emitting face */
} rte_mesh_desc_t;

rte_status_t rte_mesh_create(const rte_mesh_desc_t *desc, rte_mesh_t *out);
/* Number of volume vertices N and of emitting boundary vertices L. */
rte_status_t rte_mesh_sizes(rte_mesh_t mesh, int64_t *N, int64_t *L);
/* Natural ids of the emitting vertices in ascending order (host array of L). */
rte_status_t rte_mesh_emitting_ids(rte_mesh_t mesh, int64_t *ids);
void rte_mesh_destroy(rte_mesh_t mesh);

/* ------------------------------------------------------------------ H-matrix options
 * Section "Compression": cluster tree by geometric bisection (leaf_size),
 * admissibility max(R1,R2) < eta * dist(box1, box2), partially pivoted ACA
 * with relative Frobenius tolerance aca_eps.  dense = 1 stores every block
 * dense (no compression).  recompress = 1: the factors of every block the ACA
 * compressed (ranks up to 96) are replaced by the shortest truncation of the
 * SVD of their product whose relative Frobenius error is <= aca_eps (a block
 * whose factors are numerically dependent, or that would not get shorter,
 * keeps them); the error against the ACA product adds at most aca_eps. */
typedef struct {
    int32_t kind;        /* rte_kind_t: RTE_VOLUME (N x N matrix G) or RTE_SURFACE (N x L matrix S) */
    int32_t dense;
    int32_t leaf_size;   /* >= 1 */
    double eta;          /* > 0 */
    double aca_eps;      /* in (0,1) */
    int32_t precision;   /* rte_precision_t */
    int32_t recompress;  /* 0 or 1 */
    int32_t aca_hits;    /* 0 or 1 (the default): the ACA of a block stops at the first rank step with
                            |u_k| |v_k| <= aca_eps |S_k|_F; 2: only after two consecutive such steps
                            (a somewhat higher rank; the worst blocks' true error about halves) */
} rte_hmat_opts_t;

/* ------------------------------------------------------------------ plan (host only)
 * The cluster trees and the block tree, built on the host without touching
 * the device.  Export: tgt_perm[N_tgt] and src_perm[N_src] map cluster order
 * to natural ids (surface sources: to emitting-vertex natural ids); blocks
 * [nblocks][5] = (t0, t1, s0, s1, admissible) as half-open ranges in cluster
 * order, dense leaves first, then admissible blocks, each in tree order. */
typedef struct {
    int64_t n_tgt, n_src;
    int64_t n_dense, n_lowrank;
    int64_t dense_entries;       /* sum of m*n over dense leaves */
    int64_t lowrank_sum_mn;      /* sum of m+n over admissible blocks */
    int64_t n_tgt_leaves;
} rte_plan_info_t;

rte_status_t rte_plan_create(rte_mesh_t mesh, const rte_hmat_opts_t *opts, rte_plan_t *out);
rte_status_t rte_plan_info(rte_plan_t plan, rte_plan_info_t *info);
rte_status_t rte_plan_export(rte_plan_t plan, int64_t *tgt_perm, int64_t *src_perm, int64_t *blocks);
void rte_plan_destroy(rte_plan_t plan);

/* ------------------------------------------------------------------ entries
 * Direct evaluation of n matrix entries (rows[k], cols[k]) for one kappa field
 * (tests and diagnostics).  Volume: G^{ij} = exp(-tau) g^{ij} + R exp(-tau_bar) g_bar^{ij}
 * (Section "FEM discretization"), cols are vertex ids.  Surface: S^{il} of the
 * boundary source matrix, cols are natural ids of emitting vertices.
 * kappa: device, [N] FP64 vertex values.  rows, cols: device int64 [n].
 * out: device [n], FP64 (precision RTE_FP64) or FP32 values widened to FP64. */
rte_status_t rte_entries(rte_mesh_t mesh, int32_t kind, const double *kappa, int64_t n,
                         const int64_t *rows, const int64_t *cols, double *out,
                         int32_t precision, void *stream);

/* ------------------------------------------------------------------ assembly
 * Builds one H-matrix per band from kappa (device, [n_bands][N] FP64): dense
 * leaves are filled directly, admissible blocks by partially pivoted ACA on
 * the GPU (Section "Compression").  Synchronises `stream`. */
rte_status_t rte_hmat_assemble(rte_mesh_t mesh, int32_t n_bands, const double *kappa,
                               const rte_hmat_opts_t *opts, void *stream, rte_hmat_t *out);

/* y = H_band x for nrhs right-hand sides (Section "Compression": once the
 * matrix is compressed, the fixed-point iterations only need such products;
 * dense leaves contribute A x, admissible blocks U (V^T x)).  x: device [nrhs][N_src] FP64 (surface:
 * N_src = L, emitting vertices in ascending id order); y: device [nrhs][N_tgt].
 * Natural order on both sides.  Stored precision as assembled; FP64 accumulate
 * for FP64 storage, FP32 accumulate otherwise, results returned in FP64. */
rte_status_t rte_hmat_matvec(rte_hmat_t h, int32_t band, int32_t nrhs, const double *x,
                             double *y, void *stream);

/* The same product for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * y = H_band x with every intermediate (x and y in cluster order, the
 * matvec's partial sums and staged operands) in a fixed workspace of 64 MiB
 * that the library holds on each device for the life of the process; no
 * hipMalloc, hipFree or allocating library call is made.  Calls on one device
 * share that workspace: calls that overlap in time on one device (different
 * streams or host threads) race and must be serialised by the caller.  Returns
 * RTE_E_BUDGET, with nothing enqueued, when the product needs more workspace
 * than that (about N_src + N_tgt doubles per right-hand side plus the partial
 * sums).  Synchronises `stream`. */
rte_status_t rte_hmat_matvec_noalloc(rte_hmat_t h, int32_t band, int32_t nrhs, const double *x,
                                     double *y, void *stream);

/* Operator of a matvec on RTE_MIXED_BF16 storage (the other storages have one):
 * RTE_OP_ACCURATE multiplies by the hi + lo factors, with the vector carried
 * as three BF16 parts (24 significant bits), and adds the FP32 matrix-core
 * steps in FP64 (the operator of the defect steps); RTE_OP_LOW multiplies the
 * BF16 hi factors by the vector (and the intermediate V^T x) carried as two
 * BF16 parts (16 significant bits) with FP32 accumulation: the operator of
 * the inner sweeps, which apply it to the change of the source since the last
 * defect step. */
typedef enum { RTE_OP_ACCURATE = 0, RTE_OP_LOW = 1 } rte_operator_t;

/* y_b = H_b x_b for every band b and nrhs right-hand sides, each phase one
 * launch over all bands and right-hand sides (Section "Compression").
 * x: device [n_bands][nrhs][N_src] FP64, y: device [n_bands][nrhs][N_tgt],
 * natural order on both sides.  op: an rte_operator_t.  Synchronises `stream`. */
rte_status_t rte_hmat_matvec_batched(rte_hmat_t h, int32_t nrhs, const double *x, double *y, int32_t op,
                                     void *stream);

/* Launch shape of the matvec of one H-matrix: wavefronts per phase-B
 * workgroup (one workgroup per target leaf and band; matrix cores: 2, 4 or 8,
 * vector ALU: 4 or 8), bytes of V per phase-A task (KiB), and 16-rank tiles
 * per phase-A task on the matrix cores (1, 2, 4 or 8; the rank bucket a task
 * covers; with 8 the accurate operator still takes tasks of at most 4).
 * Changing it rebuilds the work lists and regroups partial sums:
 * results agree to rounding (FP32 accumulation: ~1e-7, FP64: ~1e-15). */
typedef struct {
    int32_t phase_b_waves;
    int32_t phase_a_kib;
    int32_t phase_a_tiles;
} rte_matvec_config_t;

rte_status_t rte_hmat_get_config(rte_hmat_t h, rte_matvec_config_t *cfg);
rte_status_t rte_hmat_set_config(rte_hmat_t h, const rte_matvec_config_t *cfg, void *stream);
/* Autotuner: times every candidate shape (reps all-band matvecs of nrhs
 * right-hand sides, operator op, HIP events) on this matrix and keeps the
 * fastest; best_ms: its time per matvec; trials: candidates timed.
 * Synchronises `stream`. */
rte_status_t rte_hmat_autotune(rte_hmat_t h, int32_t nrhs, int32_t op, int32_t reps, void *stream,
                               rte_matvec_config_t *best, double *best_ms, int32_t *trials);
/* HIP-event time of one all-band matvec (nrhs right-hand sides, operator op), mean of reps. */
rte_status_t rte_hmat_time_matvec(rte_hmat_t h, int32_t nrhs, int32_t op, int32_t reps, void *stream, double *ms);

typedef struct {
    int64_t n_tgt, n_src;
    int32_t n_bands, precision;
    int64_t n_dense, n_lowrank, n_fallback_dense; /* fallback: ACA did not converge below the cap */
    int64_t dense_entries;                        /* stored dense entries, per band, summed */
    int64_t lowrank_entries;                      /* sum over LR blocks of (m+n)*rank, summed over bands */
    int32_t max_rank;
    double mean_rank;                             /* (m+n)-weighted */
    double compression;                           /* 1 - stored entries / (N_tgt*N_src*bands) */
    int64_t bytes;                                /* device bytes of the stored operator */
    int64_t entries_evaluated;                    /* kernel entries computed during assembly */
    double assemble_ms;                           /* host wall time of the assembly call */
    double aca_kernel_ms;                         /* HIP-event time of the whole ACA (all rank steps),
                                                     summed over bands (bands of a multi-band matrix are
                                                     assembled two at a time, so the sum can exceed
                                                     assemble_ms) */
    int32_t aca_launches;                         /* ACA batches */
    double aca_entry_ms;                          /* HIP-event time of the ACA row/column entry launches,
                                                     summed over bands */
    int32_t aca_entry_launches;
    double fill_kernel_ms;                        /* HIP-event time of the dense-fill launches, summed */
    int32_t fill_launches;
    int64_t aca_entries;                          /* entries evaluated inside the ACA launches */
    int64_t aca_retried;                          /* blocks run again with the larger second-pass cap */
    double alloc_ms;                              /* host time spent allocating and freeing device memory
                                                     during the assembly, summed over its threads */
    int64_t free_bytes;                           /* device memory free when the assembly started (including
                                                     the library's idle scratch pool) */
    int64_t lowrank_entries_aca;                  /* lowrank_entries before the recompression (equal without it) */
    int64_t recompressed_blocks;                  /* blocks the recompression examined, summed over bands */
    double recompress_ms;                         /* HIP-event time of the recompression, summed over bands */
} rte_hmat_stats_t;

rte_status_t rte_hmat_stats(rte_hmat_t h, rte_hmat_stats_t *stats);

/* ------------------------------------------------------------------ kappa levels
 * Section "Compression": a few values of kappa_nu, each with its two matrices,
 * stand for all frequencies as a piecewise-constant interpolation (Section
 * "Test 2: the General Case": 8 values for 583 frequencies).  Adaptive
 * levels for n positive multipliers values[b] (host): the fewest levels such
 * that every value lies within a factor (1 + tol) of its level, chosen on the
 * sorted logarithms by the greedy cover (optimal for intervals of one length
 * on a line): each level is (1 + tol) times the smallest value it takes.
 * levels[] (host, ascending, room for max_levels) and map[b] (host, the
 * level of value b) are written; *n_levels the count.  tol > 0; more than
 * max_levels needed: RTE_E_INVALID_ARG (raise tol). */
rte_status_t rte_kappa_levels(const double *values, int32_t n, double tol, int32_t max_levels, double *levels,
                              int32_t *map, int32_t *n_levels);

/* A band-mapped view of an H-matrix: band b of the view is band band_op[b]
 * of h (host array of n_bands entries, each in [0, h's band count)), with the
 * absorption of that band.  The view shares h's stored operator (h must
 * outlive it; destroy it with rte_hmat_destroy) and builds its own matvec
 * work lists, so a solve on views of G and S runs each of its bands with its
 * own frequency, weight and right-hand sides on the operator of its level
 * (the levels of rte_kappa_levels); rte_hmat_stats of a view reports h's
 * figures with the view's band count.  Synchronises `stream`. */
rte_status_t rte_hmat_select_bands(rte_hmat_t h, int32_t n_bands, const int32_t *band_op, void *stream,
                                   rte_hmat_t *out);

/* Factors of admissible block `block` (0-based among admissible blocks, plan
 * order) of band `band`, copied to host FP64: U [m][rank] and V [n][rank],
 * rows in cluster order of the block's ranges; the block approximates rows
 * tgt_perm[t0..t1) x cols src_perm[s0..s1) as U V^T.  rank, m and n are always
 * written (rank -1: the block is stored dense); pass NULL U/V to query them,
 * then buffers of m*rank and n*rank doubles.  Synchronous. */
rte_status_t rte_hmat_block_factors(rte_hmat_t h, int32_t band, int64_t block, int32_t *rank, int64_t *m,
                                    int64_t *n, double *U, double *V);
/* Same for one operator of RTE_MIXED_BF16 storage (op: rte_operator_t):
 * RTE_OP_ACCURATE reads hi + lo, RTE_OP_LOW the BF16 hi parts alone, the
 * values the low operator multiplies by.  Other storages ignore op. */
rte_status_t rte_hmat_block_factors_op(rte_hmat_t h, int32_t band, int64_t block, int32_t op, int32_t *rank,
                                       int64_t *m, int64_t *n, double *U, double *V);
/* Dense blocks of band `band` (Section "Compression": blocks that reach the
 * leaves without becoming admissible are stored whole; here also the
 * admissible blocks whose ACA rank reached the storage break-even and were
 * stored whole instead), read back to host FP64 so that the stored operator
 * can be applied by an independent product.  *count receives the number of
 * dense blocks of the band (the plan's dense leaves, then the admissible
 * blocks stored dense).  When range or A is non-NULL, block `index` (0 <=
 * index < *count) is read: range[4] = (t0, t1, s0, s1), half-open row and
 * column ranges in the cluster orders of rte_plan_export; A: host
 * [t1 - t0][s1 - s0] row-major, the stored values (FP64, FP32 widened, BF16
 * hi + lo, or hi alone for op = RTE_OP_LOW).  Synchronous. */
rte_status_t rte_hmat_dense_block(rte_hmat_t h, int32_t band, int64_t index, int32_t op, int64_t *count,
                                  int64_t *range, double *A);
void rte_hmat_destroy(rte_hmat_t h);

/* ------------------------------------------------------------------ fixed point
 * Algorithm of Section "Fixed Point Iterations" (eq. algo), with J^0 = 0:
 *   S_b   = (1 - a_b) B_{nu_b}(T) + a_b J_b
 *   J_b  <- S^E_b + G_b S_b,  S^E_b = S_b_hat Q_b,  Q_b = B_{nu_b}(T_wall)
 *   T     : per vertex root of sum_b w_b kappa_b (1 - a_b)(J_b - B_{nu_b}(T)) = 0 (FP64 Newton)
 * grey = 1: one band, B(T) = sigma T^4 with sigma = pi^4/15 (eq. grey), T = (J/sigma)^{1/4}.
 * Stops when max_b ||J_b^{k+1} - J_b^k||_2 / ||J_b^{k+1}||_2 <= tol, per right-hand side.
 * nu, w, a: host arrays of n_bands (w: NULL = trapezoid weights on sorted nu;
 * a: NULL = no scattering).  T_wall: device [nrhs][L]; T0: device [nrhs][N] or NULL (= 0).
 * T_out: device [nrhs][N]; J_out: device [nrhs][n_bands][N] or NULL. */
typedef struct {
    int32_t n_bands;
    const double *nu;
    const double *w;
    const double *a;
    int32_t grey;
    int32_t nrhs;
    const double *T_wall;
    const double *T0;
    double tol;
    int32_t max_iter;
    int32_t precision;     /* RTE_MIXED_BF16: inner sweeps on BF16-hi factors, FP64 defect steps */
    int32_t launch;        /* RTE_LAUNCH_STREAM: kernels enqueued one by one; RTE_LAUNCH_GRAPH: each
                              distinct sweep captured once in a hipGraph and replayed (same kernels,
                              same results; fewer launch round trips for small meshes) */
    int32_t time_matvecs;  /* 1: HIP events around every volume matvec (stats ms_matvec_low/acc); with
                              RTE_LAUNCH_GRAPH a sweep is then captured as three graphs, before the
                              matvec, the matvec and after it, with the events between them.  0: stream
                              launch still times the matvecs; graph launch times whole sweeps only */
    double *residuals;     /* host [max_iter] or NULL: receives the residual of each sweep in order (the
                              first stats.iterations entries are written; a mixed solve's defect steps
                              and inner sweeps interleave as they ran) */
} rte_solve_desc_t;

enum { RTE_LAUNCH_STREAM = 0, RTE_LAUNCH_GRAPH = 1 };

typedef struct {
    int32_t iterations;         /* matvec sweeps over all bands (from T0 = 0 the first sweep has a zero
                                   source, G S = 0 exactly: it applies no operator and is counted here
                                   but in neither matvecs_low nor matvecs_acc) */
    int32_t outer_steps;        /* FP64 defect-correction steps (mixed precision) */
    double residual;            /* final relative change of J */
    int64_t monotone_violations;/* vertex-steps where T decreased by more than 8 units of rounding
                                   (2^-52 relative): from T0 = 0 it should be 0 */
    double ms_total, ms_matvec; /* ms_matvec: HIP-event time of the volume matvecs (graph launch without
                                   time_matvecs: of the whole sweeps) */
    int32_t graphs;             /* sweep graphs captured (RTE_LAUNCH_GRAPH) */
    double ms_matvec_low;       /* HIP-event time of the volume matvecs on the low operator (mixed
                                   inner sweeps); -1 when not timed (graph launch without time_matvecs) */
    int32_t matvecs_low;        /* their number */
    double ms_matvec_acc;       /* same for the matvecs on the accurate (or only) operator */
    int32_t matvecs_acc;
} rte_solve_stats_t;

rte_status_t rte_fixed_point_solve(rte_mesh_t mesh, rte_hmat_t vol, rte_hmat_t surf,
                                   const rte_solve_desc_t *desc, double *T_out, double *J_out,
                                   rte_solve_stats_t *stats, void *stream);

/* ------------------------------------------------------------------ request server
 * Fixed-point solves of many requests on resident meshes, continuously
 * batched: a request names a mesh, a subset of the band catalogue, a kappa
 * multiplier per band (of the mesh's base field) and wall temperatures.  A
 * multiplier m is snapped to the level l = round(levels_per_decade log10 m)
 * of the ladder 10^(l / levels_per_decade) (ties to the lower level); the
 * snapped value defines the request.  The operators of a (mesh, level) are
 * assembled on first use, shared by every band of every request at that
 * level and evicted least recently used, when unused, to stay within the HBM
 * budget.  A waiting request whose operators are resident is admitted, in
 * arrival order among such requests, once its state fits; missing operators
 * are assembled by a thread of the server on a stream of its own, for the
 * oldest few waiting requests, and only the oldest may evict.  Each
 * rte_server_step runs one sweep of every admitted request (columns that
 * share an operator in one matvec) and retires the ones that converged.  Band
 * weights are the trapezoid weights of the whole catalogue (the band sum of
 * Section "Test 2: the General Case").  The fixed point of every request is the
 * one of Section "Fixed Point Iterations", defect-corrected with mixed
 * precision storage as in rte_fixed_point_solve.
 * Not thread safe: one thread drives a server. */
typedef struct rte_server *rte_server_t;

typedef struct {
    int64_t hbm_budget;          /* bytes of operators and request state; 0 = 80% of the free device memory */
    int32_t n_catalogue;         /* band catalogue size */
    const double *nu;            /* host [n_catalogue], increasing */
    int32_t levels_per_decade;   /* kappa ladder resolution */
    int32_t leaf_size;
    double eta, aca_eps;
    int32_t precision;           /* RTE_FP64 (plain sweeps) or RTE_MIXED_BF16 (defect-corrected) */
    int32_t max_active;          /* requests iterated together (1: one at a time) */
    int32_t recompress;          /* 1: volume operators take the SVD recompression of their ACA factors
                                    (rte_hmat_opts_t.recompress): smaller, longer to assemble */
} rte_server_desc_t;

typedef struct {
    int32_t mesh_id;
    int32_t n_bands;
    const int32_t *bands;        /* host [n_bands], increasing catalogue indices */
    const double *kappa_mult;    /* host [n_bands], > 0 */
    const double *a;             /* host [n_bands] scattering coefficients in [0, 1) (eq. eqS:
                                    S = (1 - a) B(T) + a J), or NULL for none */
    const double *T_wall;        /* device [L] (emitting vertices in ascending id order), copied at submit */
    double tol;                  /* relative change of J that ends the request (FP64 residual) */
    int32_t max_iter;
} rte_request_t;

enum { RTE_REQ_PENDING = 0, RTE_REQ_ACTIVE = 1, RTE_REQ_DONE = 2 };

typedef struct {
    int32_t state;               /* RTE_REQ_* */
    int32_t converged;
    int32_t iterations, outer_steps;
    double residual;
    int32_t n_bands;
} rte_request_info_t;

typedef struct {
    int64_t budget, resident_bytes, operators;
    int64_t assembled, evicted, over_budget;   /* over_budget: admitted alone beyond the budget */
    int64_t submitted, completed, steps, columns;
    double assemble_ms, sweep_ms;
} rte_server_stats_t;

rte_status_t rte_server_create(const rte_server_desc_t *desc, void *stream, rte_server_t *out);
/* kappa: device [N], natural order (the base field); copied */
rte_status_t rte_server_add_mesh(rte_server_t s, const rte_mesh_desc_t *mesh, const double *kappa, int32_t *mesh_id);
rte_status_t rte_server_submit(rte_server_t s, const rte_request_t *req, int64_t *id);
/* admission, then one sweep of every admitted request; synchronises the server's stream */
rte_status_t rte_server_step(rte_server_t s, int32_t *n_active, int32_t *n_pending);
rte_status_t rte_server_poll(rte_server_t s, int64_t id, rte_request_info_t *info);
/* the snapped ladder level of every band of a request: host [n_bands] */
rte_status_t rte_server_levels(rte_server_t s, int64_t id, int32_t *levels);
/* T of a finished request (device [N], natural order); the request is then forgotten */
rte_status_t rte_server_fetch(rte_server_t s, int64_t id, double *T_out);
rte_status_t rte_server_stats(rte_server_t s, rte_server_stats_t *stats);
void rte_server_destroy(rte_server_t s);

/* ------------------------------------------------------------------ misc */
const char *rte_status_string(rte_status_t s);
const char *rte_last_error(void);
const char *rte_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RTE_H */
