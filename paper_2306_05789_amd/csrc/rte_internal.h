// Internal declarations of the rte library (host C++ and HIP device code).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <mutex>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "rte.h"

namespace rte {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
    rte_status_t code;
    Error(rte_status_t c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define RTE_REQUIRE(cond, msg)                                                          \
    do {                                                                                \
        if (!(cond)) throw ::rte::Error(RTE_E_INVALID_ARG, std::string(msg));           \
    } while (0)

#define HIP_CHECK(expr)                                                                 \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            throw ::rte::Error(e_ == hipErrorOutOfMemory ? RTE_E_OUT_OF_MEMORY : RTE_E_DEVICE, \
                               std::string(#expr) + ": " + hipGetErrorString(e_));     \
    } while (0)

#define HIP_LAUNCH_CHECK() HIP_CHECK(hipGetLastError())

// ---------------------------------------------------------------- quadrature rules
// Symmetric simplex rules obtained by solving their moment equations
// (quadrule.cpp).  Points are barycentric ([nq][nvert]), weights sum to 1.
struct Rule {
    int nvert = 0, nq = 0, degree = 0;
    std::vector<double> p, w;
};
const Rule &tet_rule(int degree);   // 2 (4 points) or 5 (14 points)
const Rule &tri_rule(int degree);   // 2 (3 points) or 5 (7 points)

// ---------------------------------------------------------------- device geometry
constexpr int kNearCheb = 2;        // near rule iff grid Chebyshev distance <= 2
constexpr int kTets = 24;           // Kuhn tetrahedra around an interior vertex
constexpr int kTris = 6;            // boundary triangles around a face vertex

struct GridDev {
    int n[3];
    int stride[3];          // natural-order strides: n1*n2, n2, 1
    double lo[3], h[3];
    int n_walls;            // planar reflective walls (whole box faces, one reflection each)
    int wall_axis[6];
    int wall_side[6];       // 0: the plane at lo, 1: at hi
    double R[6];
    unsigned emit_faces;
    int has_hole;           // non-convex domain: the cells [hole_lo, hole_hi) are removed
    int hole_lo[3], hole_hi[3];
    unsigned hole_open;     // bit 2a (2a+1): the hole reaches the box face at the low (high) end of axis a
    unsigned hole_emit;     // bit f: the hole's face on side f%2 of axis f/2 emits
    unsigned emission;      // 0: isotropic wall source (eq. SE1); 1: cosine-weighted (Section "Example")
    double vol_scale;       // |tet| / (4 pi)
    double area_scale[3];   // |triangle| / (4 pi) for faces normal to axis a
};

// Surface stencil tables on the device, one set per precision (T = double or
// float), per rule: [kTris][nq][4] = offset along the face's two axes (grid
// units), coef = w_q * lambda_l(y_q), pad.  (The volume rules reach the device
// through the per-mesh tables of NearTables.)
template <typename T>
struct StencilDev {
    const T *tri_far, *tri_near;
    int nq_tri_far, nq_tri_near;
    const int *tet_meta;    // [kTets][5]: 4 neighbour slots (0..26 of the 3x3x3 block), cell corner bits
    const int *tri_meta;    // [kTris][2]: square offset bits along the face axes (b, c)
};

// ---------------------------------------------------------------- mesh
// Volume quadrature tables of a mesh (they depend on the spacing only).
// Near field (the degree-5 rule, grid Chebyshev distance <= 2 between target
// and source): for each offset d in [-2, 2]^3, each of the 8 cells around the
// source vertex and each of the cell's 8 corners, the weight of the corner's
// kappa in g(x_j + d, j).  Far field (the degree-2 rule): per tetrahedron of
// the star and quadrature point, A_a = -2 h_a^2 e_a and C = sum h_a^2 e_a^2
// (e the point's offset from the source vertex, grid units), so that
// |x - y|^2 = |h d|^2 + A.d + C, then w_q lambda_j b_k for the 4 vertices.
// Host copy at mesh creation, device copies on first use.
constexpr int kNearOffsets = 125;
constexpr int kNearSize = kNearOffsets * 64;
constexpr int kFarSize = kTets * 4 * 8;
struct NearTables {
    std::vector<double> host;    // near [kNearOffsets][8 cells][8 corners], then far [kTets][4][8]
    std::mutex mu;
    std::map<int, std::pair<void *, void *>> dev;   // device -> (FP64, FP32) copies
    ~NearTables();
};

struct PlanCache;   // block-tree plans of a mesh (htree.cpp)

// An emitting rectangle of the boundary: the plane x_a = plane (grid index),
// the normal into the domain sign * e_a, square index ranges [lo, hi) along
// the two other axes b < c.
struct EmitRect {
    int a, plane, sign, lo[2], hi[2];
};
std::vector<EmitRect> emit_rects(const rte_mesh_desc_t &d);   // box faces, then the hole's

struct Mesh {
    rte_mesh_desc_t desc{};
    int64_t N = 0, L = 0;
    double h[3] = {0, 0, 0};
    std::vector<int64_t> emitting;   // natural ids, ascending
    GridDev dev{};
    std::shared_ptr<NearTables> near;
    std::shared_ptr<PlanCache> plans;
    const void *near_table(bool fp64) const;   // device copy on the current device
    std::vector<double> positions() const;            // [N][3]
    std::vector<double> emitting_positions() const;   // [L][3]
};

// Host copies of the stencil tables (built once per process from the rules).
struct StencilHost {
    std::vector<double> vol_far, vol_near, tri_far, tri_near;
    int nq_vol_far = 0, nq_vol_near = 0, nq_tri_far = 0, nq_tri_near = 0;
    std::vector<int> tet_meta, tri_meta;
};
const StencilHost &stencil_host();

// Per-device uploaded copies.
struct StencilBuffers {
    StencilDev<double> d;
    StencilDev<float> f;
};
const StencilBuffers &stencil_device();   // uploads on first use on the current device

// ---------------------------------------------------------------- trees (htree.cpp)
struct ClusterNode {
    int64_t start, stop;
    double bmin[3], bmax[3];
    int child[2] = {-1, -1};
};

struct ClusterTree {
    std::vector<int64_t> perm;        // cluster position -> caller's point index
    std::vector<ClusterNode> nodes;   // nodes[0] is the root
    std::vector<int> leaves;          // node ids of the leaves in order
};

ClusterTree build_cluster_tree(const std::vector<double> &pts, int leaf_size);

struct Block {
    int64_t t0, t1, s0, s1;
};

struct Plan {
    rte_hmat_opts_t opts{};
    ClusterTree tgt, src;
    std::vector<int64_t> tgt_nat, src_nat;   // cluster position -> natural vertex id
    std::vector<Block> dense, lowrank;
    std::vector<std::pair<int64_t, int64_t>> tgt_leaves;   // [start, stop) of target leaves
    std::vector<int64_t> leaf_start;   // [n_leaves + 1] first row of each target leaf, then N_tgt
    std::vector<int32_t> row_leaf;     // [N_tgt] target leaf of each row (cluster order)
    int leaf_of(int64_t row) const { return row_leaf[(size_t)row]; }
};

void validate_opts(const Mesh &m, const rte_hmat_opts_t &opts);
std::unique_ptr<Plan> build_plan(const Mesh &m, const rte_hmat_opts_t &opts);
// The plan of a mesh for (kind, leaf size, eta, dense), built on first use and
// shared afterwards: the trees and the block partition depend on the geometry
// and these options only, not on kappa, precision or the ACA tolerance (the
// returned plan's own `opts` are those of its first use).  Thread-safe.
std::shared_ptr<const Plan> mesh_plan(const Mesh &m, const rte_hmat_opts_t &opts);
std::shared_ptr<PlanCache> new_plan_cache();

// ---------------------------------------------------------------- device memory helper
// An owned device allocation.  DevBuf(b) / alloc(b) take it from hipMalloc
// (on out-of-memory the idle scratch pool is released and the call retried);
// DevBuf::scratch(b) takes it from the per-device scratch pool (pool.cpp).
// A scratch buffer goes back to the pool on release only when `settled` was
// set, which says that no queued work reads it any more (its stream has
// drained); otherwise it is freed with hipFree, which waits for the device.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    size_t cap = 0;          // scratch: capacity of the pooled allocation
    bool pooled = false;
    bool settled = false;
    DevBuf() = default;
    explicit DevBuf(size_t b) { alloc(b); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept { take(o); }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            release();
            take(o);
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t b);
    void release() noexcept;
    static DevBuf scratch(size_t b);
    template <typename T> T *as() const { return static_cast<T *>(p); }

private:
    void take(DevBuf &o) noexcept {
        p = o.p;
        bytes = o.bytes;
        cap = o.cap;
        pooled = o.pooled;
        settled = o.settled;
        o.p = nullptr;
        o.bytes = o.cap = 0;
        o.pooled = o.settled = false;
    }
};

// Scratch pool of the current device (pool.cpp).
void *pool_take(size_t bytes, size_t *cap);
void pool_give(void *p, size_t cap);
size_t pool_idle_bytes();   // idle pooled bytes on the current device
void pool_trim();           // free the idle pooled buffers of the current device
double &alloc_ms_this_thread();   // host ms this thread spent allocating and freeing device memory

// Checking aid: with RTE_POISON_WORKSPACE set in the environment, scratch
// buffers are filled with 0xFF bytes (NaN in every floating format) when they
// are allocated, so a read of something never written shows up as NaN instead
// of hiding behind freshly zeroed memory.  Called outside graph capture.
inline void poison(DevBuf &b, hipStream_t s) {
    static const bool on = std::getenv("RTE_POISON_WORKSPACE") != nullptr;
    if (on && b.bytes) HIP_CHECK(hipMemsetAsync(b.p, 0xFF, b.bytes, s));
}

template <typename T>
DevBuf upload(const std::vector<T> &v, hipStream_t s) {
    DevBuf b(v.size() * sizeof(T));
    if (!v.empty()) {
        HIP_CHECK(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    }
    return b;
}

// Same into pooled scratch (for task lists retired with the band's scratch).
template <typename T>
DevBuf upload_scratch(const std::vector<T> &v, hipStream_t s) {
    DevBuf b = DevBuf::scratch(v.size() * sizeof(T));
    if (!v.empty()) {
        HIP_CHECK(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    }
    return b;
}

// ---------------------------------------------------------------- H-matrix storage
// Storage of a block whose target range covers target leaves li0..li1-1:
//  - the row side (a dense block's columns, or U of a low-rank block with K =
//    rank columns) is split into one slice per target leaf, and the slices
//    follow each other;
//  - FP64 and FP32 storage: slice s is column-major [K][rp_s], rp_s = leaf
//    rows rounded up to 4, and starts K * (prp[li0 + s] - prp[li0]) elements
//    in; V of a low-rank block is row-major [n][pad4(rank)];
//  - BF16 storage is K-grouped for the matrix cores: slice s is [K8/8][r_s][8]
//    (8 consecutive columns of one row are contiguous; K8 = K rounded up to 8,
//    rows not padded), and V is [n8/8][rank][8] (8 consecutive sources of one
//    rank index contiguous).  Sources are counted in stored coordinates in
//    which every source leaf is rounded up to 8 (src_p maps a source to its
//    stored coordinate), so a dense block has pwidth(s0, s1) >= n columns and
//    V has pwidth rows; the vectors a matvec multiplies are staged in the same
//    coordinates.
// Padding is zero.  Mixed precision stores every element x as BF16 hi =
// bf16(x) and lo = bf16(x - hi) in two arrays of the same layout (BF16
// keeps FP32's exponent range, so no scale is needed).
// The two events around one queued launch (read after the stream has drained).
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    EventPair() {
        HIP_CHECK(hipEventCreate(&a));
        HIP_CHECK(hipEventCreate(&b));
    }
    EventPair(const EventPair &) = delete;
    EventPair &operator=(const EventPair &) = delete;
    EventPair(EventPair &&o) noexcept : a(o.a), b(o.b) { o.a = o.b = nullptr; }
    EventPair &operator=(EventPair &&o) noexcept {
        std::swap(a, o.a);
        std::swap(b, o.b);
        return *this;
    }
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

struct BandStore {
    std::vector<DevBuf> bufs;               // owning storage chunks
    // Work still queued when the band's host work goes on: buffers its kernels
    // read (task lists, ACA scratch) and the events of its fill launches.
    // band_settle() waits for the stream, adds the fill times and frees them.
    std::vector<DevBuf> retire;
    std::vector<EventPair> fill_events;
    std::vector<Block> dense_blocks;        // plan dense leaves, then ACA fallbacks
    std::vector<const void *> dense_ptr;    // per dense block
    std::vector<const void *> dense_lo;     // per dense block: BF16 lo part (mixed precision)
    std::vector<int32_t> rank;              // per plan LR block; -1 = stored dense (fallback)
    std::vector<const void *> U, V;         // per plan LR block (nullptr for fallbacks)
    std::vector<const void *> Ulo, Vlo;     // mixed precision: BF16 lo parts
    int64_t bytes = 0, dense_entries = 0, lr_entries = 0, evaluated = 0, aca_entries = 0, aca_retried = 0;
    int64_t rc_before = 0, rc_after = 0, rc_blocks = 0;      // recompression: (m+n) k before and after
    double aca_ms = 0.0, fill_ms = 0.0, aca_entry_ms = 0.0;   // HIP-event kernel times
    double rc_ms = 0.0;
    int aca_launches = 0, fill_launches = 0, aca_entry_launches = 0;
};

struct MatvecPlan;   // device work lists (hmatvec.hip)

// Launch shape of the matvec (chosen by the autotuner, or set).
struct MatvecConfig {
    int waves_b = 4;      // phase B wavefronts per workgroup (matrix cores: 2, 4, 8; vector ALU: 4, 8)
    int task_kib = 64;    // phase A: bytes of V per task, KiB
    int tiles = 4;        // matrix cores: 16-rank tiles per phase A task (1, 2, 4)
};

struct HMat {
    const Mesh *mesh = nullptr;     // not owned: the mesh must outlive the matrix
    std::shared_ptr<const Plan> plan;
    rte_hmat_opts_t opts{};   // the options of this assembly
    int n_bands = 0;
    int precision = RTE_FP64;
    int kind = RTE_VOLUME;
    std::vector<BandStore> bands;
    DevBuf tgt_nat, src_nat;        // int64: cluster position -> natural id (surface sources: vertex ids)
    DevBuf src_pos;                 // int64: cluster position -> position in the caller's source vector
    DevBuf kappa_c;                 // FP64 [n_bands][N_tgt] kappa at the targets, cluster order
    std::vector<int64_t> leaf_prp_h;   // [n_leaves + 1] prefix sums of the padded leaf rows
    DevBuf leaf_start, leaf_prp;       // device copies of the target-leaf tables
    int kgroup = 1;                    // columns per group in the slices: 1, or 8 (BF16, K-grouped)
    std::vector<int64_t> src_p_h;      // [N_src + 1] cluster source -> stored coordinate; [N_src] = n_src_p
    DevBuf src_p, src_pmap;            // device src_p; src_pmap [n_src_p]: stored coordinate -> source or -1
    int64_t n_src_p = 0;
    // stored width of the source range [s0, s1) (a union of source leaves)
    int64_t pwidth(int64_t s0, int64_t s1) const { return src_p_h[s1] - src_p_h[s0]; }
    MatvecConfig cfg;
    std::vector<std::unique_ptr<MatvecPlan>> mv;   // per band
    std::unique_ptr<MatvecPlan> mv_all;            // all bands in one launch (multi-band matrices)
    rte_hmat_stats_t stats{};
    int device = 0;
    HMat();
    ~HMat();
};

// ---------------------------------------------------------------- entry points implemented in .hip files
void entries_launch(const Mesh &m, int kind, const double *kappa, int64_t n, const int64_t *rows,
                    const int64_t *cols, double *out, int precision, hipStream_t s);
void assemble_band(HMat &H, int band, const double *kappa_band, hipStream_t s);
void band_settle(BandStore &B, hipStream_t s);   // after the band's last queued work
void matvec_reserve(HMat &H, int n_bands);   // room for the per-band plans (before building them concurrently)
void matvec_build(HMat &H, int band, hipStream_t s);
// Operator applied by a matvec on mixed-precision storage: the BF16-hi
// factors with FP32 accumulation (inner sweeps), or hi + lo with FP64
// accumulation (defect steps and external calls).  Other storages ignore it.
constexpr int kMatvecLow = 0;
constexpr int kMatvecAccurate = 1;
void matvec_launch(const HMat &H, int band, int nrhs, const double *x_c, double *y_c, const double *y0_c,
                   hipStream_t s, int mode = kMatvecAccurate);
// Same with a caller-provided workspace of matvec_ws(H, band, nrhs) doubles; does not synchronise.
void matvec_launch_ws(const HMat &H, int band, int nrhs, const double *x_c, double *y_c, const double *y0_c,
                      double *tbuf, hipStream_t s, int mode = kMatvecAccurate);
int64_t matvec_ws(const HMat &H, int band, int nrhs);
// All bands at once: x, y, y0 are [n_bands][nrhs][N] (band-major); workspace
// matvec_ws_all(H, nrhs) doubles.  Does not synchronise.
void matvec_build_all(HMat &H, hipStream_t s);
int64_t matvec_ws_all(const HMat &H, int nrhs);
void matvec_launch_all(const HMat &H, int nrhs, const double *x_c, double *y_c, const double *y0_c, double *tbuf,
                       hipStream_t s, int mode = kMatvecAccurate);
// Rebuild the work lists of every band and of the all-band launch for `cfg`.
void matvec_configure(HMat &H, const MatvecConfig &cfg, hipStream_t s);
// HIP-event time (ms) of one all-band matvec with nrhs right-hand sides, mean of reps.
double matvec_time(const HMat &H, int nrhs, int mode, int reps, hipStream_t s);
// Time every candidate launch shape on H itself, keep the fastest.
MatvecConfig matvec_autotune(HMat &H, int nrhs, int mode, int reps, hipStream_t s, double *best_ms, int *trials);
void permute_gather(const int64_t *perm, int64_t n, int nrhs, int64_t ld_in, int64_t ld_out, const double *in,
                    double *out, hipStream_t s);
void permute_scatter(const int64_t *perm, int64_t n, int nrhs, int64_t ld_in, int64_t ld_out, const double *in,
                     double *out, hipStream_t s);
rte_status_t fixed_point_solve(const Mesh &m, const HMat &G, const HMat &S, const rte_solve_desc_t &d,
                               double *T_out, double *J_out, rte_solve_stats_t *st, hipStream_t s);

}  // namespace rte

struct rte_mesh { rte::Mesh m; };
struct rte_hmat;
namespace rte {
std::unique_ptr<rte_hmat> assemble_hmat(const Mesh &m, std::shared_ptr<const Plan> plan,
                                        const rte_hmat_opts_t &opts, int n_bands, const double *kappa,
                                        hipStream_t s);
}
struct rte_plan { std::unique_ptr<rte::Plan> p; };
struct rte_hmat { rte::HMat h; };
