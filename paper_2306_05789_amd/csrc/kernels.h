// Work descriptors shared by the host planners and the kernels.
#pragma once

#include "rte_internal.h"

namespace rte {

constexpr int kFillChunk = 4096;   // entries of a dense block per fill task

// bfloat16 as the upper half of an IEEE binary32: round to nearest even on
// the way in (finite inputs), exact widening on the way out.
__host__ __device__ __forceinline__ uint16_t f2bf(float x) {
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__host__ __device__ __forceinline__ float bf2f(uint16_t h) {
    return __builtin_bit_cast(float, (uint32_t)h << 16);
}
constexpr int kAcaMaxRank = 192;     // rank cap of an ACA block in the first pass
constexpr int kAcaRetryRank = 1024;  // cap of the second pass (blocks whose break-even rank is larger)

__host__ __device__ constexpr int64_t pad4(int64_t k) { return (k + 3) & ~(int64_t)3; }
__host__ __device__ constexpr int64_t pad8(int64_t k) { return (k + 7) & ~(int64_t)7; }

// Target-leaf tables of a plan on the device: where an element of a block
// lands in its leaf-sliced storage (see the storage notes in rte_internal.h).
struct SliceMap {
    const int64_t *start;   // [n_leaves + 1]
    const int64_t *prp;     // [n_leaves + 1]
    const int64_t *src_p;   // [N_src + 1] source (cluster order) -> stored column coordinate
    int nleaf;
    int g;                  // columns per group: 1 (column-major slices) or 8 (K-grouped)
};

// Where row `grow` of a block of stored width K (first target leaf li0) sits:
// element (grow, col) is at base + ((col / g) * rp + r) * g + col % g.
struct SliceRow {
    int64_t base, rp, r;
};
// `hi_bound` (optional) is a leaf index known to lie past the row's leaf.
__device__ __forceinline__ SliceRow slice_row(const SliceMap &sm, int li0, int64_t grow, int64_t K,
                                              int hi_bound = 0x7fffffff) {
    int lo = li0, hi = hi_bound < sm.nleaf ? hi_bound : sm.nleaf;   // start[lo] <= grow < start[hi]
    if (hi - lo > 1 && sm.start[lo + 1] > grow) hi = lo + 1;         // in the first leaf: the common case
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (sm.start[mid] <= grow) lo = mid;
        else hi = mid;
    }
    const int64_t g = sm.g, Kp = (K + g - 1) / g * g;
    return {Kp * (sm.prp[lo] - sm.prp[li0]), sm.prp[lo + 1] - sm.prp[lo], grow - sm.start[lo]};
}

// element offset of (row `grow`, stored column `col`) in a block of stored
// width K whose first target leaf is li0
__device__ __forceinline__ int64_t slice_offset(const SliceMap &sm, int li0, int64_t grow, int64_t K, int64_t col,
                                                int hi_bound = 0x7fffffff) {
    const SliceRow sr = slice_row(sm, li0, grow, K, hi_bound);
    const int64_t g = sm.g;
    return sr.base + ((col / g) * sr.rp + sr.r) * g + col % g;
}

struct FillTask {
    void *out;        // first element of the block (leaf-sliced, K = n columns)
    void *outlo;      // BF16 lo part (mixed precision), else null
    int64_t t0, s0;   // block ranges start, in cluster order
    int32_t m, n, li0;
    int32_t kw;       // stored width (columns) of the block
    int64_t first;    // first entry (column-major over m x n) of this task
    // volume operator: the transposed block (rows s0.., columns t0..) filled by
    // the same lanes (the optical depth of a vertex pair is symmetric), or null
    void *out_t, *outlo_t;
    int32_t li0_t, kw_t;
};

struct AcaTask {
    int64_t t0, s0;
    int32_t m, n;
    int32_t kcap;     // rank cap (<= min(m n / (m + n), the pass's cap))
    int32_t pad;
    int64_t uoff, voff;   // scratch offsets (elements) of U^T [kcap][m] and V^T [kcap][n]
};

// Recompression of a batch's ACA factors (recompress.hip): the converged
// blocks of rank 2..96 get the shortest truncation of the SVD of U V^T within
// eps, computed and written in place in the ACA scratch (U^T at uoff, V^T at
// voff); rk[t] becomes the new rank.  Synchronises `s` once per round.
template <typename T>
void recompress_batch(const std::vector<AcaTask> &tasks, std::vector<int> &rk, T *Us, T *Vs, double eps,
                      BandStore &B, hipStream_t s);

// Times the device work enqueued on `s` between start() and stop() with HIP events.
struct EventTimer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    explicit EventTimer(hipStream_t st) : s(st) {
        HIP_CHECK(hipEventCreate(&a));
        HIP_CHECK(hipEventCreate(&b));
    }
    ~EventTimer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    void start() { HIP_CHECK(hipEventRecord(a, s)); }
    void stop() { HIP_CHECK(hipEventRecord(b, s)); }
    double ms() {   // after stop(); synchronises on the stop event
        HIP_CHECK(hipEventSynchronize(b));
        float v = 0.0f;
        HIP_CHECK(hipEventElapsedTime(&v, a, b));
        return (double)v;
    }
};

template <typename T> struct EntryCtx;
// One band's absorption as the entry kernels read it: the vertex values and
// the table the ray march samples (tet_table): FP32 the four vertex values
// of every (cell base, Kuhn tetrahedron) pair, FP64 the eight corner values
// of every cell base.
template <typename T>
struct BandKappa {
    const T *v;     // [N]
    const T *tet;   // FP32 [N][6][4], FP64 [N][8]
};
template <typename T> EntryCtx<T> make_ctx(const Mesh &m, BandKappa<T> kappa);
// the march's table of `kappa` on the mesh, queued on s (scratch; the caller
// keeps it until the launches that read it have run)
template <typename T> DevBuf tet_table(const Mesh &m, const T *kappa, hipStream_t s);
void to_float(const double *in, float *out, int64_t n, hipStream_t s);
// queues the fill on s without waiting: the task list and the launch's event
// pair go to B.retire / B.fill_events (read by band_settle); split: write BF16 hi/lo
template <typename T>
void dense_fill_launch(const Mesh &m, int kind, BandKappa<T> kappa, const std::vector<FillTask> &tasks,
                       const int64_t *tgt_nat, const int64_t *src_nat, SliceMap sm, bool split, BandStore &B,
                       hipStream_t s);

}  // namespace rte
