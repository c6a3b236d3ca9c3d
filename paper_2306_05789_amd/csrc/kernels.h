// Work descriptors shared by the host planners and the kernels.
#pragma once

#include "rte_internal.h"

namespace rte {

constexpr int kFillChunk = 4096;   // entries of a dense block per fill task
constexpr int kAcaMaxRank = 192;   // rank cap of one ACA block before dense fallback
constexpr int kAcaMaxRows = 32768; // LDS bitmap of used pivot rows

struct FillTask {
    void *out;        // first element of the block's column-major storage
    int64_t t0, s0;   // block ranges start, in cluster order
    int32_t m, n;
    int64_t first;    // first entry of this task
};

struct AcaTask {
    int64_t t0, s0;
    int32_t m, n;
    int32_t kcap;     // rank cap (<= min(m n / (m + n), kAcaMaxRank))
    int32_t pad;
    int64_t uoff, voff;   // scratch offsets (elements) of U^T [kcap][m] and V^T [kcap][n]
};

template <typename T> struct EntryCtx;
template <typename T> EntryCtx<T> make_ctx(const Mesh &m, const T *kappa);
void to_float(const double *in, float *out, int64_t n, hipStream_t s);
template <typename T>
void dense_fill_launch(const Mesh &m, int kind, const T *kappa, const std::vector<FillTask> &tasks,
                       const int64_t *tgt_nat, const int64_t *src_nat, hipStream_t s);

}  // namespace rte
