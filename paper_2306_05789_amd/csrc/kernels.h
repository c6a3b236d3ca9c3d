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
constexpr int kAcaMaxRank = 192;   // rank cap of one ACA block before dense fallback

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
template <typename T> EntryCtx<T> make_ctx(const Mesh &m, const T *kappa);
void to_float(const double *in, float *out, int64_t n, hipStream_t s);
// returns the HIP-event time of the fill launch in ms
template <typename T>
double dense_fill_launch(const Mesh &m, int kind, const T *kappa, const std::vector<FillTask> &tasks,
                         const int64_t *tgt_nat, const int64_t *src_nat, hipStream_t s);

}  // namespace rte
