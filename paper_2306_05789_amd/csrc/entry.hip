// Kernels that evaluate kernel entries directly: arbitrary (row, col) pairs,
// and the dense near-field leaves of the H-matrix (Section "Compression": a
// block that reaches the leaves without being admissible is computed in full).
#include "entry_dev.h"
#include "kernels.h"

namespace rte {

template <typename T, int KIND>
__global__ __launch_bounds__(256) void k_entries(EntryCtx<T> c, int64_t n, const int64_t *__restrict__ rows,
                                                 const int64_t *__restrict__ cols, double *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    out[k] = (double)entry<T, KIND>(c, rows[k], cols[k]);
}

// One task = up to kFillChunk consecutive entries (column-major) of one
// dense block: the lanes of a wavefront march rays from a cluster of targets
// to one source and write contiguous rows of the leaf-sliced storage.  FP64:
// a task is spread over kFillChunk / 256 workgroups of one entry per thread
// (with a loop over entries the compiler hoists the quadrature tables'
// uniform loads into scalar registers, which spill at FP64 width and cost
// an occupancy step).  FP32: one workgroup loops over the task's entries,
// the hoisted tables being the cheaper form there (measured: 2x faster).
template <typename T>
constexpr int fill_split() { return sizeof(T) == 8 ? kFillChunk / 256 : 1; }
static_assert(kFillChunk % 256 == 0, "fill tasks are whole workgroups");

// KIND of the tasks that fill a volume block and its transpose together
constexpr int kPairedVolume = 2;

template <typename T, int KIND, bool SPLIT, int NW>
__device__ __forceinline__ void fill_one(const EntryCtx<T> &c, const FillTask &tk, int64_t e,
                                         const int64_t *__restrict__ tgt_nat, const int64_t *__restrict__ src_nat,
                                         const SliceMap &sm) {
    const int64_t jl = e / tk.m, il = e - jl * tk.m;
    auto put = [&](void *out, void *outlo, int64_t o, T v) {
        if constexpr (SPLIT) {
            const uint16_t h = f2bf((float)v);
            static_cast<uint16_t *>(out)[o] = h;
            static_cast<uint16_t *>(outlo)[o] = f2bf((float)v - bf2f(h));
        } else {
            static_cast<T *>(out)[o] = v;
        }
    };
    // the stored positions are looked up after the entries (not live through the march)
    if constexpr (KIND == kPairedVolume) {
        // this entry and its transpose (the volume tree's targets and sources coincide)
        T v, vt;
        volume_entry_pair<T, NW>(c, tgt_nat[tk.t0 + il], tgt_nat[tk.s0 + jl], v, vt);
        put(tk.out, tk.outlo,
            slice_offset(sm, tk.li0, tk.t0 + il, tk.kw, sm.src_p[tk.s0 + jl] - sm.src_p[tk.s0], tk.li0 + (int)il + 1),
            v);
        put(tk.out_t, tk.outlo_t,
            slice_offset(sm, tk.li0_t, tk.s0 + jl, tk.kw_t, sm.src_p[tk.t0 + il] - sm.src_p[tk.t0],
                         tk.li0_t + (int)jl + 1),
            vt);
    } else {
        const T v = entry<T, KIND, NW>(c, tgt_nat[tk.t0 + il], src_nat[tk.s0 + jl]);
        put(tk.out, tk.outlo,
            slice_offset(sm, tk.li0, tk.t0 + il, tk.kw, sm.src_p[tk.s0 + jl] - sm.src_p[tk.s0], tk.li0 + (int)il + 1),
            v);
    }
}

template <typename T, int KIND, bool SPLIT, int NW>
__global__ __launch_bounds__(256, sizeof(T) == 8 ? 4 : 3) void k_dense_fill(EntryCtx<T> c,
                                                                        const FillTask *__restrict__ tasks,
                                                                        const int64_t *__restrict__ tgt_nat,
                                                                        const int64_t *__restrict__ src_nat,
                                                                        SliceMap sm) {
    constexpr int split = fill_split<T>();
    const FillTask tk = tasks[blockIdx.x / split];
    const int64_t total = (int64_t)tk.m * tk.n;
    if constexpr (split == kFillChunk / 256) {
        const int64_t e = tk.first + (int64_t)(blockIdx.x % split) * 256 + threadIdx.x;
        if (e < total) fill_one<T, KIND, SPLIT, NW>(c, tk, e, tgt_nat, src_nat, sm);
    } else {
        const int64_t end = min(total, tk.first + (int64_t)kFillChunk);
        for (int64_t e = tk.first + threadIdx.x; e < end; e += blockDim.x)
            fill_one<T, KIND, SPLIT, NW>(c, tk, e, tgt_nat, src_nat, sm);
    }
}

__global__ void k_to_float(const double *__restrict__ in, float *__restrict__ out, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = (float)in[k];
}

void to_float(const double *in, float *out, int64_t n, hipStream_t s) {
    if (n == 0) return;
    k_to_float<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(in, out, n);
    HIP_LAUNCH_CHECK();
}

// The four vertex values of every (cell base b, Kuhn tetrahedron t) pair, in
// the order tet_sample reads them: b, b + s_L, b + s0 + s1 + 1 - s_S and
// b + s0 + s1 + 1, L and S the tetrahedron's largest and smallest axes
// (t = 2 L + (S > L ? S - 1 : S)).  A vertex past the grid (bases on the
// upper faces) gives 0.
template <typename T>
__global__ void k_tet_table(GridDev g, const T *__restrict__ kap, T *__restrict__ out) {
    const int64_t N = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N * 6) return;
    const int64_t b = k / 6;
    const int t = (int)(k - b * 6), L = t >> 1, r = t & 1, S = r < L ? r : r + 1;
    const int64_t s0 = g.stride[0], s1 = g.stride[1];
    const int64_t sL = L == 0 ? s0 : (L == 1 ? s1 : 1), sS = S == 0 ? s0 : (S == 1 ? s1 : 1);
    const int64_t v3 = b + s0 + s1 + 1;
    const int64_t v1 = b + sL, v2 = v3 - sS;
    out[4 * k + 0] = kap[b];
    out[4 * k + 1] = v1 < N ? kap[v1] : (T)0;
    out[4 * k + 2] = v2 < N ? kap[v2] : (T)0;
    out[4 * k + 3] = v3 < N ? kap[v3] : (T)0;
}

// FP64: the eight corner values of every cell base b, in the order
// b, b + s0 + s1 + 1, b + s0, b + s1, b + 1, b + s0 + s1, b + s1 + 1, b + s0 + 1
// (a vertex past the grid gives 0)
__global__ void k_cell_table(GridDev g, const double *__restrict__ kap, double *__restrict__ out) {
    const int64_t N = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= N) return;
    const int64_t s0 = g.stride[0], s1 = g.stride[1];
    const int64_t v[8] = {b, b + s0 + s1 + 1, b + s0, b + s1, b + 1, b + s0 + s1, b + s1 + 1, b + s0 + 1};
#pragma unroll
    for (int q = 0; q < 8; ++q) out[8 * b + q] = v[q] < N ? kap[v[q]] : 0.0;
}

template <typename T>
DevBuf tet_table(const Mesh &m, const T *kappa, hipStream_t s) {
    if constexpr (sizeof(T) == 4) {
        DevBuf d = DevBuf::scratch(sizeof(T) * (size_t)m.N * 24);
        const int64_t n = m.N * 6;
        k_tet_table<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(m.dev, kappa, d.as<T>());
        HIP_LAUNCH_CHECK();
        return d;
    } else {
        DevBuf d = DevBuf::scratch(sizeof(T) * (size_t)m.N * 8);
        k_cell_table<<<(unsigned)((m.N + 255) / 256), 256, 0, s>>>(m.dev, kappa, d.as<T>());
        HIP_LAUNCH_CHECK();
        return d;
    }
}
template DevBuf tet_table<float>(const Mesh &, const float *, hipStream_t);
template DevBuf tet_table<double>(const Mesh &, const double *, hipStream_t);

template <typename T>
EntryCtx<T> make_ctx(const Mesh &m, BandKappa<T> kappa) {
    EntryCtx<T> c;
    c.g = m.dev;
    c.kappa = kappa.v;
    c.ktet = kappa.tet;
    c.near = static_cast<const T *>(m.near_table(std::is_same<T, double>::value));
    if constexpr (std::is_same<T, double>::value) c.st = stencil_device().d;
    else c.st = stencil_device().f;
    return c;
}
template EntryCtx<double> make_ctx<double>(const Mesh &, BandKappa<double>);
template EntryCtx<float> make_ctx<float>(const Mesh &, BandKappa<float>);

void entries_launch(const Mesh &m, int kind, const double *kappa, int64_t n, const int64_t *rows,
                    const int64_t *cols, double *out, int precision, hipStream_t s) {
    if (n == 0) return;
    const unsigned grid = (unsigned)((n + 255) / 256);
    if (precision == RTE_FP64) {
        DevBuf kt = tet_table<double>(m, kappa, s);
        auto c = make_ctx<double>(m, BandKappa<double>{kappa, kt.as<double>()});
        if (kind == RTE_VOLUME) k_entries<double, RTE_VOLUME><<<grid, 256, 0, s>>>(c, n, rows, cols, out);
        else k_entries<double, RTE_SURFACE><<<grid, 256, 0, s>>>(c, n, rows, cols, out);
        HIP_LAUNCH_CHECK();
        HIP_CHECK(hipStreamSynchronize(s));   // kt is released on return
    } else {
        DevBuf kf(sizeof(float) * (size_t)m.N);
        to_float(kappa, kf.as<float>(), m.N, s);
        DevBuf kt = tet_table<float>(m, kf.as<float>(), s);
        auto c = make_ctx<float>(m, BandKappa<float>{kf.as<float>(), kt.as<float>()});
        if (kind == RTE_VOLUME) k_entries<float, RTE_VOLUME><<<grid, 256, 0, s>>>(c, n, rows, cols, out);
        else k_entries<float, RTE_SURFACE><<<grid, 256, 0, s>>>(c, n, rows, cols, out);
        HIP_LAUNCH_CHECK();
        HIP_CHECK(hipStreamSynchronize(s));   // kf and kt are released on return
    }
}

template <typename T>
void dense_fill_launch(const Mesh &m, int kind, BandKappa<T> kappa, const std::vector<FillTask> &tasks,
                       const int64_t *tgt_nat, const int64_t *src_nat, SliceMap sm, bool split, BandStore &B,
                       hipStream_t s) {
    if (tasks.empty()) return;
    // the paired tasks (volume block and transpose) first, then the single ones
    std::vector<FillTask> order;
    order.reserve(tasks.size());
    for (const FillTask &t : tasks)
        if (t.out_t) order.push_back(t);
    const size_t npair = order.size();
    for (const FillTask &t : tasks)
        if (!t.out_t) order.push_back(t);
    RTE_REQUIRE(npair == 0 || kind == RTE_VOLUME, "dense fill: paired tasks are for the volume operator");
    if (order.size() > ((size_t)1 << 31) / fill_split<T>())
        throw std::runtime_error("dense fill: too many tasks for one grid");
    DevBuf dt = upload_scratch(order, s);
    auto c = make_ctx<T>(m, kappa);
    const FillTask *d = dt.as<FillTask>();
    const unsigned gp = (unsigned)(npair * fill_split<T>()), gs = (unsigned)((order.size() - npair) * fill_split<T>());
    const FillTask *ds = d + npair;
    EventPair ev;
    HIP_CHECK(hipEventRecord(ev.a, s));
    auto launch = [&](auto nw) {
        constexpr int NW = decltype(nw)::value;
        if (split) {
            if (gp) k_dense_fill<T, kPairedVolume, true, NW><<<gp, 256, 0, s>>>(c, d, tgt_nat, src_nat, sm);
            if (gs && kind == RTE_VOLUME) k_dense_fill<T, RTE_VOLUME, true, NW><<<gs, 256, 0, s>>>(c, ds, tgt_nat, src_nat, sm);
            else if (gs) k_dense_fill<T, RTE_SURFACE, true, NW><<<gs, 256, 0, s>>>(c, ds, tgt_nat, src_nat, sm);
        } else {
            if (gp) k_dense_fill<T, kPairedVolume, false, NW><<<gp, 256, 0, s>>>(c, d, tgt_nat, src_nat, sm);
            if (gs && kind == RTE_VOLUME) k_dense_fill<T, RTE_VOLUME, false, NW><<<gs, 256, 0, s>>>(c, ds, tgt_nat, src_nat, sm);
            else if (gs) k_dense_fill<T, RTE_SURFACE, false, NW><<<gs, 256, 0, s>>>(c, ds, tgt_nat, src_nat, sm);
        }
    };
    switch (wall_mode(m.dev)) {
        case kNoWall: launch(std::integral_constant<int, kNoWall>()); break;
        case kOneWall: launch(std::integral_constant<int, kOneWall>()); break;
        default: launch(std::integral_constant<int, kAnyWalls>()); break;
    }
    HIP_LAUNCH_CHECK();
    HIP_CHECK(hipEventRecord(ev.b, s));
    B.fill_events.push_back(std::move(ev));
    B.retire.push_back(std::move(dt));   // read by the queued launches
}
template void dense_fill_launch<double>(const Mesh &, int, BandKappa<double>, const std::vector<FillTask> &,
                                        const int64_t *, const int64_t *, SliceMap, bool, BandStore &, hipStream_t);
template void dense_fill_launch<float>(const Mesh &, int, BandKappa<float>, const std::vector<FillTask> &,
                                       const int64_t *, const int64_t *, SliceMap, bool, BandStore &, hipStream_t);

}  // namespace rte
