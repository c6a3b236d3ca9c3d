// H-matrix times vector(s): y = H x for nrhs right-hand sides (Section
// "Compression": after compression the fixed point only needs matrix-vector
// products, O(N ln N) each).
//
// Phase A: t_b = V_b^T x[s-range of b] for every low-rank block b.  V is
//          row-major [n][k]; a wavefront takes a chunk of source rows, lane
//          l accumulates t_l and 64/kpad rows are read per step, so loads
//          are contiguous and no per-l reduction is needed.  Blocks larger
//          than one chunk write partial sums that a second pass adds in a
//          fixed order.
// Phase B: one workgroup per target leaf owns its rows: it sums the dense
//          leaves of its block row and the row slices of every low-rank block
//          that covers it, y = y0 + sum_seg D x or U t.  Each of the 4
//          wavefronts takes every 4th segment; lanes are rows, so every load
//          of D or U^T is contiguous; the 4 partial sums are added in a fixed
//          order.  No atomics: results are bitwise reproducible.
#include <algorithm>

#include "kernels.h"

namespace rte {

struct VtTask {
    const void *V;      // first row of the chunk in V [n][k]
    const void *Vlo;    // same position in the BF16 lo part (mixed precision)
    int64_t s0;         // source (cluster order) of the chunk's first row
    int64_t out;        // offset of the result (t buffer, or partial buffer if partial)
    int32_t nj, k;      // rows in the chunk, rank
    int32_t partial, pad;
};

struct VtReduce {
    int64_t part;       // first partial (elements) in the partial buffer
    int64_t toff;       // offset of t_b
    int32_t chunks, k;
};

struct Seg {
    const void *data;   // column-major [K][ld] (dense: x columns; low rank: U^T rows)
    const void *lo;     // BF16 lo part of U^T (mixed precision low rank)
    int64_t coef_off;   // offset into x (dense: s0) or t (low rank: toff)
    int32_t ld, row_off, K, is_lr;
};

struct LeafWork {
    int64_t r0;         // first row (cluster order)
    int32_t rows, seg0, seg1, pad;
};

struct MatvecPlan {
    DevBuf vt, seg, leaf, red;
    int64_t n_vt = 0, n_leaf = 0, ktot = 0, n_red = 0, n_red_threads = 0, npart = 0;
    int64_t n_src = 0, n_tgt = 0;
    int max_rows = 0;
};

namespace {

// factor storage: FP64, FP32, or BF16 (hi part, plus the lo part in MODE_ACC)
enum : int { ST_F64 = 0, ST_F32 = 1, ST_BF16 = 2 };

template <int ST, int MODE, typename A>
__device__ __forceinline__ A load_factor(const void *p, const void *lo, int64_t i) {
    if constexpr (ST == ST_F64) return (A) static_cast<const double *>(p)[i];
    else if constexpr (ST == ST_F32) return (A) static_cast<const float *>(p)[i];
    else {
        A v = (A)bf2f(static_cast<const uint16_t *>(p)[i]);
        if constexpr (MODE == kMatvecAccurate) v += (A)bf2f(static_cast<const uint16_t *>(lo)[i]);
        return v;
    }
}

template <typename A>
__device__ __forceinline__ A wsum(A v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int ST, int MODE, typename A, int NR>
__global__ __launch_bounds__(256) void k_phase_a(const VtTask *__restrict__ tasks, int64_t ntask,
                                                 const double *__restrict__ x, int64_t ldx, double *__restrict__ t,
                                                 int64_t ldt, double *__restrict__ part, int64_t ldp, int r0, int nr) {
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= ntask) return;
    const VtTask tk = tasks[w];
    double *dst = tk.partial ? part : t;
    const int64_t ldd = tk.partial ? ldp : ldt;
    for (int l0 = 0; l0 < tk.k; l0 += 64) {
        const int kk = min(64, tk.k - l0);
        int kp = 1;
        while (kp < kk) kp <<= 1;
        const int G = 64 / kp;
        const int g = lane / kp, l = lane - g * kp;
        const bool live = l < kk;
        A acc[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] = (A)0;
        int jj = g;
        for (; jj + 3 * G < tk.nj; jj += 4 * G) {
            A v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                v[u] = live ? load_factor<ST, MODE, A>(tk.V, tk.Vlo, (int64_t)(jj + u * G) * tk.k + l0 + l) : (A)0;
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                if (r < nr) {
                    const double *xr = x + (int64_t)(r0 + r) * ldx + tk.s0 + jj;
                    acc[r] += v[0] * (A)xr[0] + v[1] * (A)xr[G] + v[2] * (A)xr[2 * G] + v[3] * (A)xr[3 * G];
                }
            }
        }
        for (; jj < tk.nj; jj += G) {
            const A v = live ? load_factor<ST, MODE, A>(tk.V, tk.Vlo, (int64_t)jj * tk.k + l0 + l) : (A)0;
#pragma unroll
            for (int r = 0; r < NR; ++r)
                if (r < nr) acc[r] += v * (A)x[(int64_t)(r0 + r) * ldx + tk.s0 + jj];
        }
        // add the G row groups (lanes l, l + kp, ...) in a fixed order
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (r < nr) {
                A a = acc[r];
                for (int o = kp; o < 64; o <<= 1) a += __shfl_xor(a, o, 64);
                if (g == 0 && live) dst[(int64_t)(r0 + r) * ldd + tk.out + l0 + l] = (double)a;
            }
        }
    }
}

__global__ void k_phase_a_reduce(const VtReduce *__restrict__ red, int64_t nred, const double *__restrict__ part,
                                 int64_t ldp, double *__restrict__ t, int64_t ldt, int r0, int nr) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t item = blockIdx.y;
    if (item >= nred) return;
    const VtReduce rd = red[item];
    if (w >= rd.k) return;
    for (int r = 0; r < nr; ++r) {
        double s = 0.0;
        for (int c = 0; c < rd.chunks; ++c) s += part[(int64_t)(r0 + r) * ldp + rd.part + (int64_t)c * rd.k + w];
        t[(int64_t)(r0 + r) * ldt + rd.toff + w] = s;
    }
}

template <int ST, int MODE, typename A, int NR>
__global__ __launch_bounds__(256) void k_phase_b(const LeafWork *__restrict__ leaves, const Seg *__restrict__ segs,
                                                 const double *__restrict__ x, int64_t ldx,
                                                 const double *__restrict__ t, int64_t ldt,
                                                 const double *__restrict__ y0, double *__restrict__ y, int64_t ldy,
                                                 int r0, int nr) {
    constexpr int SD = ST == ST_F64 ? ST_F64 : ST_F32;   // dense leaves: FP64, else FP32
    __shared__ A part[4][NR][64];
    const LeafWork lw = leaves[blockIdx.x];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int rb = 0; rb < lw.rows; rb += 64) {
        const int row = rb + lane;
        const bool live = row < lw.rows;
        A acc[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] = (A)0;
        for (int s = lw.seg0 + wid; s < lw.seg1; s += 4) {
            const Seg sg = segs[s];
            const int64_t base = sg.row_off + row;
            const double *cb = sg.is_lr ? t : x;
            const int64_t ldc = sg.is_lr ? ldt : ldx;
            const double *cf = cb + sg.coef_off;
            auto ld = [&](int64_t i) -> A {
                return sg.is_lr ? load_factor<ST, MODE, A>(sg.data, sg.lo, i) : load_factor<SD, 0, A>(sg.data, nullptr, i);
            };
            int l = 0;
            for (; l + 4 <= sg.K; l += 4) {
                A d0 = (A)0, d1 = (A)0, d2 = (A)0, d3 = (A)0;
                if (live) {
                    d0 = ld(base + (int64_t)(l + 0) * sg.ld);
                    d1 = ld(base + (int64_t)(l + 1) * sg.ld);
                    d2 = ld(base + (int64_t)(l + 2) * sg.ld);
                    d3 = ld(base + (int64_t)(l + 3) * sg.ld);
                }
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    if (r < nr) {
                        const double *c = cf + (int64_t)(r0 + r) * ldc + l;
                        acc[r] += d0 * (A)c[0] + d1 * (A)c[1] + d2 * (A)c[2] + d3 * (A)c[3];
                    }
                }
            }
            for (; l < sg.K; ++l) {
                const A d = live ? ld(base + (int64_t)l * sg.ld) : (A)0;
#pragma unroll
                for (int r = 0; r < NR; ++r)
                    if (r < nr) acc[r] += d * (A)cf[(int64_t)(r0 + r) * ldc + l];
            }
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) part[wid][r][lane] = acc[r];
        __syncthreads();
        if (wid == 0 && live) {
            const int64_t gr = lw.r0 + row;
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                if (r < nr) {
                    double v = y0 ? y0[(int64_t)(r0 + r) * ldy + gr] : 0.0;
                    v += (double)(((part[0][r][lane] + part[1][r][lane]) + part[2][r][lane]) + part[3][r][lane]);
                    y[(int64_t)(r0 + r) * ldy + gr] = v;
                }
            }
        }
        __syncthreads();
    }
}

__global__ void k_gather(const int64_t *__restrict__ perm, int64_t n, int nrhs, int64_t ld_in, int64_t ld_out,
                         const double *__restrict__ in, double *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n * nrhs) return;
    const int64_t r = k / n, p = k - r * n;
    out[r * ld_out + p] = in[r * ld_in + perm[p]];
}

__global__ void k_scatter(const int64_t *__restrict__ perm, int64_t n, int nrhs, int64_t ld_in, int64_t ld_out,
                          const double *__restrict__ in, double *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n * nrhs) return;
    const int64_t r = k / n, p = k - r * n;
    out[r * ld_out + perm[p]] = in[r * ld_in + p];
}

template <int ST, int MODE, typename A>
void launch_typed(const MatvecPlan &mp, int nrhs, const double *x, const double *y0, double *y, double *tb,
                  hipStream_t s) {
    double *part = tb + mp.ktot * (int64_t)nrhs;   // the workspace holds t, then the partials
    const int64_t ldp = std::max<int64_t>(mp.npart, 1);
    for (int r0 = 0; r0 < nrhs; r0 += 16) {
        const int nr = std::min(16, nrhs - r0);
        if (mp.n_vt) {
            const unsigned ga = (unsigned)((mp.n_vt + 3) / 4);
            const VtTask *vt = mp.vt.as<VtTask>();
            if (nr == 1)
                k_phase_a<ST, MODE, A, 1><<<ga, 256, 0, s>>>(vt, mp.n_vt, x, mp.n_src, tb, mp.ktot, part, ldp, r0, nr);
            else if (nr <= 4)
                k_phase_a<ST, MODE, A, 4><<<ga, 256, 0, s>>>(vt, mp.n_vt, x, mp.n_src, tb, mp.ktot, part, ldp, r0, nr);
            else
                k_phase_a<ST, MODE, A, 16><<<ga, 256, 0, s>>>(vt, mp.n_vt, x, mp.n_src, tb, mp.ktot, part, ldp, r0, nr);
            HIP_LAUNCH_CHECK();
            if (mp.n_red) {
                dim3 grid((unsigned)((mp.n_red_threads + 63) / 64), (unsigned)mp.n_red);
                k_phase_a_reduce<<<grid, 64, 0, s>>>(mp.red.as<VtReduce>(), mp.n_red, part, ldp, tb, mp.ktot, r0, nr);
                HIP_LAUNCH_CHECK();
            }
        }
        const unsigned gb = (unsigned)mp.n_leaf;
        const LeafWork *lw = mp.leaf.as<LeafWork>();
        const Seg *sg = mp.seg.as<Seg>();
        if (nr == 1)
            k_phase_b<ST, MODE, A, 1><<<gb, 256, 0, s>>>(lw, sg, x, mp.n_src, tb, mp.ktot, y0, y, mp.n_tgt, r0, nr);
        else if (nr <= 4)
            k_phase_b<ST, MODE, A, 4><<<gb, 256, 0, s>>>(lw, sg, x, mp.n_src, tb, mp.ktot, y0, y, mp.n_tgt, r0, nr);
        else
            k_phase_b<ST, MODE, A, 16><<<gb, 256, 0, s>>>(lw, sg, x, mp.n_src, tb, mp.ktot, y0, y, mp.n_tgt, r0, nr);
        HIP_LAUNCH_CHECK();
    }
}

}  // namespace

HMat::HMat() = default;
HMat::~HMat() = default;

void matvec_build(HMat &H, int band, hipStream_t s) {
    const Plan &P = *H.plan;
    const BandStore &B = H.bands[band];
    auto mp = std::make_unique<MatvecPlan>();
    mp->n_src = (int64_t)P.src_nat.size();
    mp->n_tgt = (int64_t)P.tgt_nat.size();
    std::vector<VtTask> vt;
    std::vector<VtReduce> red;
    std::vector<int64_t> toff(P.lowrank.size(), -1);
    int64_t ktot = 0, npart = 0, maxk = 0;
    // about this many bytes of V per wavefront task
    const int64_t chunk_bytes = 48 * 1024;
    const int64_t esz = H.precision == RTE_FP64 ? 8 : H.precision == RTE_FP32 ? 4 : 2;
    for (size_t b = 0; b < P.lowrank.size(); ++b) {
        if (B.rank[b] <= 0) continue;
        const Block &bl = P.lowrank[b];
        const int32_t k = B.rank[b];
        const int64_t n = bl.s1 - bl.s0;
        toff[b] = ktot;
        const int64_t rows = std::max<int64_t>(64, chunk_bytes / (k * esz));
        const int64_t chunks = (n + rows - 1) / rows;
        const char *V = static_cast<const char *>(B.V[b]);
        const char *Vl = static_cast<const char *>(B.Vlo.empty() ? nullptr : B.Vlo[b]);
        if (chunks == 1) {
            vt.push_back({V, Vl, bl.s0, ktot, (int32_t)n, k, 0, 0});
        } else {
            red.push_back({npart, ktot, (int32_t)chunks, k});
            for (int64_t c = 0; c < chunks; ++c) {
                const int64_t j0 = c * rows, nj = std::min(rows, n - j0);
                vt.push_back({V + j0 * k * esz, Vl ? Vl + j0 * k * esz : nullptr, bl.s0 + j0, npart + c * k,
                              (int32_t)nj, k, 1, 0});
            }
            npart += chunks * k;
        }
        maxk = std::max<int64_t>(maxk, k);
        ktot += k;
    }
    // large tasks first so that long wavefronts start early
    std::stable_sort(vt.begin(), vt.end(), [](const VtTask &a, const VtTask &b) {
        return (int64_t)a.nj * a.k > (int64_t)b.nj * b.k;
    });
    mp->ktot = std::max<int64_t>(ktot, 1);
    mp->npart = npart;
    mp->n_vt = (int64_t)vt.size();
    mp->n_red = (int64_t)red.size();
    mp->n_red_threads = maxk;
    mp->red = upload(red, s);
    const auto &leaves = P.tgt_leaves;
    std::vector<int64_t> starts;
    for (auto &lf : leaves) starts.push_back(lf.first);
    auto leaf_of = [&](int64_t row) {
        return (int64_t)(std::upper_bound(starts.begin(), starts.end(), row) - starts.begin()) - 1;
    };
    std::vector<std::vector<Seg>> per(leaves.size());
    for (size_t d = 0; d < B.dense_blocks.size(); ++d) {
        const Block &bl = B.dense_blocks[d];
        const int32_t m = (int32_t)(bl.t1 - bl.t0);
        for (int64_t li = leaf_of(bl.t0); li < (int64_t)leaves.size() && leaves[li].first < bl.t1; ++li) {
            per[li].push_back({B.dense_ptr[d], nullptr, bl.s0, m, (int32_t)(leaves[li].first - bl.t0),
                               (int32_t)(bl.s1 - bl.s0), 0});
        }
    }
    // a dense block spanning several leaves is read once per leaf as a column slice
    for (size_t b = 0; b < P.lowrank.size(); ++b) {
        if (B.rank[b] <= 0) continue;
        const Block &bl = P.lowrank[b];
        const int32_t m = (int32_t)(bl.t1 - bl.t0);
        for (int64_t li = leaf_of(bl.t0); li < (int64_t)leaves.size() && leaves[li].first < bl.t1; ++li)
            per[li].push_back({B.U[b], B.Ulo.empty() ? nullptr : B.Ulo[b], toff[b], m,
                               (int32_t)(leaves[li].first - bl.t0), B.rank[b], 1});
    }
    std::vector<Seg> segs;
    std::vector<LeafWork> lw;
    for (size_t li = 0; li < leaves.size(); ++li) {
        LeafWork w{};
        w.r0 = leaves[li].first;
        w.rows = (int32_t)(leaves[li].second - leaves[li].first);
        w.seg0 = (int32_t)segs.size();
        segs.insert(segs.end(), per[li].begin(), per[li].end());
        w.seg1 = (int32_t)segs.size();
        lw.push_back(w);
        mp->max_rows = std::max(mp->max_rows, w.rows);
    }
    mp->n_leaf = (int64_t)lw.size();
    mp->vt = upload(vt, s);
    mp->seg = upload(segs, s);
    mp->leaf = upload(lw, s);
    HIP_CHECK(hipStreamSynchronize(s));
    if ((int)H.mv.size() <= band) H.mv.resize(band + 1);
    H.mv[band] = std::move(mp);
}

// workspace doubles per right-hand side: t, then the partial sums of chunked blocks
int64_t matvec_ktot(const HMat &H, int band) { return H.mv[band]->ktot + H.mv[band]->npart; }

void matvec_launch_ws(const HMat &H, int band, int nrhs, const double *x_c, double *y_c, const double *y0_c,
                      double *tbuf, hipStream_t s, int mode) {
    const MatvecPlan &mp = *H.mv[band];
    if (H.precision == RTE_FP64) launch_typed<ST_F64, 0, double>(mp, nrhs, x_c, y0_c, y_c, tbuf, s);
    else if (H.precision == RTE_FP32) launch_typed<ST_F32, 0, float>(mp, nrhs, x_c, y0_c, y_c, tbuf, s);
    else if (mode == kMatvecAccurate) launch_typed<ST_BF16, kMatvecAccurate, double>(mp, nrhs, x_c, y0_c, y_c, tbuf, s);
    else launch_typed<ST_BF16, kMatvecLow, float>(mp, nrhs, x_c, y0_c, y_c, tbuf, s);
}

void matvec_launch(const HMat &H, int band, int nrhs, const double *x_c, double *y_c, const double *y0_c,
                   hipStream_t s, int mode) {
    DevBuf tb(sizeof(double) * (size_t)matvec_ktot(H, band) * nrhs);
    matvec_launch_ws(H, band, nrhs, x_c, y_c, y0_c, tb.as<double>(), s, mode);
    HIP_CHECK(hipStreamSynchronize(s));
}

void permute_gather(const int64_t *perm, int64_t n, int nrhs, int64_t ld_in, int64_t ld_out, const double *in,
                    double *out, hipStream_t s) {
    const int64_t tot = n * nrhs;
    if (tot == 0) return;
    k_gather<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(perm, n, nrhs, ld_in, ld_out, in, out);
    HIP_LAUNCH_CHECK();
}

void permute_scatter(const int64_t *perm, int64_t n, int nrhs, int64_t ld_in, int64_t ld_out, const double *in,
                     double *out, hipStream_t s) {
    const int64_t tot = n * nrhs;
    if (tot == 0) return;
    k_scatter<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(perm, n, nrhs, ld_in, ld_out, in, out);
    HIP_LAUNCH_CHECK();
}

}  // namespace rte
