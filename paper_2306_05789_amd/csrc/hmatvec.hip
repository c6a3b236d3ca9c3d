// H-matrix times vector(s): y = H x for nrhs right-hand sides (Section
// "Compression": after compression the fixed point only needs matrix-vector
// products, O(N ln N) each).
//
// Phase A: t_b = V_b^T x[s-range of b] for every low-rank block b (one
//          wavefront per block, lanes along the source points, V^T rows
//          contiguous).
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
    const void *V;      // V^T [k][n]
    int64_t s0;         // first source (cluster order)
    int64_t toff;       // offset of t_b in the t buffer
    int32_t n, k;
};

struct Seg {
    const void *data;   // column-major [K][ld] (dense: x columns; low rank: U^T rows)
    int64_t coef_off;   // offset into x (dense: s0) or t (low rank: toff)
    int32_t ld, row_off, K, is_lr;
};

struct LeafWork {
    int64_t r0;         // first row (cluster order)
    int32_t rows, seg0, seg1, pad;
};

struct MatvecPlan {
    DevBuf vt, seg, leaf;
    int64_t n_vt = 0, n_leaf = 0, ktot = 0;
    int64_t n_src = 0, n_tgt = 0;
    int max_rows = 0;
};

namespace {

template <typename T>
__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename T, int NR>
__global__ __launch_bounds__(256) void k_phase_a(const VtTask *__restrict__ tasks, int64_t ntask,
                                                 const double *__restrict__ x, int64_t ldx, double *__restrict__ t,
                                                 int64_t ldt, int r0, int nr) {
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= ntask) return;
    const VtTask tk = tasks[w];
    const T *V = static_cast<const T *>(tk.V);
    for (int l = 0; l < tk.k; ++l) {
        double acc[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] = 0.0;
        const T *row = V + (int64_t)l * tk.n;
        for (int j = lane; j < tk.n; j += 64) {
            const double v = (double)row[j];
#pragma unroll
            for (int r = 0; r < NR; ++r)
                if (r < nr) acc[r] += v * x[(int64_t)(r0 + r) * ldx + tk.s0 + j];
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (r < nr) {
                const double s = wsum<T>(acc[r]);
                if (lane == 0) t[(int64_t)(r0 + r) * ldt + tk.toff + l] = s;
            }
        }
    }
}

template <typename T, typename A, int NR>
__global__ __launch_bounds__(256) void k_phase_b(const LeafWork *__restrict__ leaves, const Seg *__restrict__ segs,
                                                 const double *__restrict__ x, int64_t ldx,
                                                 const double *__restrict__ t, int64_t ldt,
                                                 const double *__restrict__ y0, double *__restrict__ y, int64_t ldy,
                                                 int r0, int nr) {
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
            const T *D = static_cast<const T *>(sg.data) + sg.row_off + row;
            const double *cb = sg.is_lr ? t : x;
            const int64_t ldc = sg.is_lr ? ldt : ldx;
            const double *cf = cb + sg.coef_off;
            int l = 0;
            for (; l + 4 <= sg.K; l += 4) {
                A d0 = (A)0, d1 = (A)0, d2 = (A)0, d3 = (A)0;
                if (live) {
                    d0 = (A)D[(int64_t)(l + 0) * sg.ld];
                    d1 = (A)D[(int64_t)(l + 1) * sg.ld];
                    d2 = (A)D[(int64_t)(l + 2) * sg.ld];
                    d3 = (A)D[(int64_t)(l + 3) * sg.ld];
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
                const A d = live ? (A)D[(int64_t)l * sg.ld] : (A)0;
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

template <typename T, typename A>
void launch_typed(const MatvecPlan &mp, int nrhs, const double *x, const double *y0, double *y, double *tb,
                  hipStream_t s) {
    for (int r0 = 0; r0 < nrhs; r0 += 16) {
        const int nr = std::min(16, nrhs - r0);
        if (mp.n_vt) {
            const unsigned ga = (unsigned)((mp.n_vt + 3) / 4);
            if (nr == 1) k_phase_a<T, 1><<<ga, 256, 0, s>>>(mp.vt.as<VtTask>(), mp.n_vt, x, mp.n_src, tb, mp.ktot, r0, nr);
            else if (nr <= 4) k_phase_a<T, 4><<<ga, 256, 0, s>>>(mp.vt.as<VtTask>(), mp.n_vt, x, mp.n_src, tb, mp.ktot, r0, nr);
            else k_phase_a<T, 16><<<ga, 256, 0, s>>>(mp.vt.as<VtTask>(), mp.n_vt, x, mp.n_src, tb, mp.ktot, r0, nr);
            HIP_LAUNCH_CHECK();
        }
        const unsigned gb = (unsigned)mp.n_leaf;
        if (nr == 1)
            k_phase_b<T, A, 1><<<gb, 256, 0, s>>>(mp.leaf.as<LeafWork>(), mp.seg.as<Seg>(), x, mp.n_src, tb, mp.ktot,
                                                  y0, y, mp.n_tgt, r0, nr);
        else if (nr <= 4)
            k_phase_b<T, A, 4><<<gb, 256, 0, s>>>(mp.leaf.as<LeafWork>(), mp.seg.as<Seg>(), x, mp.n_src, tb, mp.ktot,
                                                  y0, y, mp.n_tgt, r0, nr);
        else
            k_phase_b<T, A, 16><<<gb, 256, 0, s>>>(mp.leaf.as<LeafWork>(), mp.seg.as<Seg>(), x, mp.n_src, tb,
                                                   mp.ktot, y0, y, mp.n_tgt, r0, nr);
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
    std::vector<int64_t> toff(P.lowrank.size(), -1);
    int64_t ktot = 0;
    for (size_t b = 0; b < P.lowrank.size(); ++b) {
        if (B.rank[b] <= 0) continue;
        const Block &bl = P.lowrank[b];
        toff[b] = ktot;
        vt.push_back({B.V[b], bl.s0, ktot, (int32_t)(bl.s1 - bl.s0), B.rank[b]});
        ktot += B.rank[b];
    }
    // wide blocks first so that long wavefronts start early
    std::stable_sort(vt.begin(), vt.end(), [](const VtTask &a, const VtTask &b) {
        return (int64_t)a.n * a.k > (int64_t)b.n * b.k;
    });
    mp->ktot = std::max<int64_t>(ktot, 1);
    mp->n_vt = (int64_t)vt.size();
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
            per[li].push_back({B.dense_ptr[d], bl.s0, m, (int32_t)(leaves[li].first - bl.t0),
                               (int32_t)(bl.s1 - bl.s0), 0});
        }
    }
    // a dense block spanning several leaves is read once per leaf as a column slice
    for (size_t b = 0; b < P.lowrank.size(); ++b) {
        if (B.rank[b] <= 0) continue;
        const Block &bl = P.lowrank[b];
        const int32_t m = (int32_t)(bl.t1 - bl.t0);
        for (int64_t li = leaf_of(bl.t0); li < (int64_t)leaves.size() && leaves[li].first < bl.t1; ++li)
            per[li].push_back({B.U[b], toff[b], m, (int32_t)(leaves[li].first - bl.t0), B.rank[b], 1});
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

int64_t matvec_ktot(const HMat &H, int band) { return H.mv[band]->ktot; }

void matvec_launch_ws(const HMat &H, int band, int nrhs, const double *x_c, double *y_c, const double *y0_c,
                      double *tbuf, hipStream_t s) {
    const MatvecPlan &mp = *H.mv[band];
    if (H.precision == RTE_FP64) launch_typed<double, double>(mp, nrhs, x_c, y0_c, y_c, tbuf, s);
    else launch_typed<float, float>(mp, nrhs, x_c, y0_c, y_c, tbuf, s);
}

void matvec_launch(const HMat &H, int band, int nrhs, const double *x_c, double *y_c, const double *y0_c,
                   hipStream_t s) {
    DevBuf tb(sizeof(double) * (size_t)H.mv[band]->ktot * nrhs);
    matvec_launch_ws(H, band, nrhs, x_c, y_c, y0_c, tb.as<double>(), s);
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
