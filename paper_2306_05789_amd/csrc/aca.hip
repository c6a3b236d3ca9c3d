// Assembly of one band of an H-matrix: dense near-field leaves and partially
// pivoted ACA of the admissible blocks (Section "Compression": only r rows
// and r columns of a block are computed, r being the rank reached for the
// relative Frobenius tolerance eps).
//
// One admissible block per workgroup of 256 lanes.  Rank step k:
//   1. residual row  r_j = A(i*, j) - sum_l U_l(i*) V_l(j)       (entries in parallel)
//   2. pivot j* = argmax |r_j| (ties: lowest j), v_k = r / r_{j*}
//   3. residual column u_k(i) = A(i, j*) - sum_l V_l(j*) U_l(i)
//   4. ||S_k||^2 += ||u_k||^2 ||v_k||^2 + 2 sum_l (u_l.u_k)(v_l.v_k)
//   5. stop when ||u_k|| ||v_k|| <= eps ||S_k||; next row i* = argmax |u_k| over unused rows.
// The first row is local row 0.  A zero residual row is marked used and the
// lowest unused row is taken instead.  A block that reaches
// k = floor(m n / (m + n)) without converging is stored dense.
// Reductions go through wavefront shuffles and one LDS stage in a fixed
// order, so results are bitwise reproducible.
#include <algorithm>
#include <climits>
#include <numeric>

#include "entry_dev.h"
#include "kernels.h"

namespace rte {

namespace {

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// argmax of |value| with ties to the lowest index; carries the signed value
template <typename T>
__device__ __forceinline__ void wave_argmax(T &a, int &idx, T &sv) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const T oa = __shfl_xor(a, o, 64);
        const int oi = __shfl_xor(idx, o, 64);
        const T os = __shfl_xor(sv, o, 64);
        if (oa > a || (oa == a && oi < idx)) { a = oa; idx = oi; sv = os; }
    }
}

template <typename T>
__device__ __forceinline__ void combine4(const T *va, const int *vi, const T *vs, T &a, int &idx, T &sv) {
    a = va[0]; idx = vi[0]; sv = vs[0];
#pragma unroll
    for (int w = 1; w < 4; ++w)
        if (va[w] > a || (va[w] == a && vi[w] < idx)) { a = va[w]; idx = vi[w]; sv = vs[w]; }
}

}  // namespace

template <typename T, int KIND>
__global__ __launch_bounds__(256) void k_aca(EntryCtx<T> c, const AcaTask *__restrict__ tasks,
                                             const int64_t *__restrict__ tgt_nat,
                                             const int64_t *__restrict__ src_nat, T *__restrict__ Us,
                                             T *__restrict__ Vs, int *__restrict__ ranks, T eps) {
    __shared__ unsigned used[kAcaMaxRows / 32];
    __shared__ T red_u[4][kAcaMaxRank + 1];
    __shared__ T red_v[4][kAcaMaxRank + 1];
    __shared__ T ra[4], rs[4], ca[4], cs[4];
    __shared__ int ri[4], ci[4];
    __shared__ int s_ctrl[2];

    const AcaTask tk = tasks[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    T *U = Us + tk.uoff;
    T *V = Vs + tk.voff;
    const int m = tk.m, n = tk.n;
    for (int w = tid; w < (m + 31) / 32; w += 256) used[w] = 0u;
    __syncthreads();

    int k = 0, istar = 0;
    bool conv = false;
    T normS2 = (T)0;   // meaningful in thread 0 only
    const int max_iter = tk.kcap + m + 1;
    for (int iter = 0; iter < max_iter; ++iter) {
        if (tid == 0) used[istar >> 5] |= 1u << (istar & 31);
        // 1. residual row i*
        const int64_t gi = tgt_nat[tk.t0 + istar];
        T best = (T)-1, bsv = (T)0;
        int bj = INT_MAX;
        for (int j = tid; j < n; j += 256) {
            T a = entry<T, KIND>(c, gi, src_nat[tk.s0 + j]);
            for (int l = 0; l < k; ++l) a -= U[(int64_t)l * m + istar] * V[(int64_t)l * n + j];
            V[(int64_t)k * n + j] = a;
            const T av = fabs(a);
            if (av > best) { best = av; bj = j; bsv = a; }
        }
        // 2. pivot column
        wave_argmax(best, bj, bsv);
        if (lane == 0) { ra[wid] = best; ri[wid] = bj; rs[wid] = bsv; }
        __syncthreads();
        combine4(ra, ri, rs, best, bj, bsv);
        if (!(best > (T)0)) {
            // zero residual row: continue from the lowest unused row
            if (tid == 0) {
                int cand = -1;
                for (int r = 0; r < m && cand < 0; ++r)
                    if (!((used[r >> 5] >> (r & 31)) & 1u)) cand = r;
                s_ctrl[1] = cand;
            }
            __syncthreads();
            const int cand = s_ctrl[1];
            __syncthreads();
            if (cand < 0) { conv = true; break; }
            istar = cand;
            continue;
        }
        const T inv = (T)1 / bsv;
        T nv2 = (T)0;
        for (int j = tid; j < n; j += 256) {
            const T v = V[(int64_t)k * n + j] * inv;
            V[(int64_t)k * n + j] = v;
            nv2 += v * v;
        }
        __syncthreads();   // V_k(j*) and earlier V_l(j*) are read by every lane below
        // 3. residual column j*
        const int64_t gj = src_nat[tk.s0 + bj];
        T bu = (T)-1, busv = (T)0, nu2 = (T)0;
        int bi = INT_MAX;
        for (int i = tid; i < m; i += 256) {
            T a = entry<T, KIND>(c, tgt_nat[tk.t0 + i], gj);
            for (int l = 0; l < k; ++l) a -= V[(int64_t)l * n + bj] * U[(int64_t)l * m + i];
            U[(int64_t)k * m + i] = a;
            nu2 += a * a;
            const T av = fabs(a);
            if (!((used[i >> 5] >> (i & 31)) & 1u) && av > bu) { bu = av; bi = i; busv = a; }
        }
        // 4. Frobenius norm update (each lane reads only the elements it wrote)
        for (int l = 0; l < k; ++l) {
            T pu = (T)0, pv = (T)0;
            for (int i = tid; i < m; i += 256) pu += U[(int64_t)l * m + i] * U[(int64_t)k * m + i];
            for (int j = tid; j < n; j += 256) pv += V[(int64_t)l * n + j] * V[(int64_t)k * n + j];
            pu = wave_sum(pu);
            pv = wave_sum(pv);
            if (lane == 0) { red_u[wid][l] = pu; red_v[wid][l] = pv; }
        }
        nu2 = wave_sum(nu2);
        nv2 = wave_sum(nv2);
        if (lane == 0) { red_u[wid][k] = nu2; red_v[wid][k] = nv2; }
        wave_argmax(bu, bi, busv);
        if (lane == 0) { ca[wid] = bu; ci[wid] = bi; cs[wid] = busv; }
        __syncthreads();
        if (tid == 0) {
            T cross = (T)0;
            for (int l = 0; l < k; ++l)
                cross += (red_u[0][l] + red_u[1][l] + red_u[2][l] + red_u[3][l]) *
                         (red_v[0][l] + red_v[1][l] + red_v[2][l] + red_v[3][l]);
            const T u2 = red_u[0][k] + red_u[1][k] + red_u[2][k] + red_u[3][k];
            const T v2 = red_v[0][k] + red_v[1][k] + red_v[2][k] + red_v[3][k];
            normS2 += u2 * v2 + (T)2 * cross;
            s_ctrl[0] = (sqrt(u2 * v2) <= eps * sqrt(fabs(normS2))) ? 1 : 0;
        }
        combine4(ca, ci, cs, bu, bi, busv);
        __syncthreads();
        const int stop = s_ctrl[0];
        ++k;
        if (stop) { conv = true; break; }
        if (k >= tk.kcap) break;
        if (bi == INT_MAX) { conv = true; break; }   // every row used: the residual is zero
        istar = bi;
    }
    if (tid == 0) ranks[blockIdx.x] = conv ? k : -1;
}

struct CompactTask {
    const void *su, *sv;
    void *du, *dv;
    int64_t nu, nv;   // elements to copy
};

template <typename T>
__global__ __launch_bounds__(256) void k_compact(const CompactTask *__restrict__ tasks) {
    const CompactTask t = tasks[blockIdx.x];
    const T *su = static_cast<const T *>(t.su), *sv = static_cast<const T *>(t.sv);
    T *du = static_cast<T *>(t.du), *dv = static_cast<T *>(t.dv);
    for (int64_t e = threadIdx.x; e < t.nu; e += blockDim.x) du[e] = su[e];
    for (int64_t e = threadIdx.x; e < t.nv; e += blockDim.x) dv[e] = sv[e];
}

// ---------------------------------------------------------------- host side

namespace {

template <typename T>
void fill_dense_blocks(HMat &H, BandStore &B, const T *kap, const std::vector<Block> &blocks, hipStream_t s) {
    if (blocks.empty()) return;
    int64_t total = 0;
    for (auto &b : blocks) total += (b.t1 - b.t0) * (b.s1 - b.s0);
    DevBuf buf(sizeof(T) * (size_t)total);
    std::vector<FillTask> tasks;
    int64_t off = 0;
    for (auto &b : blocks) {
        const int m = (int)(b.t1 - b.t0), n = (int)(b.s1 - b.s0);
        T *p = buf.as<T>() + off;
        B.dense_blocks.push_back(b);
        B.dense_ptr.push_back(p);
        for (int64_t f = 0; f < (int64_t)m * n; f += kFillChunk) tasks.push_back({p, b.t0, b.s0, m, n, f});
        off += (int64_t)m * n;
    }
    B.fill_ms += dense_fill_launch<T>(*H.mesh, H.kind, kap, tasks, H.tgt_nat.as<int64_t>(), H.src_nat.as<int64_t>(), s);
    B.fill_launches += 1;
    B.dense_entries += total;
    B.evaluated += total;
    B.bytes += (int64_t)buf.bytes;
    B.bufs.push_back(std::move(buf));
}

template <typename T>
void run_aca(HMat &H, BandStore &B, const T *kap, hipStream_t s) {
    const Plan &P = *H.plan;
    const size_t nlr = P.lowrank.size();
    B.rank.assign(nlr, -1);
    B.U.assign(nlr, nullptr);
    B.V.assign(nlr, nullptr);
    std::vector<Block> fallback;
    std::vector<size_t> order;
    for (size_t b = 0; b < nlr; ++b) {
        const Block &bl = P.lowrank[b];
        const int64_t m = bl.t1 - bl.t0, n = bl.s1 - bl.s0;
        const int64_t kcap = std::min<int64_t>(m * n / (m + n), kAcaMaxRank);
        if (kcap < 1 || m > kAcaMaxRows) fallback.push_back(bl);
        else order.push_back(b);
    }
    // large blocks first: they take longest
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
        const Block &x = P.lowrank[a], &y = P.lowrank[b];
        return (x.t1 - x.t0) + (x.s1 - x.s0) > (y.t1 - y.t0) + (y.s1 - y.s0);
    });
    const T eps = (T)P.opts.aca_eps;
    const size_t scratch_limit = (size_t)6 << 30;   // bytes of U/V scratch per batch
    auto c = make_ctx<T>(*H.mesh, kap);
    size_t pos = 0;
    while (pos < order.size()) {
        std::vector<AcaTask> tasks;
        std::vector<size_t> ids;
        int64_t uo = 0, vo = 0;
        while (pos < order.size()) {
            const Block &bl = P.lowrank[order[pos]];
            const int32_t m = (int32_t)(bl.t1 - bl.t0), n = (int32_t)(bl.s1 - bl.s0);
            const int32_t kcap = (int32_t)std::min<int64_t>((int64_t)m * n / (m + n), kAcaMaxRank);
            const int64_t need = (int64_t)kcap * (m + n);
            if (!tasks.empty() && (size_t)(uo + vo + need) * sizeof(T) > scratch_limit) break;
            tasks.push_back({bl.t0, bl.s0, m, n, kcap, 0, uo, vo});
            ids.push_back(order[pos]);
            uo += (int64_t)kcap * m;
            vo += (int64_t)kcap * n;
            ++pos;
        }
        DevBuf Us(sizeof(T) * (size_t)uo), Vs(sizeof(T) * (size_t)vo), dr(sizeof(int) * tasks.size());
        DevBuf dt = upload(tasks, s);
        EventTimer tm(s);
        tm.start();
        if (H.kind == RTE_VOLUME)
            k_aca<T, RTE_VOLUME><<<(unsigned)tasks.size(), 256, 0, s>>>(c, dt.as<AcaTask>(), H.tgt_nat.as<int64_t>(),
                                                                    H.src_nat.as<int64_t>(), Us.as<T>(), Vs.as<T>(),
                                                                    dr.as<int>(), eps);
        else
            k_aca<T, RTE_SURFACE><<<(unsigned)tasks.size(), 256, 0, s>>>(c, dt.as<AcaTask>(), H.tgt_nat.as<int64_t>(),
                                                                     H.src_nat.as<int64_t>(), Us.as<T>(), Vs.as<T>(),
                                                                     dr.as<int>(), eps);
        HIP_LAUNCH_CHECK();
        tm.stop();
        B.aca_ms += tm.ms();
        B.aca_launches += 1;
        std::vector<int> rk(tasks.size());
        HIP_CHECK(hipMemcpyAsync(rk.data(), dr.p, sizeof(int) * rk.size(), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        int64_t total = 0;
        for (size_t t = 0; t < tasks.size(); ++t) {
            if (rk[t] > 0) total += (int64_t)rk[t] * (tasks[t].m + tasks[t].n);
            // entries evaluated: one row and one column per rank step (zero rows aside)
            const int64_t ev = (int64_t)std::max(rk[t], tasks[t].kcap * (rk[t] < 0)) * (tasks[t].m + tasks[t].n);
            B.evaluated += ev;
            B.aca_entries += ev;
        }
        DevBuf out(sizeof(T) * (size_t)total);
        std::vector<CompactTask> ct;
        int64_t off = 0;
        for (size_t t = 0; t < tasks.size(); ++t) {
            const size_t b = ids[t];
            if (rk[t] < 0) {
                fallback.push_back(P.lowrank[b]);
                continue;
            }
            const int64_t nu = (int64_t)rk[t] * tasks[t].m, nv = (int64_t)rk[t] * tasks[t].n;
            T *du = out.as<T>() + off, *dv = du + nu;
            ct.push_back({Us.as<T>() + tasks[t].uoff, Vs.as<T>() + tasks[t].voff, du, dv, nu, nv});
            B.rank[b] = rk[t];
            B.U[b] = du;
            B.V[b] = dv;
            B.lr_entries += nu + nv;
            off += nu + nv;
        }
        if (!ct.empty()) {
            DevBuf dct = upload(ct, s);
            k_compact<T><<<(unsigned)ct.size(), 256, 0, s>>>(dct.as<CompactTask>());
            HIP_LAUNCH_CHECK();
            HIP_CHECK(hipStreamSynchronize(s));
        }
        B.bytes += (int64_t)out.bytes;
        B.bufs.push_back(std::move(out));
    }
    fill_dense_blocks<T>(H, B, kap, fallback, s);
}

template <typename T>
void assemble_typed(HMat &H, int band, const T *kap, hipStream_t s) {
    BandStore &B = H.bands[band];
    fill_dense_blocks<T>(H, B, kap, H.plan->dense, s);
    run_aca<T>(H, B, kap, s);
}

}  // namespace

void assemble_band(HMat &H, int band, const double *kappa_band, hipStream_t s) {
    if (H.precision == RTE_FP64) {
        assemble_typed<double>(H, band, kappa_band, s);
    } else {
        DevBuf kf(sizeof(float) * (size_t)H.mesh->N);
        to_float(kappa_band, kf.as<float>(), H.mesh->N, s);
        assemble_typed<float>(H, band, kf.as<float>(), s);
        HIP_CHECK(hipStreamSynchronize(s));
    }
}

}  // namespace rte
