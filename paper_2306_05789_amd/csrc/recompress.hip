// Recompression of the ACA factors of the admissible blocks.
//
// Section "Compression": the partially pivoted ACA approximates the first
// terms of a block's SVD.  Its factors U (m x k) and V (n x k) are not
// orthogonal, and the rank at which its stopping test fires is usually
// longer than what the SVD of U V^T needs for the same relative Frobenius
// tolerance.  The recompression replaces them by the shortest truncation of
// that SVD within eps (eps: the ACA tolerance), so every later matvec streams
// fewer bytes:
//
//   1. Gram matrices Gu = U^T U and Gv = V^T V (k x k, FP64);
//   2. with D the square roots of their diagonals, the Cholesky factors of the
//      scaled Grams D^-1 G D^-1 = L L^T, so that U = Qu Ru with
//      Ru = L_u^T D_u and Qu = U Ru^-1 (the scaling keeps the Cholesky away
//      from the spread of the ACA columns' norms);
//   3. the core M = Ru Rv^T (U V^T = Qu M Qv^T) and its SVD by one-sided
//      Jacobi rotations of M's columns, accumulated in Z: M Z = B with
//      orthogonal columns of norms sigma_j;
//   4. r = the fewest columns of B, by decreasing sigma, whose dropped sigmas
//      have a norm <= eps ||sigma||;
//   5. U' = U Ru^-1 B_r, V' = V Rv^-1 Z_r (triangular solves on the small
//      matrices, then one product per factor, written in place).
//
// A block whose scaled Gram is numerically singular, or that would not get
// shorter, keeps its ACA factors.  The Gram matrices and the core are FP64
// whatever the storage type; every reduction has a fixed order, so results
// are bitwise reproducible.
#include <cmath>

#include "kernels.h"

namespace rte {

namespace {

constexpr int kRcMax = kAcaMaxRank;   // blocks of the first ACA pass (ranks <= 192)

struct RcTask {
    int64_t uoff, voff;   // U^T [kcap][m] and V^T [kcap][n] in the ACA scratch (elements)
    int64_t woff;         // FP64 workspace of the block: Gu, Gv, Mt, Zt (k x k each)
    int32_t m, n, k, idx; // idx: the block's slot in the rank and order outputs
};

struct RcApply {
    int32_t task, side, i0, i1;   // rows [i0, i1) of U (side 0) or V (side 1)
};

// Step 1: one workgroup per (block, factor).  The factor's rows are staged
// 32 columns at a time in LDS (FP64); a thread accumulates a 4 x 4 tile of
// the lower triangle of the Gram matrix, passes of 256 tiles cover it.
template <typename T>
__global__ __launch_bounds__(256) void k_rc_gram(const RcTask *__restrict__ tasks, const T *__restrict__ Us,
                                                 const T *__restrict__ Vs, double *__restrict__ W) {
    __shared__ double sx[kRcMax][33];
    const RcTask t = tasks[blockIdx.x];
    const int side = blockIdx.y;
    const T *__restrict__ X = side ? Vs + t.voff : Us + t.uoff;
    const int L = side ? t.n : t.m, k = t.k;
    double *__restrict__ G = W + t.woff + (int64_t)side * k * k;
    const int kt = (k + 3) / 4, ntile = kt * (kt + 1) / 2;
    for (int p0 = 0; p0 < ntile; p0 += 256) {
        const int p = p0 + (int)threadIdx.x;
        int a = 0, b = 0;
        if (p < ntile) {   // tile (a, b), a >= b, of lower-triangle index p = a (a + 1) / 2 + b
            a = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
            while (a * (a + 1) / 2 > p) --a;
            while ((a + 1) * (a + 2) / 2 <= p) ++a;
            b = p - a * (a + 1) / 2;
        }
        double acc[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
        for (int i0 = 0; i0 < L; i0 += 32) {
            __syncthreads();
            for (int e = threadIdx.x; e < kt * 4 * 32; e += 256) {
                const int l = e >> 5, i = e & 31;
                sx[l][i] = (l < k && i0 + i < L) ? (double)X[(int64_t)l * L + i0 + i] : 0.0;
            }
            __syncthreads();
            if (p < ntile) {
                for (int i = 0; i < 32; ++i) {
                    double xa[4], xb[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        xa[u] = sx[4 * a + u][i];
                        xb[u] = sx[4 * b + u][i];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[u][v] = fma(xa[u], xb[v], acc[u][v]);
                }
            }
        }
        if (p < ntile) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 4 * a + u, c = 4 * b + v;
                    if (r < k && c < k) {
                        G[(int64_t)r * k + c] = acc[u][v];
                        G[(int64_t)c * k + r] = acc[u][v];
                    }
                }
        }
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Steps 2 to 5 (small matrices): one workgroup per block.  Output: the new
// rank (-1: keep the ACA factors) and the order of B's columns; the
// transforms Ru^-1 B and Rv^-1 Z overwrite the columns of Mt and Zt.
__global__ __launch_bounds__(256) void k_rc_core(const RcTask *__restrict__ tasks, double *__restrict__ W,
                                                 int *__restrict__ ord, int *__restrict__ rnew, double eps) {
    __shared__ double du[kRcMax], dv[kRcMax], sig[kRcMax];
    __shared__ int order[kRcMax];
    __shared__ int fail, rotated, rk;
    const RcTask t = tasks[blockIdx.x];
    const int k = t.k, tid = threadIdx.x;
    double *__restrict__ Gu = W + t.woff;
    double *__restrict__ Gv = Gu + (int64_t)k * k;
    double *__restrict__ Mt = Gv + (int64_t)k * k;   // Mt[j * k + i] = M(i, j): column j contiguous
    double *__restrict__ Zt = Mt + (int64_t)k * k;
    if (tid == 0) fail = 0;
    __syncthreads();
    for (int l = tid; l < k; l += 256) {
        du[l] = sqrt(Gu[(int64_t)l * k + l]);
        dv[l] = sqrt(Gv[(int64_t)l * k + l]);
        if (!(du[l] > 0.0) || !(dv[l] > 0.0)) fail = 1;
    }
    __syncthreads();
    if (fail) {
        if (tid == 0) rnew[t.idx] = -1;
        return;
    }
    for (int e = tid; e < k * k; e += 256) {
        const int i = e / k, j = e - i * k;
        Gu[e] /= du[i] * du[j];
        Gv[e] /= dv[i] * dv[j];
    }
    __syncthreads();
    // Cholesky of both scaled Grams at once (threads 0-127: Gu, 128-255: Gv),
    // lower factor in place, column by column
    {
        const int half = tid >> 7, lt = tid & 127;
        double *__restrict__ G = half ? Gv : Gu;
        for (int j = 0; j < k; ++j) {
            if (lt == 0) {
                double d = G[(int64_t)j * k + j];
                for (int p = 0; p < j; ++p) d -= G[(int64_t)j * k + p] * G[(int64_t)j * k + p];
                if (!(d > 1e-13)) {   // numerically dependent columns
                    fail = 1;
                    d = 1.0;
                }
                G[(int64_t)j * k + j] = sqrt(d);
            }
            __syncthreads();
            const double piv = G[(int64_t)j * k + j];
            for (int i = j + 1 + lt; i < k; i += 128) {
                double s = G[(int64_t)i * k + j];
                for (int p = 0; p < j; ++p) s -= G[(int64_t)i * k + p] * G[(int64_t)j * k + p];
                G[(int64_t)i * k + j] = s / piv;
            }
            __syncthreads();
        }
    }
    if (fail) {
        if (tid == 0) rnew[t.idx] = -1;
        return;
    }
    // core M = Ru Rv^T, Ru(i, p) = L_u(p, i) du(p) for p >= i; Z = I
    for (int e = tid; e < k * k; e += 256) {
        const int j = e / k, i = e - j * k;
        double s = 0.0;
        for (int p = i > j ? i : j; p < k; ++p)
            s += (Gu[(int64_t)p * k + i] * du[p]) * (Gv[(int64_t)p * k + j] * dv[p]);
        Mt[e] = s;
        Zt[e] = i == j ? 1.0 : 0.0;
    }
    __syncthreads();
    // one-sided Jacobi: sweeps of the round-robin pairing of the columns (a
    // dummy column when k is odd), a wavefront per pair, until a sweep rotates
    // nothing
    const int n = k + (k & 1), wave = tid >> 6, lane = tid & 63;
    for (int sweep = 0; sweep < 60; ++sweep) {
        if (tid == 0) rotated = 0;
        __syncthreads();
        for (int r = 0; r < n - 1; ++r) {
            for (int pi = wave; pi < n / 2; pi += 4) {
                const int qa = pi, qb = n - 1 - pi;
                const int a = qa == 0 ? 0 : (qa - 1 + r) % (n - 1) + 1;
                const int b = qb == 0 ? 0 : (qb - 1 + r) % (n - 1) + 1;
                if (a >= k || b >= k) continue;   // the dummy column
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int i = lane; i < k; i += 64) {
                    const double x = Mt[(int64_t)a * k + i], y = Mt[(int64_t)b * k + i];
                    al = fma(x, x, al);
                    be = fma(y, y, be);
                    ga = fma(x, y, ga);
                }
                al = wave_sum(al);
                be = wave_sum(be);
                ga = wave_sum(ga);
                if (ga != 0.0 && fabs(ga) > 1e-15 * sqrt(al * be)) {
                    const double zeta = (be - al) / (2.0 * ga);
                    const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double c = 1.0 / sqrt(1.0 + tt * tt), s = c * tt;
                    for (int i = lane; i < k; i += 64) {
                        const double x = Mt[(int64_t)a * k + i], y = Mt[(int64_t)b * k + i];
                        Mt[(int64_t)a * k + i] = c * x - s * y;
                        Mt[(int64_t)b * k + i] = s * x + c * y;
                        const double zx = Zt[(int64_t)a * k + i], zy = Zt[(int64_t)b * k + i];
                        Zt[(int64_t)a * k + i] = c * zx - s * zy;
                        Zt[(int64_t)b * k + i] = s * zx + c * zy;
                    }
                    if (lane == 0) rotated = 1;
                }
            }
            __syncthreads();
        }
        const int any = rotated;
        __syncthreads();
        if (!any) break;
    }
    // singular values, their decreasing order, the truncation rank
    for (int j = tid; j < k; j += 256) {
        double s = 0.0;
        for (int i = 0; i < k; ++i) s = fma(Mt[(int64_t)j * k + i], Mt[(int64_t)j * k + i], s);
        sig[j] = sqrt(s);
    }
    __syncthreads();
    for (int j = tid; j < k; j += 256) {
        int pos = 0;
        for (int i = 0; i < k; ++i) pos += (sig[i] > sig[j] || (sig[i] == sig[j] && i < j)) ? 1 : 0;
        order[pos] = j;
    }
    __syncthreads();
    if (tid == 0) {
        double total = 0.0;
        for (int c = 0; c < k; ++c) total += sig[order[c]] * sig[order[c]];
        int r = k;
        double tail = 0.0;
        for (int c = k - 1; c >= 1; --c) {
            tail += sig[order[c]] * sig[order[c]];
            if (tail <= eps * eps * total) r = c;
            else break;
        }
        rk = r;
    }
    __syncthreads();
    const int r = rk;
    if (r >= k) {
        if (tid == 0) rnew[t.idx] = -1;
        return;
    }
    // transforms: column ord[c] of Mt becomes Ru^-1 B(:, ord[c]) = D_u^-1 L_u^-T b,
    // the same column of Zt Rv^-1 Z(:, ord[c]); one thread per kept column
    for (int c = tid; c < r; c += 256) {
        const int j = order[c];
        for (int side = 0; side < 2; ++side) {
            const double *__restrict__ Lf = side ? Gv : Gu;
            const double *__restrict__ d = side ? dv : du;
            double *__restrict__ y = (side ? Zt : Mt) + (int64_t)j * k;
            for (int i = k - 1; i >= 0; --i) {
                double s = y[i];
                for (int p = i + 1; p < k; ++p) s -= Lf[(int64_t)p * k + i] * y[p];
                y[i] = s / Lf[(int64_t)i * k + i];
            }
            for (int i = 0; i < k; ++i) y[i] /= d[i];
        }
        ord[(int64_t)t.idx * kRcMax + c] = j;
    }
    if (tid == 0) rnew[t.idx] = r;
}

// Step 5, the products: rows [i0, i1) of a factor, all k of its columns
// staged in LDS, times the kept transform columns; written in place (columns
// 0..r-1 of the factor's transposed storage).
template <typename T>
__global__ __launch_bounds__(256) void k_rc_apply(const RcApply *__restrict__ ap, const RcTask *__restrict__ tasks,
                                                  T *__restrict__ Us, T *__restrict__ Vs, const double *__restrict__ W,
                                                  const int *__restrict__ ord, const int *__restrict__ rnew) {
    __shared__ double sx[kRcMax][33];
    const RcApply a = ap[blockIdx.x];
    const RcTask t = tasks[a.task];
    const int r = rnew[t.idx];
    if (r <= 0) return;   // uniform: the block keeps its factors
    T *__restrict__ X = a.side ? Vs + t.voff : Us + t.uoff;
    const int L = a.side ? t.n : t.m, k = t.k, w = a.i1 - a.i0;
    const double *__restrict__ Tm = W + t.woff + (int64_t)(2 + a.side) * k * k;
    for (int e = threadIdx.x; e < k * 32; e += 256) {
        const int l = e >> 5, i = e & 31;
        sx[l][i] = i < w ? (double)X[(int64_t)l * L + a.i0 + i] : 0.0;
    }
    __syncthreads();
    const int i = threadIdx.x & 31, g = threadIdx.x >> 5;
    if (i >= w) return;
    for (int c = g; c < r; c += 8) {
        const double *__restrict__ col = Tm + (int64_t)ord[(int64_t)t.idx * kRcMax + c] * k;
        double s = 0.0;
        for (int l = 0; l < k; ++l) s = fma(sx[l][i], col[l], s);
        X[(int64_t)c * L + a.i0 + i] = (T)s;
    }
}

}  // namespace

template <typename T>
void recompress_batch(const std::vector<AcaTask> &tasks, std::vector<int> &rk, T *Us, T *Vs, double eps,
                      BandStore &B, hipStream_t s) {
    std::vector<size_t> cand;
    for (size_t t = 0; t < tasks.size(); ++t)
        if (rk[t] >= 2 && rk[t] <= kRcMax) cand.push_back(t);
    if (cand.empty()) return;
    EventTimer timer(s);
    timer.start();
    // rounds whose FP64 workspace (4 k^2 per block) stays within 1 GiB
    const int64_t cap_words = (int64_t)1 << 27;
    size_t c0 = 0;
    while (c0 < cand.size()) {
        std::vector<RcTask> rt;
        std::vector<RcApply> ap;
        int64_t words = 0;
        size_t c1 = c0;
        for (; c1 < cand.size(); ++c1) {
            const AcaTask &a = tasks[cand[c1]];
            const int64_t k = rk[cand[c1]];
            if (!rt.empty() && words + 4 * k * k > cap_words) break;
            const int32_t idx = (int32_t)rt.size();
            rt.push_back({a.uoff, a.voff, words, a.m, a.n, (int32_t)k, idx});
            words += 4 * k * k;
            for (int side = 0; side < 2; ++side) {
                const int L = side ? a.n : a.m;
                for (int i0 = 0; i0 < L; i0 += 32) ap.push_back({idx, side, i0, std::min(L, i0 + 32)});
            }
        }
        const int nt = (int)rt.size();
        DevBuf dt = upload_scratch(rt, s), dap = upload_scratch(ap, s);
        DevBuf W = DevBuf::scratch(sizeof(double) * (size_t)words);
        DevBuf dord = DevBuf::scratch(sizeof(int) * (size_t)nt * kRcMax), dr = DevBuf::scratch(sizeof(int) * (size_t)nt);
        k_rc_gram<T><<<dim3((unsigned)nt, 2), 256, 0, s>>>(dt.as<RcTask>(), Us, Vs, W.as<double>());
        HIP_LAUNCH_CHECK();
        k_rc_core<<<(unsigned)nt, 256, 0, s>>>(dt.as<RcTask>(), W.as<double>(), dord.as<int>(), dr.as<int>(), eps);
        HIP_LAUNCH_CHECK();
        k_rc_apply<T><<<(unsigned)ap.size(), 256, 0, s>>>(dap.as<RcApply>(), dt.as<RcTask>(), Us, Vs, W.as<double>(),
                                                          dord.as<int>(), dr.as<int>());
        HIP_LAUNCH_CHECK();
        std::vector<int> rn(nt);
        HIP_CHECK(hipMemcpyAsync(rn.data(), dr.p, sizeof(int) * nt, hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        for (int q = 0; q < nt; ++q) {
            const size_t t = cand[c0 + q];
            const int64_t mn = (int64_t)tasks[t].m + tasks[t].n;
            B.rc_before += rk[t] * mn;
            if (rn[q] > 0) rk[t] = rn[q];
            B.rc_after += rk[t] * mn;
        }
        for (DevBuf *d : {&dt, &dap, &W, &dord, &dr}) B.retire.push_back(std::move(*d));
        c0 = c1;
    }
    timer.stop();
    B.rc_ms += timer.ms();
    B.rc_blocks += (int64_t)cand.size();
}

template void recompress_batch<double>(const std::vector<AcaTask> &, std::vector<int> &, double *, double *, double,
                                       BandStore &, hipStream_t);
template void recompress_batch<float>(const std::vector<AcaTask> &, std::vector<int> &, float *, float *, double,
                                      BandStore &, hipStream_t);

}  // namespace rte
