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

constexpr int kRcMax = 96;   // recompressed ranks: up to 96 (larger blocks, a few in a band, keep their factors)

struct RcTask {
    int64_t uoff, voff;   // U^T [kcap][m] and V^T [kcap][n] in the ACA scratch (elements)
    int64_t woff;         // FP64 workspace of the block: Gu, Gv, Mt, Zt (k x k each)
    int32_t m, n, k, idx; // idx: the block's slot in the rank and order outputs
};

struct RcApply {
    int32_t task, side, i0, i1;   // rows [i0, i1) of U (side 0) or V (side 1)
};

// Launches go by rank bucket, each with the LDS its largest rank needs: the
// factor tiles of k_rc_gram and k_rc_apply take kb x 33 doubles, the core of
// k_rc_core (ranks up to kRcShared) 4 kb^2; small ranks then keep many
// workgroups per CU.
constexpr int kRcShared = 64;
constexpr int kRcBuckets[] = {16, 32, 48, 64, 96};
constexpr int kRcStaticLds = 6144;   // k_rc_core's fixed LDS (per-rank vectors, flags), rounded up

// Step 1: one workgroup per (block, factor).  The factor's rows are staged
// 32 columns at a time in LDS (FP64); a thread accumulates a 4 x 4 tile of
// the lower triangle of the Gram matrix, passes of 256 tiles cover it.
template <typename T>
__global__ __launch_bounds__(256) void k_rc_gram(const RcTask *__restrict__ tasks, const T *__restrict__ Us,
                                                 const T *__restrict__ Vs, double *__restrict__ W) {
    extern __shared__ double sx[];   // [4 kt][33]
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
                sx[l * 33 + i] = (l < k && i0 + i < L) ? (double)X[(int64_t)l * L + i0 + i] : 0.0;
            }
            __syncthreads();
            if (p < ntile) {
                for (int i = 0; i < 32; ++i) {
                    double xa[4], xb[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        xa[u] = sx[(4 * a + u) * 33 + i];
                        xb[u] = sx[(4 * b + u) * 33 + i];
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

// Steps 2 to 5 (small matrices): one workgroup per block.  Output: the new
// rank (-1: keep the ACA factors) and the order of B's columns; the
// transforms Ru^-1 B and Rv^-1 Z are written over the columns of the global
// Mt and Zt, where k_rc_apply reads them.  Where the working matrices live:
// SH = kRcAllLds (ranks up to kRcShared): the scaled Grams, their factors, the
// core and Z in LDS; SH = kRcJacobiLds: the core and Z in LDS (the Jacobi
// sweeps), the factors in the global workspace; SH = kRcGlobal: all global.
enum { kRcGlobal = 0, kRcAllLds = 1, kRcJacobiLds = 2 };
template <int SH>
__global__ __launch_bounds__(256) void k_rc_core(const RcTask *__restrict__ tasks, double *__restrict__ W,
                                                 int *__restrict__ ord, int *__restrict__ rnew, double eps) {
    extern __shared__ double smem[];   // the working matrices kept in LDS
    __shared__ double du[kRcMax], dv[kRcMax], sig[kRcMax];
    __shared__ int order[kRcMax];
    __shared__ int fail, rotated, rk;
    const RcTask t = tasks[blockIdx.x];
    const int k = t.k, tid = threadIdx.x;
    const int64_t kk = (int64_t)k * k;
    double *const Gg = W + t.woff;        // global: Gu, Gv, Mt, Zt (row stride k)
    double *const Mg = Gg + 2 * kk;       // Mt[j * k + i] = M(i, j): column j contiguous
    double *const Zg = Gg + 3 * kk;
    // working copies: row strides ldl (factors) and ld (core, Z), odd in LDS so
    // that a column's elements (stride ld doubles) fall in different banks
    const int ldl = SH == kRcAllLds ? (k | 1) : k;
    const int ld = SH != kRcGlobal ? (k | 1) : k;
    const int64_t kl = (int64_t)k * ldl, km = (int64_t)k * ld;
    double *Lu = SH == kRcAllLds ? smem : Gg;
    double *Lv = Lu + kl;
    double *Mt = SH == kRcAllLds ? smem + 2 * kl : (SH == kRcJacobiLds ? smem : Mg);
    double *Zt = SH == kRcGlobal ? Zg : Mt + km;
    if (tid == 0) fail = 0;
    __syncthreads();
    for (int l = tid; l < k; l += 256) {
        du[l] = sqrt(Gg[(int64_t)l * k + l]);
        dv[l] = sqrt(Gg[kk + (int64_t)l * k + l]);
        if (!(du[l] > 0.0) || !(dv[l] > 0.0)) fail = 1;
    }
    __syncthreads();
    if (fail) {
        if (tid == 0) rnew[t.idx] = -1;
        return;
    }
    for (int e = tid; e < k * k; e += 256) {
        const int i = e / k, j = e - i * k;
        Lu[(int64_t)i * ldl + j] = Gg[e] / (du[i] * du[j]);
        Lv[(int64_t)i * ldl + j] = Gg[kk + e] / (dv[i] * dv[j]);
    }
    __syncthreads();
    // Cholesky of both scaled Grams at once (threads 0-127: Lu, 128-255: Lv),
    // lower factor in place, column by column
    {
        const int half = tid >> 7, lt = tid & 127;
        double *G = half ? Lv : Lu;
        for (int j = 0; j < k; ++j) {
            if (lt == 0) {
                double d = G[(int64_t)j * ldl + j];
                for (int p = 0; p < j; ++p) d -= G[(int64_t)j * ldl + p] * G[(int64_t)j * ldl + p];
                if (!(d > 1e-13)) {   // numerically dependent columns
                    fail = 1;
                    d = 1.0;
                }
                G[(int64_t)j * ldl + j] = sqrt(d);
            }
            __syncthreads();
            const double piv = G[(int64_t)j * ldl + j];
            for (int i = j + 1 + lt; i < k; i += 128) {
                double s = G[(int64_t)i * ldl + j];
                for (int p = 0; p < j; ++p) s -= G[(int64_t)i * ldl + p] * G[(int64_t)j * ldl + p];
                G[(int64_t)i * ldl + j] = s / piv;
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
            s += (Lu[(int64_t)p * ldl + i] * du[p]) * (Lv[(int64_t)p * ldl + j] * dv[p]);
        Mt[(int64_t)j * ld + i] = s;
        Zt[(int64_t)j * ld + i] = i == j ? 1.0 : 0.0;
    }
    __syncthreads();
    // one-sided Jacobi: sweeps of the round-robin pairing of the columns (a
    // dummy column when k is odd), 16 lanes per pair (16 pairs at a time),
    // until a sweep rotates nothing.  A pair is rotated when its columns are
    // not orthogonal to 1e-12 of their norms, far below the truncation
    // tolerance; couplings below (1e-12 s)^2, s the largest column norm of M,
    // are left: such columns are far beyond any truncation and would only
    // trade rounding noise with the large ones.
    for (int j = tid; j < k; j += 256) {
        double c2 = 0.0;
        for (int i = 0; i < k; ++i) c2 = fma(Mt[(int64_t)j * ld + i], Mt[(int64_t)j * ld + i], c2);
        sig[j] = c2;
    }
    __syncthreads();
    double s2 = 0.0;
    for (int j = 0; j < k; ++j) s2 = sig[j] > s2 ? sig[j] : s2;
    const double floor2 = 1e-24 * s2;
    const int n = k + (k & 1), grp = tid >> 4, sl = tid & 15;
    for (int sweep = 0; sweep < 30; ++sweep) {
        __syncthreads();
        if (tid == 0) rotated = 0;
        __syncthreads();
        for (int r = 0; r < n - 1; ++r) {
            for (int pi = grp; pi < n / 2; pi += 16) {
                const int qa = pi, qb = n - 1 - pi;
                const int a = qa == 0 ? 0 : (qa - 1 + r) % (n - 1) + 1;
                const int b = qb == 0 ? 0 : (qb - 1 + r) % (n - 1) + 1;
                if (a >= k || b >= k) continue;   // the dummy column (the whole group)
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int i = sl; i < k; i += 16) {
                    const double x = Mt[(int64_t)a * ld + i], y = Mt[(int64_t)b * ld + i];
                    al = fma(x, x, al);
                    be = fma(y, y, be);
                    ga = fma(x, y, ga);
                }
#pragma unroll
                for (int o = 8; o > 0; o >>= 1) {
                    al += __shfl_xor(al, o, 16);
                    be += __shfl_xor(be, o, 16);
                    ga += __shfl_xor(ga, o, 16);
                }
                if (fabs(ga) > 1e-12 * sqrt(al * be) && fabs(ga) > floor2) {
                    const double zeta = (be - al) / (2.0 * ga);
                    const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double c = 1.0 / sqrt(1.0 + tt * tt), s = c * tt;
                    for (int i = sl; i < k; i += 16) {
                        const double x = Mt[(int64_t)a * ld + i], y = Mt[(int64_t)b * ld + i];
                        Mt[(int64_t)a * ld + i] = c * x - s * y;
                        Mt[(int64_t)b * ld + i] = s * x + c * y;
                        const double zx = Zt[(int64_t)a * ld + i], zy = Zt[(int64_t)b * ld + i];
                        Zt[(int64_t)a * ld + i] = c * zx - s * zy;
                        Zt[(int64_t)b * ld + i] = s * zx + c * zy;
                    }
                    if (sl == 0) rotated = 1;
                }
            }
            __syncthreads();
        }
        if (!rotated) break;   // read by every thread after the round's barrier
    }
    __syncthreads();
    // singular values, their decreasing order, the truncation rank
    for (int j = tid; j < k; j += 256) {
        double s = 0.0;
        for (int i = 0; i < k; ++i) s = fma(Mt[(int64_t)j * ld + i], Mt[(int64_t)j * ld + i], s);
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
    // the same column of Zt Rv^-1 Z(:, ord[c]); a thread per (kept column, side),
    // solved in place, then written to the global columns
    for (int q = tid; q < 2 * r; q += 256) {
        const int c = q >> 1, side = q & 1, j = order[c];
        const double *Lf = side ? Lv : Lu;
        const double *d = side ? dv : du;
        double *y = (side ? Zt : Mt) + (int64_t)j * ld;
        double *out = (side ? Zg : Mg) + (int64_t)j * k;
        for (int i = k - 1; i >= 0; --i) {
            double s = y[i];
            for (int p = i + 1; p < k; ++p) s -= Lf[(int64_t)p * ldl + i] * y[p];
            y[i] = s / Lf[(int64_t)i * ldl + i];
        }
        for (int i = 0; i < k; ++i) out[i] = y[i] / d[i];
        if (side == 0) ord[(int64_t)t.idx * kRcMax + c] = j;
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
    extern __shared__ double sx[];   // [k][33]
    const RcApply a = ap[blockIdx.x];
    const RcTask t = tasks[a.task];
    const int r = rnew[t.idx];
    if (r <= 0) return;   // uniform: the block keeps its factors
    T *__restrict__ X = a.side ? Vs + t.voff : Us + t.uoff;
    const int L = a.side ? t.n : t.m, k = t.k, w = a.i1 - a.i0;
    const double *__restrict__ Tm = W + t.woff + (int64_t)(2 + a.side) * k * k;
    for (int e = threadIdx.x; e < k * 32; e += 256) {
        const int l = e >> 5, i = e & 31;
        sx[l * 33 + i] = i < w ? (double)X[(int64_t)l * L + a.i0 + i] : 0.0;
    }
    __syncthreads();
    const int i = threadIdx.x & 31, g = threadIdx.x >> 5;
    if (i >= w) return;
    for (int c = g; c < r; c += 8) {
        const double *__restrict__ col = Tm + (int64_t)ord[(int64_t)t.idx * kRcMax + c] * k;
        double s = 0.0;
        for (int l = 0; l < k; ++l) s = fma(sx[l * 33 + i], col[l], s);
        X[(int64_t)c * L + a.i0 + i] = (T)s;
    }
}

}  // namespace

template <typename T>
void recompress_batch(const std::vector<AcaTask> &tasks, std::vector<int> &rk, T *Us, T *Vs, double eps,
                      BandStore &B, hipStream_t s) {
    // candidates, by rank bucket
    constexpr int NB = sizeof(kRcBuckets) / sizeof(kRcBuckets[0]);
    std::vector<size_t> cand;
    for (int bk = 0; bk < NB; ++bk)
        for (size_t t = 0; t < tasks.size(); ++t) {
            const int k = rk[t], lo = bk ? kRcBuckets[bk - 1] : 1;
            if (k >= 2 && k > lo && k <= kRcBuckets[bk]) cand.push_back(t);
        }
    if (cand.empty()) return;
    EventTimer timer(s);
    timer.start();
    // the LDS a workgroup may ask for (the cores of the larger buckets go global beyond it)
    int dev = 0, lds_max = 0;
    HIP_CHECK(hipGetDevice(&dev));
    HIP_CHECK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    // rounds whose FP64 workspace (4 k^2 per block) stays within 1 GiB
    const int64_t cap_words = (int64_t)1 << 27;
    size_t c0 = 0;
    while (c0 < cand.size()) {
        std::vector<RcTask> rt;
        std::vector<RcApply> ap;
        std::vector<int> bucket_end(NB, 0), apply_end(NB, 0);   // prefix ends per bucket
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
            int bk = 0;
            while (k > kRcBuckets[bk]) ++bk;
            for (int q = bk; q < NB; ++q) {
                bucket_end[q] = (int)rt.size();
                apply_end[q] = (int)ap.size();
            }
        }
        const int nt = (int)rt.size();
        DevBuf dt = upload_scratch(rt, s), dap = upload_scratch(ap, s);
        DevBuf W = DevBuf::scratch(sizeof(double) * (size_t)words);
        DevBuf dord = DevBuf::scratch(sizeof(int) * (size_t)nt * kRcMax), dr = DevBuf::scratch(sizeof(int) * (size_t)nt);
        const RcTask *tp = dt.as<RcTask>();
        const RcApply *app = dap.as<RcApply>();
        int t0 = 0, a0 = 0;
        for (int bk = 0; bk < NB; ++bk) {   // the blocks of a bucket: t0..t1, their products a0..a1
            const int t1 = bucket_end[bk], a1 = apply_end[bk], kb = kRcBuckets[bk];
            if (t1 > t0) {
                const size_t tile = sizeof(double) * (size_t)((kb + 3) / 4 * 4) * 33;
                k_rc_gram<T><<<dim3((unsigned)(t1 - t0), 2), 256, tile, s>>>(tp + t0, Us, Vs, W.as<double>());
                // LDS for the working matrices: all four, or the core and Z only, or none
                const size_t all_lds = sizeof(double) * 4 * kb * (kb | 1), jac_lds = all_lds / 2;
                const size_t room = (size_t)lds_max - kRcStaticLds;
                if (kb <= kRcShared && all_lds <= room)
                    k_rc_core<kRcAllLds><<<(unsigned)(t1 - t0), 256, all_lds, s>>>(
                        tp + t0, W.as<double>(), dord.as<int>(), dr.as<int>(), eps);
                else if (jac_lds <= room)
                    k_rc_core<kRcJacobiLds><<<(unsigned)(t1 - t0), 256, jac_lds, s>>>(
                        tp + t0, W.as<double>(), dord.as<int>(), dr.as<int>(), eps);
                else
                    k_rc_core<kRcGlobal><<<(unsigned)(t1 - t0), 256, 0, s>>>(tp + t0, W.as<double>(), dord.as<int>(),
                                                                             dr.as<int>(), eps);
                k_rc_apply<T><<<(unsigned)(a1 - a0), 256, sizeof(double) * kb * 33, s>>>(
                    app + a0, tp, Us, Vs, W.as<double>(), dord.as<int>(), dr.as<int>());
                HIP_LAUNCH_CHECK();
            }
            t0 = std::max(t0, t1);
            a0 = std::max(a0, a1);
        }
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
