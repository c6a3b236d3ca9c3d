// H-matrix times vector(s): y = H x for nrhs right-hand sides (Section
// "Compression": after compression the fixed point only needs matrix-vector
// products, O(N ln N) each).
//
// Storage: every block row-major with rows padded to a multiple of 4.
// Phase A: t_b = V_b^T x[s-range of b] for every low-rank block b.  A
//          wavefront takes a chunk of source rows of V [n][kp]; a lane owns 4
//          consecutive coefficients l..l+3 (one vector load per row) and the
//          wavefront covers 64/LQ rows per step, so no per-l reduction is
//          needed.  Blocks larger than one chunk write partial sums that a
//          second pass adds in a fixed order.
// Phase B: one workgroup per (band, target leaf) owns its rows: it sums the
//          dense blocks of its block row and the leaf slices of every
//          low-rank block that covers it, y = y0 + sum_seg D x or U t.  Each
//          of the W wavefronts takes every W-th segment.  A segment slice is
//          column-major [K][rp]; 16 lanes read 4 consecutive rows each of one
//          column (contiguous) and the 4 lane groups take columns l, l+1,
//          l+2, l+3, so lane use depends on the leaf size, not on the rank.
//          Partial sums are added over the lane groups by a butterfly and over
//          the W wavefronts in a fixed order.  No atomics: results are
//          bitwise reproducible.
// BF16 storage runs both phases on the matrix cores
// (v_mfma_f32_16x16x32_bf16, 16 right-hand sides per instruction): the
// vectors are first staged as BF16 splits x = hi + mid (+ lo) in the stored
// source coordinates, phase A multiplies 16-rank tiles of V^T by them, a
// fixed-order pass adds the chunk partials and splits t the same way, and
// phase B multiplies 16-row tiles of the K-grouped slices by 32-column steps
// of x or t.  The low operator (inner sweeps, applied to the change of the
// source between defect steps) takes hi factors times hi + mid with FP32
// accumulation; the accurate operator takes hi + lo factors times
// hi + mid + lo and adds every 32-column step's FP32 result into FP64.
// FP64 storage with more than 4 right-hand sides runs both phases on the
// FP64 matrix cores (v_mfma_f64_16x16x4_f64) over the same work lists, 16
// right-hand sides per pass, so the operator is streamed once per 16 instead
// of once per 4: a 16-rank (phase A) or 16-row (phase B) tile times 4 sources
// or columns times 16 right-hand sides per instruction, with 4 tiles per
// wavefront sharing the right-hand-side operand.
#include <algorithm>
#include <map>
#include <tuple>
#include <type_traits>

#include "kernels.h"

namespace rte {

struct VtTask {
    const void *V;      // first row of the chunk in V [n][kp]
    const void *Vlo;    // same position in the BF16 lo part (mixed precision)
    int64_t s0;         // source (cluster order) of the chunk's first row
    int64_t out;        // offset of the result (t buffer, or partial buffer if partial)
    int32_t nj, k;      // rows in the chunk, rank (row length kp = pad4(k))
    int32_t partial, band;
};

struct VtReduce {
    int64_t part;       // first partial (elements) in the partial buffer
    int64_t toff;       // offset of t_b
    int32_t chunks, k;
};

struct Seg {
    const void *data;   // leaf slice, column-major [K][ld]: dense block columns or U of a low-rank block
    const void *lo;     // BF16 lo part (mixed precision)
    int64_t coef_off;   // offset into x (dense: s0) or t (low rank: toff)
    int32_t ld, pad, K, is_lr;   // ld = pad4(leaf rows); K columns (dense: n, low rank: rank)
};

struct LeafWork {
    int64_t r0;         // first row (cluster order)
    int32_t rows, seg0, seg1, band;
};

// BF16 (matrix-core) phase A task: up to kMfTiles 16-rank tiles over one chunk
// of stored source rows.  The tiles may come from different low-rank blocks
// whose V covers the same chunk (blocks of one source cluster are chunked
// alike), so the x operand loaded for a step serves all of them.  The low
// operator takes up to 8 tiles per task (its x operand, 64 bytes per source
// row, then costs a quarter of the 256 bytes of V); the accurate operator,
// with twice the operand registers per tile, takes up to 4, from a task list
// of its own.
constexpr int kMfTiles = 8;
struct MfTile {
    const uint16_t *V, *Vlo;   // first 8-row group of the chunk in the block's V [nP/8][k][8]
    int64_t out;               // direct: offset of t_b in the t splits; else partial-sum offset of the chunk
    int32_t k, kt0;            // block rank, first rank of the tile
    int32_t direct, pad;       // direct: the block is one chunk, its t splits are written here
};
struct MfVt {
    MfTile tile[kMfTiles];
    int64_t xoff;              // stored source coordinate of the chunk's first row
    int32_t ng, band, nt, pad; // 8-row groups in the chunk, band, tiles used
};

// BF16 t staging: sum a block's chunk partials, split into hi, mid, lo
struct MfRed {
    int64_t part, toff;        // first partial; offset of t (a multiple of 8, pad8(k) entries)
    int32_t chunks, k;
};

struct MatvecPlan {
    DevBuf vt, seg, leaf, red;
    DevBuf vt4;                // matrix cores with 8-tile tasks: the accurate operator's list (at most 4)
    int64_t n_vt4 = 0;
    int tiles = 4;             // matrix cores: most tiles in a task of `vt`
    int64_t n_vt = 0, n_leaf = 0, ktot = 0, n_red = 0, n_red_threads = 0, npart = 0;
    int64_t n_src = 0, n_tgt = 0;
    int max_rows = 0;
    // matrix-core path (BF16 storage)
    bool mf = false;
    int nb = 1;                // bands in this plan
    int64_t np = 0;            // stored source coordinates per vector
    const int64_t *pmap_p = nullptr;   // H.src_pmap: stored coordinate -> source or -1
};

namespace {

// factor storage of the vector-ALU path: FP64 or FP32
enum : int { ST_F64 = 0, ST_F32 = 1 };

// 4 consecutive elements starting at element i (i a multiple of 4, rows aligned)
template <int ST, int MODE, typename A>
__device__ __forceinline__ void load4(const void *p, const void *, int64_t i, A v[4]) {
    if constexpr (ST == ST_F64) {
        const double2 *q = reinterpret_cast<const double2 *>(static_cast<const double *>(p) + i);
        const double2 a = q[0], b = q[1];
        v[0] = (A)a.x; v[1] = (A)a.y; v[2] = (A)b.x; v[3] = (A)b.y;
    } else {
        const float4 a = *reinterpret_cast<const float4 *>(static_cast<const float *>(p) + i);
        v[0] = (A)a.x; v[1] = (A)a.y; v[2] = (A)a.z; v[3] = (A)a.w;
    }
}

template <int ST, int MODE, typename A, int NR>
__global__ __launch_bounds__(256) void k_phase_a(const VtTask *__restrict__ tasks, int64_t ntask,
                                                 const double *__restrict__ x, int64_t ldx, int64_t xbs,
                                                 double *__restrict__ t, int64_t ldt, double *__restrict__ part,
                                                 int64_t ldp, int r0, int nr) {
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= ntask) return;
    const VtTask tk = tasks[w];
    double *dst = tk.partial ? part : t;
    const int64_t ldd = tk.partial ? ldp : ldt;
    const int kp = (int)pad4(tk.k);
    x += (int64_t)tk.band * xbs;
    for (int l0 = 0; l0 < kp; l0 += 64) {
        const int quads = min(64, kp - l0) / 4;   // vector loads per row in this slice
        int LQ = 1;
        while (LQ < quads) LQ <<= 1;
        const int G = 64 / LQ;                     // rows per step
        const int g = lane / LQ, q = lane - g * LQ;
        const bool live = q < quads;
        const int l = l0 + 4 * q;
        A acc[NR][4];
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[r][u] = (A)0;
        int jj = g;
        for (; jj + G < tk.nj; jj += 2 * G) {
            A v0[4] = {(A)0, (A)0, (A)0, (A)0}, v1[4] = {(A)0, (A)0, (A)0, (A)0};
            if (live) {
                load4<ST, MODE, A>(tk.V, tk.Vlo, (int64_t)jj * kp + l, v0);
                load4<ST, MODE, A>(tk.V, tk.Vlo, (int64_t)(jj + G) * kp + l, v1);
            }
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                if (r < nr) {
                    const double *xr = x + (int64_t)(r0 + r) * ldx + tk.s0 + jj;
                    const A x0 = (A)xr[0], x1 = (A)xr[G];
#pragma unroll
                    for (int u = 0; u < 4; ++u) acc[r][u] += v0[u] * x0 + v1[u] * x1;
                }
            }
        }
        if (jj < tk.nj) {
            A v0[4] = {(A)0, (A)0, (A)0, (A)0};
            if (live) load4<ST, MODE, A>(tk.V, tk.Vlo, (int64_t)jj * kp + l, v0);
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                if (r < nr) {
                    const A x0 = (A)x[(int64_t)(r0 + r) * ldx + tk.s0 + jj];
#pragma unroll
                    for (int u = 0; u < 4; ++u) acc[r][u] += v0[u] * x0;
                }
            }
        }
        // add the G row groups (lanes q, q + LQ, ...) in a fixed order
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (r < nr) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    A a = acc[r][u];
                    for (int o = LQ; o < 64; o <<= 1) a += __shfl_xor(a, o, 64);
                    if (g == 0 && live && l + u < tk.k) dst[(int64_t)(r0 + r) * ldd + tk.out + l + u] = (double)a;
                }
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_phase_a_reduce(const VtReduce *__restrict__ red, int64_t nred,
                                                        const double *__restrict__ part, int64_t ldp,
                                                        double *__restrict__ t, int64_t ldt, int r0, int nr) {
    const int64_t item = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (item >= nred) return;
    const VtReduce rd = red[item];
    for (int w = threadIdx.x & 63; w < rd.k; w += 64)
        for (int r = 0; r < nr; ++r) {
            double s = 0.0;
#pragma unroll 8
            for (int c = 0; c < rd.chunks; ++c) s += part[(int64_t)(r0 + r) * ldp + rd.part + (int64_t)c * rd.k + w];
            t[(int64_t)(r0 + r) * ldt + rd.toff + w] = s;
        }
}

// a lane reads RPL = 4 consecutive rows of one column per load (16 or 32
// bytes); 16 lanes cover a 64-row tile and 4 column groups run side by side
template <int ST, int MODE, typename A, int RPL>
__device__ __forceinline__ void load_rows(const void *p, const void *lo, int64_t i, A v[RPL]) {
    static_assert(RPL == 4, "4 rows per lane");
    load4<ST, MODE, A>(p, lo, i, v);
}

template <int ST> constexpr int rows_per_lane() { return 4; }

template <int ST, int MODE, typename A, int NR, int W>
__global__ __launch_bounds__(64 * W) void k_phase_b(const LeafWork *__restrict__ leaves, const Seg *__restrict__ segs,
                                                    const double *__restrict__ x, int64_t ldx, int64_t xbs,
                                                    const double *__restrict__ t, int64_t ldt,
                                                    const double *__restrict__ y0, double *__restrict__ y,
                                                    int64_t ldy, int64_t ybs, int r0, int nr) {
    constexpr int RPL = rows_per_lane<ST>();
    constexpr int LPC = 64 / RPL;   // lanes per column (a 64-row tile)
    constexpr int CG = RPL;         // column groups
    __shared__ A part[W][NR][64];
    const LeafWork lw = leaves[blockIdx.x];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int rq = lane % LPC, cg = lane / LPC;
    x += (int64_t)lw.band * xbs;
    y += (int64_t)lw.band * ybs;
    if (y0) y0 += (int64_t)lw.band * ybs;
    for (int rb = 0; rb < lw.rows; rb += 64) {
        const bool rlive = rb + RPL * rq < lw.rows;
        const int64_t cb = rb + RPL * rq;   // first row of this lane within a column
        A acc[RPL][NR];
#pragma unroll
        for (int u = 0; u < RPL; ++u)
#pragma unroll
            for (int r = 0; r < NR; ++r) acc[u][r] = (A)0;
        int s = lw.seg0 + wid;
        Seg sg;
        if (s < lw.seg1) sg = segs[s];
        for (; s < lw.seg1; s += W) {
            // the next descriptor is fetched while this segment streams
            const Seg cur = sg;
            if (s + W < lw.seg1) sg = segs[s + W];
            const double *cf = (cur.is_lr ? t : x) + cur.coef_off;
            const int64_t ldc = cur.is_lr ? ldt : ldx;
            int l = cg;
            for (; l + CG < cur.K; l += 2 * CG) {
                A d0[RPL], d1[RPL];
#pragma unroll
                for (int u = 0; u < RPL; ++u) d0[u] = d1[u] = (A)0;
                if (rlive) {
                    load_rows<ST, MODE, A, RPL>(cur.data, cur.lo, (int64_t)l * cur.ld + cb, d0);
                    load_rows<ST, MODE, A, RPL>(cur.data, cur.lo, (int64_t)(l + CG) * cur.ld + cb, d1);
                }
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    if (r < nr) {
                        const A c0 = (A)cf[(int64_t)(r0 + r) * ldc + l], c1 = (A)cf[(int64_t)(r0 + r) * ldc + l + CG];
#pragma unroll
                        for (int u = 0; u < RPL; ++u) acc[u][r] += d0[u] * c0 + d1[u] * c1;
                    }
                }
            }
            if (l < cur.K) {
                A d0[RPL];
#pragma unroll
                for (int u = 0; u < RPL; ++u) d0[u] = (A)0;
                if (rlive) load_rows<ST, MODE, A, RPL>(cur.data, cur.lo, (int64_t)l * cur.ld + cb, d0);
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    if (r < nr) {
                        const A c0 = (A)cf[(int64_t)(r0 + r) * ldc + l];
#pragma unroll
                        for (int u = 0; u < RPL; ++u) acc[u][r] += d0[u] * c0;
                    }
                }
            }
        }
        // sum over the column groups (same order on every lane)
#pragma unroll
        for (int u = 0; u < RPL; ++u)
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                A a = acc[u][r];
#pragma unroll
                for (int o = LPC; o < 64; o <<= 1) a += __shfl_xor(a, o, 64);
                acc[u][r] = a;
            }
        if (cg == 0) {
#pragma unroll
            for (int u = 0; u < RPL; ++u)
#pragma unroll
                for (int r = 0; r < NR; ++r) part[wid][r][RPL * rq + u] = acc[u][r];
        }
        __syncthreads();
        const int row = rb + lane;
        if (wid == 0 && row < lw.rows) {
            const int64_t gr = lw.r0 + row;
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                if (r < nr) {
                    double v = y0 ? y0[(int64_t)(r0 + r) * ldy + gr] : 0.0;
                    A sum = part[0][r][lane];
#pragma unroll
                    for (int w = 1; w < W; ++w) sum += part[w][r][lane];
                    y[(int64_t)(r0 + r) * ldy + gr] = v + (double)sum;
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- FP64 matrix cores, 16 right-hand sides
typedef double f64x4 __attribute__((ext_vector_type(4)));

// D += A B with A 16 x 4 (lane l holds A[l % 16][l / 16]), B 4 x 16 (lane l
// holds B[l / 16][l % 16]); lane l's component v of D is D[4 v + l / 16][l % 16]
__device__ __forceinline__ f64x4 mfma64(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Phase A: one wavefront per task (a chunk of V [nj][kp] rows), ranks in
// slices of 64 = 4 tiles of 16.  A lane loads 2 consecutive ranks of a row in
// one 16-byte load: the even one feeds tile 0 (2) and the odd one tile 1
// (3), so tile tl holds the ranks L0 + 32 (tl / 2) + 2 i + tl % 2, i < 16.  A
// rank past k but inside the row's padding to 4 reads the padding's zero.
// Per step of 4 sources a lane also loads one x value (right-hand side
// l % 16, source l / 16).
__global__ __launch_bounds__(256) void k_phase_a_mf64(const VtTask *__restrict__ tasks, int64_t ntask,
                                                      const double *__restrict__ x, int64_t ldx, int64_t xbs,
                                                      double *__restrict__ t, int64_t ldt, double *__restrict__ part,
                                                      int64_t ldp, int r0, int nr) {
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= ntask) return;
    const int lane = threadIdx.x & 63, col = lane & 15, sub = lane >> 4;
    const VtTask tk = tasks[w];
    double *dst = tk.partial ? part : t;
    const int64_t ldd = tk.partial ? ldp : ldt;
    const int kp = (int)pad4(tk.k);
    const double *V = static_cast<const double *>(tk.V);
    const bool xl = col < nr;
    const double *xr = x + (int64_t)tk.band * xbs + (int64_t)(r0 + (xl ? col : 0)) * ldx + tk.s0;
    for (int L0 = 0; L0 < tk.k; L0 += 64) {
        const bool h0 = L0 + 2 * col < tk.k, h1 = L0 + 32 + 2 * col < tk.k;
        const bool two = L0 + 32 < tk.k;   // uniform: the second pair of tiles has ranks
        f64x4 acc[4];
#pragma unroll
        for (int tl = 0; tl < 4; ++tl) acc[tl] = f64x4{0.0, 0.0, 0.0, 0.0};
        for (int jj = 0; jj < tk.nj; jj += 4) {
            const int j = jj + sub;
            const bool jl = j < tk.nj;
            const double b = xl && jl ? xr[j] : 0.0;
            const double2 *vr = reinterpret_cast<const double2 *>(V + (int64_t)j * kp + L0) + col;
            const double2 z{0.0, 0.0};
            const double2 a0 = jl && h0 ? vr[0] : z;
            acc[0] = mfma64(a0.x, b, acc[0]);
            acc[1] = mfma64(a0.y, b, acc[1]);
            if (two) {
                const double2 a1 = jl && h1 ? vr[16] : z;
                acc[2] = mfma64(a1.x, b, acc[2]);
                acc[3] = mfma64(a1.y, b, acc[3]);
            }
        }
        if (xl) {
#pragma unroll
            for (int tl = 0; tl < 4; ++tl)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int l = L0 + 32 * (tl >> 1) + 2 * (4 * v + sub) + (tl & 1);
                    if (l < tk.k) dst[(int64_t)(r0 + col) * ldd + tk.out + l] = acc[tl][v];
                }
        }
    }
}

// Phase B: W wavefronts per (band, target leaf), every W-th segment each;
// rows in passes of 64 = 4 tiles of 16, columns in steps of 4.  As in phase
// A a lane loads 2 consecutive rows in one 16-byte load, so tile tl holds the
// rows rb + 32 (tl / 2) + 2 i + tl % 2 (a row past the leaf inside the slice's
// padding to 4 reads zero).  The W partial results are added in a fixed
// order.
template <int W>
__global__ __launch_bounds__(64 * W) void k_phase_b_mf64(const LeafWork *__restrict__ leaves,
                                                         const Seg *__restrict__ segs, const double *__restrict__ x,
                                                         int64_t ldx, int64_t xbs, const double *__restrict__ t,
                                                         int64_t ldt, const double *__restrict__ y0,
                                                         double *__restrict__ y, int64_t ldy, int64_t ybs, int r0,
                                                         int nr) {
    __shared__ double red[W][4][4][64];
    const LeafWork lw = leaves[blockIdx.x];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, col = lane & 15, sub = lane >> 4;
    const bool xl = col < nr;
    const int rc = r0 + (xl ? col : 0);   // right-hand side of this lane's coefficient loads
    x += (int64_t)lw.band * xbs;
    y += (int64_t)lw.band * ybs;
    if (y0) y0 += (int64_t)lw.band * ybs;
    for (int rb = 0; rb < lw.rows; rb += 64) {
        const bool h0 = rb + 2 * col < lw.rows, h1 = rb + 32 + 2 * col < lw.rows;
        const bool two = rb + 32 < lw.rows;
        f64x4 acc[4];
#pragma unroll
        for (int tl = 0; tl < 4; ++tl) acc[tl] = f64x4{0.0, 0.0, 0.0, 0.0};
        int s = lw.seg0 + wid;
        Seg nxt;
        if (s < lw.seg1) nxt = segs[s];
        for (; s < lw.seg1; s += W) {
            // the next descriptor is fetched while this segment streams
            const Seg cur = nxt;
            if (s + W < lw.seg1) nxt = segs[s + W];
            const double *cr = (cur.is_lr ? t + (int64_t)rc * ldt : x + (int64_t)rc * ldx) + cur.coef_off;
            const double *D = static_cast<const double *>(cur.data) + rb;
            for (int c0 = 0; c0 < cur.K; c0 += 4) {
                const int c = c0 + sub;
                const bool cl = c < cur.K;
                const double b = xl && cl ? cr[c] : 0.0;
                const double2 *dc = reinterpret_cast<const double2 *>(D + (int64_t)c * cur.ld) + col;
                const double2 z{0.0, 0.0};
                const double2 a0 = cl && h0 ? dc[0] : z;
                acc[0] = mfma64(a0.x, b, acc[0]);
                acc[1] = mfma64(a0.y, b, acc[1]);
                if (two) {
                    const double2 a1 = cl && h1 ? dc[16] : z;
                    acc[2] = mfma64(a1.x, b, acc[2]);
                    acc[3] = mfma64(a1.y, b, acc[3]);
                }
            }
        }
#pragma unroll
        for (int tl = 0; tl < 4; ++tl)
#pragma unroll
            for (int v = 0; v < 4; ++v) red[wid][tl][v][lane] = acc[tl][v];
        __syncthreads();
        if (wid == 0 && xl) {
#pragma unroll
            for (int tl = 0; tl < 4; ++tl)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = rb + 32 * (tl >> 1) + 2 * (4 * v + sub) + (tl & 1);
                    if (row < lw.rows) {
                        double sum = red[0][tl][v][lane];
#pragma unroll
                        for (int q = 1; q < W; ++q) sum += red[q][tl][v][lane];
                        const int64_t at = (int64_t)(r0 + col) * ldy + lw.r0 + row;
                        y[at] = (y0 ? y0[at] : 0.0) + sum;
                    }
                }
        }
        __syncthreads();
    }
}

// Partial sums of the chunked blocks of phase A, 16 right-hand sides: a
// workgroup per block, a thread per (right-hand side, rank), the chunks added
// in order.
__global__ __launch_bounds__(256) void k_phase_a_reduce16(const VtReduce *__restrict__ red,
                                                          const double *__restrict__ part, int64_t ldp,
                                                          double *__restrict__ t, int64_t ldt, int r0, int nr) {
    const VtReduce rd = red[blockIdx.x];
    const int n = nr * rd.k;
    for (int e = threadIdx.x; e < n; e += 256) {
        const int r = e / rd.k, w = e - r * rd.k;
        const double *p = part + (int64_t)(r0 + r) * ldp + rd.part + w;
        double s = 0.0;
#pragma unroll 8
        for (int c = 0; c < rd.chunks; ++c) s += p[(int64_t)c * rd.k];
        t[(int64_t)(r0 + r) * ldt + rd.toff + w] = s;
    }
}

// ---------------------------------------------------------------- matrix-core path (BF16 storage)
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Operands are read with buffer loads relative to a per-segment (per-task)
// resource: an offset at or beyond the resource's size returns zeros, so
// masked lanes and ragged tails need no branch and every step issues the
// same loads (which lets the compiler keep the next step's loads in flight).
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr int kOOB = 0x7FFFFFF0;   // beyond every resource
__device__ __forceinline__ rsrc_t make_rsrc(const void *p, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, bytes, 0x00020000);
}
__device__ __forceinline__ bf16x8 bload(rsrc_t r, int off) {
    return __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

// v = hi + mid + lo with each part a BF16 (hi + mid carries 16 significant
// bits, all three 24)
__device__ __forceinline__ void split3(double v, uint16_t &h, uint16_t &m, uint16_t &l) {
    h = f2bf((float)v);
    const double r1 = v - (double)bf2f(h);
    m = f2bf((float)r1);
    const double r2 = r1 - (double)bf2f(m);
    l = f2bf((float)r2);
}

// Staged operands of one group of up to 16 right-hand sides: for a
// coefficient group G (8 consecutive stored coordinates or ranks) the 16
// right-hand sides follow each other, 8 BF16 each: element (G, r, e) at
// (G * 16 + r) * 8 + e, so the 16 lanes of a step read 256 contiguous bytes.
// x: [3 splits][band][np / 8][16][8]; t: [3 splits][ktot / 8][16][8].
// Right-hand sides beyond the group's count are zeros.
__global__ void k_mf_xstage(const int64_t *__restrict__ pmap, int64_t np, int nb, int nrhs, int r0, int nr,
                            const double *__restrict__ x, int64_t n_src, uint16_t *__restrict__ xs, int64_t xsplit) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (band, G, r, e)
    if (k >= (int64_t)nb * np * 16) return;
    const int e = (int)(k & 7), r = (int)((k >> 3) & 15);
    const int64_t bg = k >> 7, band = bg / (np / 8), G = bg - band * (np / 8);
    const int64_t p = G * 8 + e;
    const int64_t j = pmap[p];
    uint16_t h = 0, m = 0, l = 0;
    if (j >= 0 && r < nr) split3(x[(band * nrhs + r0 + r) * n_src + j], h, m, l);
    xs[k] = h;
    xs[xsplit + k] = m;
    xs[2 * xsplit + k] = l;
}

template <int MODE, int NT = 4>
struct MfOps {
    // operand splits used: the accurate operator carries the vector in three
    // BF16 parts (24 significant bits), the low operator in two (16 bits).
    // With the hi part alone the inner sweeps stall at the BF16 rounding of
    // the source change (measured: a mixed solve to 1e-9 no longer converged).
    static constexpr int NS = MODE == kMatvecAccurate ? 3 : 2;
    bf16x8 bx[NS], a[NT], al[MODE == kMatvecAccurate ? NT : 1];
};

template <int MODE, int NT = 4>
__device__ __forceinline__ void mf_products(const MfOps<MODE, NT> &o, int nt, f32x4 acc[NT], double a64[NT][4]) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if (t < nt) {
            if constexpr (MODE == kMatvecLow) {
                acc[t] = mfma(o.a[t], o.bx[0], acc[t]);
                acc[t] = mfma(o.a[t], o.bx[1], acc[t]);
            } else {
                f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
                z = mfma(o.a[t], o.bx[0], z);
                z = mfma(o.a[t], o.bx[1], z);
                z = mfma(o.a[t], o.bx[2], z);
                z = mfma(o.al[t], o.bx[0], z);
                z = mfma(o.al[t], o.bx[1], z);
#pragma unroll
                for (int v = 0; v < 4; ++v) a64[t][v] += (double)z[v];
            }
        }
    }
}

// Resources and geometry of one phase B segment.
template <int MODE>
struct MfSrc {
    rsrc_t a, al, x[3];
    int k;      // slice rows (ld)
    int ngr;    // 8-groups of the K dimension
};

// Resources and geometry of one phase A task: per tile its block's V.
template <int MODE, int NT>
struct MfSrcA {
    rsrc_t a[NT], al[MODE == kMatvecAccurate ? NT : 1], x[3];
    int k[NT], kt0[NT];
    int ngr, nt;
};

// Phase A.  Lane (c = lane % 16, q = lane / 16) feeds rank row c of each
// 16-rank tile and right-hand side c of the x operand, over rows 8q..8q+7 of
// each 32-row step.  Result lane layout: rank 4q + v of the tile, right-hand
// side c.  A wavefront walks tasks w, w + nw, w + 2 nw, ... (the list is
// sorted by size, so the strided walk balances) as one pipeline over
// (task, step), two operand sets in turn: the next step's operands, possibly
// of the next task, are in flight while the current products run.  A tile of
// a one-chunk block writes its t splits (zero padding up to pad8(k)
// included) directly; tiles of larger blocks leave partials (FP32 for the
// low operator, FP64 for the accurate one) for k_mf_tstage.
template <int MODE, int NT>
__device__ __forceinline__ MfSrcA<MODE, NT> mf_src_a(const MfVt &tk, const uint16_t *xs, int64_t xsplit, int64_t np) {
    MfSrcA<MODE, NT> r;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const MfTile &tl = tk.tile[t < tk.nt ? t : 0];
        const int vbytes = tk.ng * tl.k * 16;
        r.a[t] = make_rsrc(tl.V, vbytes);
        if constexpr (MODE == kMatvecAccurate) r.al[t] = make_rsrc(tl.Vlo, vbytes);
        r.k[t] = tl.k;
        r.kt0[t] = tl.kt0;
    }
    const uint16_t *xb = xs + ((int64_t)tk.band * (np / 8) + tk.xoff / 8) * 128;
#pragma unroll
    for (int sp = 0; sp < MfOps<MODE>::NS; ++sp) r.x[sp] = make_rsrc(xb + sp * xsplit, tk.ng * 256);
    r.ngr = tk.ng;
    r.nt = tk.nt;
    return r;
}

template <int MODE, int NT>
__device__ __forceinline__ void mf_load_a(const MfSrcA<MODE, NT> &r, int g0, bool valid, int c, int q,
                                          MfOps<MODE, NT> &o) {
    const int g = g0 + q;
    const int xo = valid ? (g * 16 + c) * 16 : kOOB;
#pragma unroll
    for (int sp = 0; sp < MfOps<MODE, NT>::NS; ++sp) o.bx[sp] = bload(r.x[sp], xo);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int rk = r.kt0[t] + c;
        const int off = valid && t < r.nt && rk < r.k[t] ? (g * r.k[t] + rk) * 16 : kOOB;
        o.a[t] = bload(r.a[t], off);
        if constexpr (MODE == kMatvecAccurate) o.al[t] = bload(r.al[t], off);
    }
}

template <int MODE, int NT>
__device__ __forceinline__ void mf_finish_a(const MfVt &tk, int c, int q, const f32x4 acc[NT], const double a64[NT][4],
                                            double *part, int64_t ldp, uint16_t *ts, int64_t tsplit, int r0, int nr) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if (t < tk.nt) {
            const MfTile &tl = tk.tile[t];
            if (tl.direct) {   // uniform: the tile's block is one chunk, its t splits are written here
                // lane (c, q) holds ranks kt0 + 4q .. + 3 of right-hand side c: split them
                // and pack each split's 4 values in two words; the lane with even q
                // takes its partner's (q + 1, the next 4 ranks of the same 8-group)
                // and writes the 8-group of right-hand side c as one 16-byte store
                uint32_t w[3][2];
#pragma unroll
                for (int v = 0; v < 4; v += 2) {
                    uint16_t h0, m0, l0, h1, m1, l1;
                    const int rk = tl.kt0 + 4 * q + v;
                    const double v0 = rk < tl.k ? (MODE == kMatvecLow ? (double)acc[t][v] : a64[t][v]) : 0.0;
                    const double v1 = rk + 1 < tl.k ? (MODE == kMatvecLow ? (double)acc[t][v + 1] : a64[t][v + 1]) : 0.0;
                    split3(v0, h0, m0, l0);
                    split3(v1, h1, m1, l1);
                    w[0][v / 2] = (uint32_t)h0 | ((uint32_t)h1 << 16);
                    w[1][v / 2] = (uint32_t)m0 | ((uint32_t)m1 << 16);
                    w[2][v / 2] = (uint32_t)l0 | ((uint32_t)l1 << 16);
                }
                // the splits phase B reads: hi + mid for the low operator, all three for the accurate
                constexpr int NSW = MfOps<MODE, NT>::NS;
                uint32_t p[3][2];
#pragma unroll
                for (int sp = 0; sp < NSW; ++sp)
#pragma unroll
                    for (int e = 0; e < 2; ++e) p[sp][e] = (uint32_t)__shfl_xor((int)w[sp][e], 16, 64);
                const int rk0 = tl.kt0 + 4 * q;   // a multiple of 8 when q is even
                if ((q & 1) == 0 && rk0 < (int)pad8(tl.k)) {
                    const int64_t off = ((tl.out + rk0) / 8 * 16 + c) * 8;
#pragma unroll
                    for (int sp = 0; sp < NSW; ++sp)
                        *reinterpret_cast<uint4 *>(ts + sp * tsplit + off) = make_uint4(w[sp][0], w[sp][1], p[sp][0], p[sp][1]);
                }
            } else if (c < nr) {
                // chunk partials: FP32 for the low operator (its sums are FP32), FP64 for the accurate one
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int rk = tl.kt0 + 4 * q + v;
                    const int64_t o = (int64_t)(r0 + c) * ldp + tl.out + rk;
                    if (rk < tl.k) {
                        if constexpr (MODE == kMatvecLow) reinterpret_cast<float *>(part)[o] = acc[t][v];
                        else part[o] = a64[t][v];
                    }
                }
            }
        }
    }
}

// Workgroups are dealt to the 8 XCDs in turn (workgroup b runs on XCD b % 8).
// Renumber them so that each XCD takes runs of R consecutive virtual
// workgroups, the runs dealt to the XCDs in turn: neighbouring work (tasks of
// one source chunk, target leaves with common sources) shares an XCD's L2,
// and every XCD still gets work from the whole list (measured on the 49^3
// 32-band operator, with the packed t stores of mf_finish_a: low-operator
// matvec 19.8 -> 18.3 ms, accurate 35.5 -> 33.4).
template <int R>
__device__ __forceinline__ int64_t xcd_runs(int64_t b, int64_t G) {
    const int64_t Gm = G / (8 * R) * (8 * R);   // whole rounds of runs; the tail keeps its order
    if (b >= Gm) return b;
    const int64_t x = b % 8, q = b / 8;
    return ((q / R) * 8 + x) * R + q % R;
}

template <int MODE, int NT>
__global__ __launch_bounds__(256) void k_mf_phase_a(const MfVt *__restrict__ tasks, int64_t ntask, int64_t nw,
                                                    const uint16_t *__restrict__ xs, int64_t xsplit, int64_t np,
                                                    double *__restrict__ part, int64_t ldp, uint16_t *__restrict__ ts,
                                                    int64_t tsplit, int r0, int nr) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int64_t ti = xcd_runs<8>(blockIdx.x, gridDim.x) * 4 + wave;
    if (ti >= ntask) return;
    const int lane = threadIdx.x & 63, c = lane & 15, q = lane >> 4;
    f32x4 acc[NT];
    double a64[NT][4];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) { acc[t][v] = 0.0f; a64[t][v] = 0.0; }
    // pipeline state: the task of the operands being consumed, and the next
    int64_t cur = ti;     // task being consumed
    MfSrcA<MODE, NT> rl = mf_src_a<MODE, NT>(tasks[ti], xs, xsplit, np);
    int g0 = 0, ngc = rl.ngr, ntc = rl.nt;
    MfOps<MODE, NT> o0, o1;   // two operand sets in turn (named: an indexed pair would live in scratch)
    mf_load_a<MODE, NT>(rl, 0, true, c, q, o0);
    int64_t tl = ti;      // task of the last issued load
    int gl = 0;
    bool done = false;
    // issue the loads of the step after (tl, gl) into `nx`, then the products of
    // `cu`; the loads run one step ahead, so when a task's last step is consumed
    // the next task is the one the loads have just moved to
    auto step = [&](const MfOps<MODE, NT> &cu, MfOps<MODE, NT> &nx) {
        int gn = gl + 4;
        int64_t tn = tl;
        if (gn >= rl.ngr) {
            tn = tl + nw;
            gn = 0;
            if (tn < ntask) rl = mf_src_a<MODE, NT>(tasks[tn], xs, xsplit, np);
        }
        // past the end: the same loads at out-of-range offsets (zeros)
        mf_load_a<MODE, NT>(rl, gn, tn < ntask, c, q, nx);
        mf_products<MODE, NT>(cu, ntc, acc, a64);
        g0 += 4;
        if (g0 >= ngc) {
            mf_finish_a<MODE, NT>(tasks[cur], c, q, acc, a64, part, ldp, ts, tsplit, r0, nr);
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) { acc[t][v] = 0.0f; a64[t][v] = 0.0; }
            cur += nw;
            g0 = 0;
            if (cur < ntask) {
                // the loads have just moved to task cur
                ngc = rl.ngr;
                ntc = rl.nt;
            } else {
                done = true;
            }
        }
        tl = tn;
        gl = gn;
    };
    while (true) {
        step(o0, o1);
        if (done) break;
        step(o1, o0);
        if (done) break;
    }
}

// t_b = sum of the chunk partials (fixed order, in FP64), split into hi, mid, lo, for
// the blocks of more than one chunk: one workgroup per block, a thread per
// (right-hand side, rank) pair; entries k..pad8(k)-1 and right-hand sides
// beyond the group's count are zeros
template <int MODE>
__global__ __launch_bounds__(256) void k_mf_tstage(const MfRed *__restrict__ red, const double *__restrict__ part,
                                                   int64_t ldp, uint16_t *__restrict__ ts, int64_t tsplit, int r0,
                                                   int nr) {
    const MfRed rd = red[blockIdx.x];
    const int k8 = (int)pad8(rd.k);
    for (int e = threadIdx.x; e < 16 * k8; e += blockDim.x) {
        const int r = e / k8, l = e - r * k8;
        double sum = 0.0;
        if (l < rd.k && r < nr) {
            const int64_t o0 = (int64_t)(r0 + r) * ldp + rd.part + l;
            if constexpr (MODE == kMatvecLow) {   // FP32 partials, added in FP64 as before
                const float *p = reinterpret_cast<const float *>(part) + o0;
                for (int c = 0; c < rd.chunks; ++c) sum += (double)p[(int64_t)c * rd.k];
            } else {
                const double *p = part + o0;
                for (int c = 0; c < rd.chunks; ++c) sum += p[(int64_t)c * rd.k];
            }
        }
        uint16_t h, m, lo;
        split3(sum, h, m, lo);
        const int64_t o = ((rd.toff + l) / 8 * 16 + r) * 8 + l % 8;
        ts[o] = h;
        ts[tsplit + o] = m;
        if constexpr (MODE == kMatvecAccurate) ts[2 * tsplit + o] = lo;   // the low operator reads hi + mid
    }
}

// Phase B: one workgroup per (band, target leaf), W wavefronts over its
// segments.  Lane (c, q) feeds row c of each 16-row tile and right-hand side
// c of the coefficient operand, over columns 8q..8q+7 of each 32-column step.
// Result lane layout: row 4q + v of the tile, right-hand side c; the W
// wavefront sums are added in a fixed order through LDS.  Each wavefront runs
// one pipeline over (segment, step), two operand sets in turn.
template <int MODE>
__device__ __forceinline__ MfSrc<MODE> mf_src_b(const Seg &sg, const uint16_t *xb, int64_t xsplit, const uint16_t *tb,
                                                int64_t tsplit) {
    MfSrc<MODE> r;
    const int kg = (sg.K + 7) / 8;
    const int abytes = kg * sg.ld * 16;
    r.a = make_rsrc(sg.data, abytes);
    if constexpr (MODE == kMatvecAccurate) r.al = make_rsrc(sg.lo, abytes);
    const uint16_t *src = (sg.is_lr ? tb : xb) + sg.coef_off / 8 * 128;
    const int64_t sst = sg.is_lr ? tsplit : xsplit;
#pragma unroll
    for (int sp = 0; sp < MfOps<MODE>::NS; ++sp) r.x[sp] = make_rsrc(src + sp * sst, kg * 256);
    r.k = sg.ld;
    r.ngr = kg;
    return r;
}

template <int MODE>
__device__ __forceinline__ void mf_load_b(const MfSrc<MODE> &r, int g0, bool valid, int c, int q, int rb, int rows,
                                          MfOps<MODE> &o) {
    const int g = g0 + q;
    const int xo = valid ? (g * 16 + c) * 16 : kOOB;
#pragma unroll
    for (int sp = 0; sp < MfOps<MODE>::NS; ++sp) o.bx[sp] = bload(r.x[sp], xo);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int row = rb + 16 * t + c;
        const int off = valid && row < rows ? (g * r.k + row) * 16 : kOOB;
        o.a[t] = bload(r.a, off);
        if constexpr (MODE == kMatvecAccurate) o.al[t] = bload(r.al, off);
    }
}

template <int MODE, int W>
__global__ __launch_bounds__(64 * W) void k_mf_phase_b(const LeafWork *__restrict__ leaves,
                                                       const Seg *__restrict__ segs, const uint16_t *__restrict__ xs,
                                                       int64_t xsplit, int64_t np, const uint16_t *__restrict__ ts,
                                                       int64_t tsplit, const double *__restrict__ y0,
                                                       double *__restrict__ y, int64_t ldy, int64_t ybs, int r0,
                                                       int nr) {
    using PT = typename std::conditional<MODE == kMatvecAccurate, double, float>::type;
    __shared__ PT part[W][64][17];
    const LeafWork lw = leaves[xcd_runs<16>(blockIdx.x, gridDim.x)];
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, c = lane & 15, q = lane >> 4;
    const uint16_t *xb = xs + (int64_t)lw.band * (np / 8) * 128;
    y += (int64_t)lw.band * ybs;
    if (y0) y0 += (int64_t)lw.band * ybs;
    for (int rb = 0; rb < lw.rows; rb += 64) {
        const int nrt = min(4, (lw.rows - rb + 15) / 16);
        f32x4 acc[4];
        double a64[4][4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) { acc[t][v] = 0.0f; a64[t][v] = 0.0; }
        int si = lw.seg0 + wid;
        if (si < lw.seg1) {
            Seg sl = segs[si];                       // segment of the last issued load
            MfSrc<MODE> rl = mf_src_b<MODE>(sl, xb, xsplit, ts, tsplit);
            int gl = 0, g0 = 0, sc = si;              // (sc, g0): step being consumed
            int kgc = rl.ngr;
            MfOps<MODE> o0, o1;   // two operand sets in turn (named: an indexed pair would live in scratch)
            mf_load_b<MODE>(rl, 0, true, c, q, rb, lw.rows, o0);
            int sl_i = si;
            bool done = false;
            auto step = [&](const MfOps<MODE> &cu, MfOps<MODE> &nx) {
                int gn = gl + 4, sn = sl_i;
                if (gn >= rl.ngr) {
                    sn = sl_i + W;
                    gn = 0;
                    if (sn < lw.seg1) {
                        sl = segs[sn];
                        rl = mf_src_b<MODE>(sl, xb, xsplit, ts, tsplit);
                    }
                }
                mf_load_b<MODE>(rl, gn, sn < lw.seg1, c, q, rb, lw.rows, nx);
                mf_products<MODE>(cu, nrt, acc, a64);
                g0 += 4;
                if (g0 >= kgc) {
                    sc += W;
                    g0 = 0;
                    if (sc < lw.seg1) kgc = rl.ngr;   // the loads have just moved to segment sc
                    else done = true;
                }
                sl_i = sn;
                gl = gn;
            };
            while (true) {
                step(o0, o1);
                if (done) break;
                step(o1, o0);
                if (done) break;
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                part[wid][16 * t + 4 * q + v][c] = MODE == kMatvecLow ? (PT)acc[t][v] : (PT)a64[t][v];
        __syncthreads();
        for (int idx = threadIdx.x; idx < 16 * 64; idx += 64 * W) {
            const int r = idx >> 6, row = idx & 63;
            if (r < nr && rb + row < lw.rows) {
                PT sum = part[0][row][r];
#pragma unroll
                for (int w = 1; w < W; ++w) sum += part[w][row][r];
                const int64_t gr = lw.r0 + rb + row;
                const double v0 = y0 ? y0[(int64_t)(r0 + r) * ldy + gr] : 0.0;
                y[(int64_t)(r0 + r) * ldy + gr] = v0 + (double)sum;
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

// phase B of the vector-ALU path with W wavefronts per workgroup
template <int ST, int MODE, typename A, int NR>
void phase_b_valu(int W, unsigned gb, const LeafWork *lw, const Seg *sg, const double *x, int64_t ldx, int64_t xbs,
                  const double *t, int64_t ldt, const double *y0, double *y, int64_t ldy, int64_t ybs, int r0, int nr,
                  hipStream_t s) {
    if (W == 2)
        k_phase_b<ST, MODE, A, NR, 2><<<gb, 128, 0, s>>>(lw, sg, x, ldx, xbs, t, ldt, y0, y, ldy, ybs, r0, nr);
    else if (W == 4)
        k_phase_b<ST, MODE, A, NR, 4><<<gb, 256, 0, s>>>(lw, sg, x, ldx, xbs, t, ldt, y0, y, ldy, ybs, r0, nr);
    else
        k_phase_b<ST, MODE, A, NR, 8><<<gb, 512, 0, s>>>(lw, sg, x, ldx, xbs, t, ldt, y0, y, ldy, ybs, r0, nr);
}

// wb: wavefronts per phase B workgroup.  FP64 with more than 4 right-hand
// sides: the matrix-core kernels, 16 per pass.  Otherwise groups of at most 4
// on the vector ALUs: with 16 per launch the accumulators (4 rows x 16
// columns per lane) leave one wavefront per SIMD and the stream stalls.
template <int ST, int MODE, typename A>
void launch_typed(const MatvecPlan &mp, int nrhs, const double *x, const double *y0, double *y, double *tb,
                  hipStream_t s, int wb) {
    double *part = tb + mp.ktot * (int64_t)nrhs;   // the workspace holds t, then the partials
    const int64_t ldp = std::max<int64_t>(mp.npart, 1);
    const int64_t xbs = (int64_t)nrhs * mp.n_src, ybs = (int64_t)nrhs * mp.n_tgt;
    if constexpr (ST == ST_F64) {
        if (nrhs > 4) {   // 16 right-hand sides per pass on the matrix cores
            for (int r0 = 0; r0 < nrhs; r0 += 16) {
                const int nr = std::min(16, nrhs - r0);
                if (mp.n_vt) {
                    k_phase_a_mf64<<<(unsigned)((mp.n_vt + 3) / 4), 256, 0, s>>>(
                        mp.vt.as<VtTask>(), mp.n_vt, x, mp.n_src, xbs, tb, mp.ktot, part, ldp, r0, nr);
                    HIP_LAUNCH_CHECK();
                    if (mp.n_red) {
                        k_phase_a_reduce16<<<(unsigned)mp.n_red, 256, 0, s>>>(mp.red.as<VtReduce>(), part, ldp, tb,
                                                                             mp.ktot, r0, nr);
                        HIP_LAUNCH_CHECK();
                    }
                }
                const unsigned gb = (unsigned)mp.n_leaf;
                const LeafWork *lw = mp.leaf.as<LeafWork>();
                const Seg *sg = mp.seg.as<Seg>();
                if (wb == 2)
                    k_phase_b_mf64<2><<<gb, 128, 0, s>>>(lw, sg, x, mp.n_src, xbs, tb, mp.ktot, y0, y, mp.n_tgt, ybs,
                                                         r0, nr);
                else if (wb == 4)
                    k_phase_b_mf64<4><<<gb, 256, 0, s>>>(lw, sg, x, mp.n_src, xbs, tb, mp.ktot, y0, y, mp.n_tgt, ybs,
                                                         r0, nr);
                else
                    k_phase_b_mf64<8><<<gb, 512, 0, s>>>(lw, sg, x, mp.n_src, xbs, tb, mp.ktot, y0, y, mp.n_tgt, ybs,
                                                         r0, nr);
                HIP_LAUNCH_CHECK();
            }
            return;
        }
    }
    constexpr int kGroup = 4;
    for (int r0 = 0; r0 < nrhs; r0 += kGroup) {
        const int nr = std::min(kGroup, nrhs - r0);
        if (mp.n_vt) {
            const unsigned ga = (unsigned)((mp.n_vt + 3) / 4);
            const VtTask *vt = mp.vt.as<VtTask>();
            if (nr == 1)
                k_phase_a<ST, MODE, A, 1><<<ga, 256, 0, s>>>(vt, mp.n_vt, x, mp.n_src, xbs, tb, mp.ktot, part, ldp, r0, nr);
            else
                k_phase_a<ST, MODE, A, 4><<<ga, 256, 0, s>>>(vt, mp.n_vt, x, mp.n_src, xbs, tb, mp.ktot, part, ldp, r0, nr);
            HIP_LAUNCH_CHECK();
            if (mp.n_red) {
                k_phase_a_reduce<<<(unsigned)((mp.n_red + 3) / 4), 256, 0, s>>>(mp.red.as<VtReduce>(), mp.n_red, part,
                                                                               ldp, tb, mp.ktot, r0, nr);
                HIP_LAUNCH_CHECK();
            }
        }
        const unsigned gb = (unsigned)mp.n_leaf;
        const LeafWork *lw = mp.leaf.as<LeafWork>();
        const Seg *sg = mp.seg.as<Seg>();
        if (nr == 1)
            phase_b_valu<ST, MODE, A, 1>(wb, gb, lw, sg, x, mp.n_src, xbs, tb, mp.ktot, y0, y, mp.n_tgt, ybs, r0, nr, s);
        else
            phase_b_valu<ST, MODE, A, 4>(wb, gb, lw, sg, x, mp.n_src, xbs, tb, mp.ktot, y0, y, mp.n_tgt, ybs, r0, nr, s);
        HIP_LAUNCH_CHECK();
    }
}

// Workgroups of `kernel` (block threads, no dynamic LDS) that are resident at
// once on the current device: a persistent launch uses exactly these.
template <typename K>
int64_t resident_workgroups(K kernel, int block) {
    int dev = 0, cus = 0, per_cu = 0;
    HIP_CHECK(hipGetDevice(&dev));
    HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0));
    return std::max<int64_t>(1, (int64_t)cus * std::max(per_cu, 1));
}

// BF16 storage on the matrix cores.  Workspace: phase A partials [nrhs][npart]
// FP64, then the staged operands of one group of 16 right-hand sides, x
// [3][nb][np / 8][16][8] and t [3][ktot / 8][16][8] BF16.
template <int MODE>
void launch_mf(const MatvecPlan &mp, int nrhs, const double *x, const double *y0, double *y, double *tb,
               hipStream_t s, int wb) {
    const int64_t ldp = std::max<int64_t>(mp.npart, 1);
    double *part = tb;
    uint16_t *xs = reinterpret_cast<uint16_t *>(tb + ((ldp * nrhs + 1) & ~(int64_t)1));   // 16-byte aligned
    const int64_t xsplit = (int64_t)mp.nb * mp.np * 16;
    uint16_t *ts = xs + 3 * xsplit;
    const int64_t tsplit = mp.ktot * 16;
    const int64_t ybs = (int64_t)nrhs * mp.n_tgt;
    for (int r0 = 0; r0 < nrhs; r0 += 16) {
        const int nr = std::min(16, nrhs - r0);
        k_mf_xstage<<<(unsigned)((xsplit + 255) / 256), 256, 0, s>>>(mp.pmap_p, mp.np, mp.nb, nrhs, r0, nr, x,
                                                                     mp.n_src, xs, xsplit);
        HIP_LAUNCH_CHECK();
        if (mp.n_vt) {
            // the resident wavefronts, each walking a strided task list
            auto phase_a = [&](auto kernel, const MfVt *tasks, int64_t ntask) {
                static const int64_t resident = resident_workgroups(kernel, 256);
                const int64_t nwg = std::min<int64_t>((ntask + 3) / 4, resident);
                kernel<<<(unsigned)nwg, 256, 0, s>>>(tasks, ntask, nwg * 4, xs, xsplit, mp.np, part, ldp, ts, tsplit,
                                                     r0, nr);
            };
            bool eight = false;
            if constexpr (MODE == kMatvecLow) {
                if (mp.tiles == 8) {
                    phase_a(k_mf_phase_a<MODE, 8>, mp.vt.as<MfVt>(), mp.n_vt);
                    eight = true;
                }
            }
            if (!eight) {
                if (mp.n_vt4) phase_a(k_mf_phase_a<MODE, 4>, mp.vt4.as<MfVt>(), mp.n_vt4);
                else phase_a(k_mf_phase_a<MODE, 4>, mp.vt.as<MfVt>(), mp.n_vt);
            }
            HIP_LAUNCH_CHECK();
            if (mp.n_red) {
                k_mf_tstage<MODE><<<(unsigned)mp.n_red, 256, 0, s>>>(mp.red.as<MfRed>(), part, ldp, ts, tsplit, r0,
                                                                     nr);
                HIP_LAUNCH_CHECK();
            }
        }
        const unsigned gb = (unsigned)mp.n_leaf;
        const LeafWork *lw = mp.leaf.as<LeafWork>();
        const Seg *sg = mp.seg.as<Seg>();
        if (wb == 2)
            k_mf_phase_b<MODE, 2><<<gb, 128, 0, s>>>(lw, sg, xs, xsplit, mp.np, ts, tsplit, y0, y, mp.n_tgt, ybs, r0, nr);
        else if (wb == 8)
            k_mf_phase_b<MODE, 8><<<gb, 512, 0, s>>>(lw, sg, xs, xsplit, mp.np, ts, tsplit, y0, y, mp.n_tgt, ybs, r0, nr);
        else
            k_mf_phase_b<MODE, 4><<<gb, 256, 0, s>>>(lw, sg, xs, xsplit, mp.np, ts, tsplit, y0, y, mp.n_tgt, ybs, r0, nr);
        HIP_LAUNCH_CHECK();
    }
}

// workspace doubles of a call with nrhs right-hand sides
int64_t ws_words(const MatvecPlan &mp, int nrhs) {
    if (!mp.mf) return (mp.ktot + mp.npart) * nrhs;
    const int64_t bf16 = 3 * 16 * ((int64_t)mp.nb * mp.np + mp.ktot);
    return std::max<int64_t>(mp.npart, 1) * nrhs + 2 + (2 * bf16 + 7) / 8;
}

}  // namespace

HMat::HMat() = default;
HMat::~HMat() = default;

namespace {

// Work lists of y = H x for the bands in `bands`, all in one launch per phase:
// band b's vectors sit at x + b' * nrhs * N_src (b' its position in the list),
// and its t coefficients follow those of the previous bands.
std::unique_ptr<MatvecPlan> build_plan(const HMat &H, const std::vector<int> &bands, hipStream_t s) {
    const Plan &P = *H.plan;
    auto mp = std::make_unique<MatvecPlan>();
    mp->n_src = (int64_t)P.src_nat.size();
    mp->n_tgt = (int64_t)P.tgt_nat.size();
    std::vector<VtTask> vt;
    std::vector<VtReduce> red;
    int64_t ktot = 0, npart = 0, maxk = 0;
    // about this many bytes of V per wavefront task
    const int64_t chunk_bytes = (int64_t)H.cfg.task_kib * 1024;
    const int tiles = H.cfg.tiles;
    const int64_t esz = H.precision == RTE_FP64 ? 8 : H.precision == RTE_FP32 ? 4 : 2;
    const auto &leaves = P.tgt_leaves;
    auto leaf_of = [&](int64_t row) { return (int64_t)P.leaf_of(row); };
    std::vector<Seg> segs;
    std::vector<LeafWork> lw;
    const bool mf = H.precision == RTE_MIXED_BF16;
    std::vector<MfVt> mvt;
    std::vector<MfRed> mred;
    // matrix-core phase A: tiles grouped by (band, first stored row, rows) of their chunk
    std::map<std::tuple<int, int64_t, int64_t>, std::vector<MfTile>> mtiles;
    const int64_t mf_rows = std::min<int64_t>(8192, std::max<int64_t>(256, chunk_bytes / 128)) / 8 * 8;
    const int64_t g = H.kgroup;
    for (int bi = 0; bi < (int)bands.size(); ++bi) {
        const BandStore &B = H.bands[bands[bi]];
        std::vector<int64_t> toff(P.lowrank.size(), -1);
        for (size_t b = 0; b < P.lowrank.size() && mf; ++b) {
            if (B.rank[b] <= 0) continue;
            const Block &bl = P.lowrank[b];
            const int32_t k = B.rank[b];
            const int64_t wp = H.pwidth(bl.s0, bl.s1);
            toff[b] = ktot;
            // chunks of mf_rows stored rows from the source cluster's start:
            // blocks of one source cluster are chunked alike and their tiles
            // can share a task
            const int64_t chunks = (wp + mf_rows - 1) / mf_rows;
            const uint16_t *V = static_cast<const uint16_t *>(B.V[b]), *Vl = static_cast<const uint16_t *>(B.Vlo[b]);
            if (chunks > 1) mred.push_back({npart, ktot, (int32_t)chunks, k});
            for (int64_t c = 0; c < chunks; ++c) {
                const int64_t nj = std::min(mf_rows, wp - c * mf_rows);
                auto &grp = mtiles[std::make_tuple(bi, H.src_p_h[bl.s0] + c * mf_rows, nj)];
                for (int32_t kt0 = 0; kt0 < k; kt0 += 16)
                    grp.push_back({V + c * mf_rows * k, Vl + c * mf_rows * k, chunks == 1 ? ktot : npart + c * k, k,
                                   kt0, chunks == 1 ? 1 : 0, 0});
            }
            if (chunks > 1) npart += chunks * k;
            maxk = std::max<int64_t>(maxk, k);
            ktot += pad8(k);
        }
        for (size_t b = 0; b < P.lowrank.size() && !mf; ++b) {
            if (B.rank[b] <= 0) continue;
            const Block &bl = P.lowrank[b];
            const int32_t k = B.rank[b];
            const int64_t n = bl.s1 - bl.s0;
            toff[b] = ktot;
            const int64_t rows = std::max<int64_t>(64, chunk_bytes / (pad4(k) * esz));
            const int64_t chunks = (n + rows - 1) / rows;
            const char *V = static_cast<const char *>(B.V[b]);
            const char *Vl = static_cast<const char *>(B.Vlo.empty() ? nullptr : B.Vlo[b]);
            if (chunks == 1) {
                vt.push_back({V, Vl, bl.s0, ktot, (int32_t)n, k, 0, bi});
            } else {
                red.push_back({npart, ktot, (int32_t)chunks, k});
                for (int64_t c = 0; c < chunks; ++c) {
                    const int64_t j0 = c * rows, nj = std::min(rows, n - j0);
                    vt.push_back({V + j0 * pad4(k) * esz, Vl ? Vl + j0 * pad4(k) * esz : nullptr, bl.s0 + j0,
                                  npart + c * k, (int32_t)nj, k, 1, bi});
                }
                npart += chunks * k;
            }
            maxk = std::max<int64_t>(maxk, k);
            ktot += k;
        }
        // one segment per (block, target leaf slice); slice li of a block with K
        // columns starts K * (prp[li] - prp[li0]) elements after the block.
        // Laid out per target leaf (dense blocks, then low-rank ones, each in
        // block order): a counting pass, then a filling pass.
        const int64_t nleaf = (int64_t)leaves.size();
        auto for_slices = [&](const Block &bl, auto &&fn) {
            const int64_t li0 = leaf_of(bl.t0);
            for (int64_t li = li0; li < nleaf && leaves[li].first < bl.t1; ++li) fn(li0, li);
        };
        std::vector<int64_t> pos(nleaf + 1, 0);
        auto count = [&](int64_t, int64_t li) { ++pos[li + 1]; };
        for (const Block &bl : B.dense_blocks) for_slices(bl, count);
        for (size_t b = 0; b < P.lowrank.size(); ++b)
            if (B.rank[b] > 0) for_slices(P.lowrank[b], count);
        const int64_t base = (int64_t)segs.size();
        for (int64_t li = 0; li < nleaf; ++li) pos[li + 1] += pos[li];
        segs.resize((size_t)(base + pos[nleaf]));
        std::vector<int64_t> cur(pos.begin(), pos.end() - 1);
        auto put = [&](const Block &bl, const void *hi, const void *lo, int64_t K, int64_t coef, int is_lr) {
            const int64_t Kp = (K + g - 1) / g * g;
            for_slices(bl, [&](int64_t li0, int64_t li) {
                const int64_t off = Kp * (H.leaf_prp_h[li] - H.leaf_prp_h[li0]) * esz;
                const int32_t rp = (int32_t)(H.leaf_prp_h[li + 1] - H.leaf_prp_h[li]);
                segs[(size_t)(base + cur[li]++)] = {static_cast<const char *>(hi) + off,
                                                    lo ? static_cast<const char *>(lo) + off : nullptr, coef, rp, 0,
                                                    (int32_t)K, is_lr};
            });
        };
        for (size_t d = 0; d < B.dense_blocks.size(); ++d) {
            const Block &bl = B.dense_blocks[d];
            put(bl, B.dense_ptr[d], B.dense_lo[d], H.pwidth(bl.s0, bl.s1), H.src_p_h[bl.s0], 0);
        }
        for (size_t b = 0; b < P.lowrank.size(); ++b) {
            if (B.rank[b] <= 0) continue;
            put(P.lowrank[b], B.U[b], B.Ulo.empty() ? nullptr : B.Ulo[b], B.rank[b], toff[b], 1);
        }
        for (int64_t li = 0; li < nleaf; ++li) {
            LeafWork w{};
            w.r0 = leaves[li].first;
            w.rows = (int32_t)(leaves[li].second - leaves[li].first);
            w.seg0 = (int32_t)(base + pos[li]);
            w.seg1 = (int32_t)(base + pos[li + 1]);
            w.band = bi;
            lw.push_back(w);
            mp->max_rows = std::max(mp->max_rows, w.rows);
        }
    }
    // large tasks first so that long wavefronts start early (a stable order:
    // (size, position) keys sorted, then the tasks gathered once)
    {
        std::vector<std::pair<int64_t, uint32_t>> key(vt.size());
        for (size_t i = 0; i < vt.size(); ++i) key[i] = {-(int64_t)vt[i].nj * vt[i].k, (uint32_t)i};
        std::sort(key.begin(), key.end());
        std::vector<VtTask> sorted(vt.size());
        for (size_t i = 0; i < key.size(); ++i) sorted[i] = vt[key[i].second];
        vt.swap(sorted);
    }
    // tasks of up to `per` tiles of one chunk (in block order), large first
    auto group_tasks = [&](int per) {
        std::vector<MfVt> out;
        for (auto &kv : mtiles) {
            const std::vector<MfTile> &grp = kv.second;
            for (size_t i = 0; i < grp.size(); i += (size_t)per) {
                MfVt t{};
                t.nt = (int32_t)std::min<size_t>((size_t)per, grp.size() - i);
                for (int j = 0; j < t.nt; ++j) t.tile[j] = grp[i + j];
                t.xoff = std::get<1>(kv.first);
                t.ng = (int32_t)(std::get<2>(kv.first) / 8);
                t.band = std::get<0>(kv.first);
                out.push_back(t);
            }
        }
        std::stable_sort(out.begin(), out.end(), [](const MfVt &a, const MfVt &b) {
            return (int64_t)a.ng * a.nt > (int64_t)b.ng * b.nt;
        });
        return out;
    };
    std::vector<MfVt> mvt4;
    if (mf) {
        mvt = group_tasks(tiles);
        if (tiles > 4) mvt4 = group_tasks(4);   // the accurate operator's list
    }
    mp->ktot = std::max<int64_t>(ktot, mf ? 8 : 1);
    mp->npart = npart;
    mp->n_red_threads = maxk;
    mp->n_leaf = (int64_t)lw.size();
    mp->mf = mf;
    mp->nb = (int)bands.size();
    mp->np = H.n_src_p;
    mp->pmap_p = H.src_pmap.as<int64_t>();
    if (mf) {
        mp->n_vt = (int64_t)mvt.size();
        mp->n_red = (int64_t)mred.size();
        mp->vt = upload(mvt, s);
        mp->red = upload(mred, s);
        mp->tiles = tiles;
        if (!mvt4.empty()) {
            mp->n_vt4 = (int64_t)mvt4.size();
            mp->vt4 = upload(mvt4, s);
        }
    } else {
        mp->n_vt = (int64_t)vt.size();
        mp->n_red = (int64_t)red.size();
        mp->vt = upload(vt, s);
        mp->red = upload(red, s);
    }
    mp->seg = upload(segs, s);
    mp->leaf = upload(lw, s);
    HIP_CHECK(hipStreamSynchronize(s));
    return mp;
}

void launch_plan(const HMat &H, const MatvecPlan &mp, int nrhs, const double *x_c, double *y_c, const double *y0_c,
                 double *tbuf, hipStream_t s, int mode) {
    const int wb = H.cfg.waves_b;
    if (H.precision == RTE_FP64) launch_typed<ST_F64, 0, double>(mp, nrhs, x_c, y0_c, y_c, tbuf, s, wb);
    else if (H.precision == RTE_FP32) launch_typed<ST_F32, 0, float>(mp, nrhs, x_c, y0_c, y_c, tbuf, s, wb);
    else if (mode == kMatvecAccurate) launch_mf<kMatvecAccurate>(mp, nrhs, x_c, y0_c, y_c, tbuf, s, wb);
    else launch_mf<kMatvecLow>(mp, nrhs, x_c, y0_c, y_c, tbuf, s, wb);
}

}  // namespace

void matvec_reserve(HMat &H, int n_bands) {
    if ((int)H.mv.size() < n_bands) H.mv.resize(n_bands);
}

void matvec_build(HMat &H, int band, hipStream_t s) {
    if ((int)H.mv.size() <= band) H.mv.resize(band + 1);
    H.mv[band] = build_plan(H, {band}, s);
}

void matvec_build_all(HMat &H, hipStream_t s) {
    if (H.n_bands == 1) return;   // the band-0 plan serves
    std::vector<int> all(H.n_bands);
    for (int b = 0; b < H.n_bands; ++b) all[b] = b;
    H.mv_all = build_plan(H, all, s);
}

int64_t matvec_ws_all(const HMat &H, int nrhs) { return ws_words(H.mv_all ? *H.mv_all : *H.mv[0], nrhs); }

void matvec_launch_all(const HMat &H, int nrhs, const double *x_c, double *y_c, const double *y0_c, double *tbuf,
                       hipStream_t s, int mode) {
    launch_plan(H, H.mv_all ? *H.mv_all : *H.mv[0], nrhs, x_c, y_c, y0_c, tbuf, s, mode);
}

void matvec_configure(HMat &H, const MatvecConfig &cfg, hipStream_t s) {
    const bool mf = H.precision == RTE_MIXED_BF16;
    RTE_REQUIRE(cfg.waves_b == 2 || cfg.waves_b == 4 || cfg.waves_b == 8, "matvec config: waves must be 2, 4 or 8");
    RTE_REQUIRE(mf || cfg.waves_b >= 4, "matvec config: the vector-ALU path takes 4 or 8 waves");
    RTE_REQUIRE(cfg.task_kib >= 4 && cfg.task_kib <= 4096, "matvec config: task size out of range");
    RTE_REQUIRE(cfg.tiles == 1 || cfg.tiles == 2 || cfg.tiles == 4 || cfg.tiles == 8,
                "matvec config: tiles must be 1, 2, 4 or 8");
    H.cfg = cfg;
    for (int b = 0; b < H.n_bands; ++b) matvec_build(H, b, s);
    matvec_build_all(H, s);
}

namespace {
__global__ void k_fill(double *p, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
}  // namespace

double matvec_time(const HMat &H, int nrhs, int mode, int reps, hipStream_t s) {
    const int64_t nx = (int64_t)H.n_bands * nrhs * H.stats.n_src, ny = (int64_t)H.n_bands * nrhs * H.stats.n_tgt;
    DevBuf x(sizeof(double) * nx), y(sizeof(double) * ny), ws(sizeof(double) * (size_t)matvec_ws_all(H, nrhs));
    poison(ws, s);
    k_fill<<<(unsigned)((nx + 255) / 256), 256, 0, s>>>(x.as<double>(), nx, 1.0);
    HIP_LAUNCH_CHECK();
    matvec_launch_all(H, nrhs, x.as<double>(), y.as<double>(), nullptr, ws.as<double>(), s, mode);   // warm-up
    EventTimer tm(s);
    tm.start();
    for (int r = 0; r < reps; ++r)
        matvec_launch_all(H, nrhs, x.as<double>(), y.as<double>(), nullptr, ws.as<double>(), s, mode);
    tm.stop();
    const double ms = tm.ms() / std::max(reps, 1);
    HIP_CHECK(hipStreamSynchronize(s));
    return ms;
}

MatvecConfig matvec_autotune(HMat &H, int nrhs, int mode, int reps, hipStream_t s, double *best_ms, int *trials) {
    const bool mf = H.precision == RTE_MIXED_BF16;
    const std::vector<int> waves = mf ? std::vector<int>{2, 4, 8} : std::vector<int>{4, 8};
    const std::vector<int> kib = {16, 64, 256};
    const std::vector<int> tiles = mf ? std::vector<int>{4, 8} : std::vector<int>{4};
    MatvecConfig best = H.cfg;
    double bt = INFINITY;
    int n = 0;
    for (int w : waves)
        for (int k : kib)
            for (int t : tiles) {
                matvec_configure(H, MatvecConfig{w, k, t}, s);
                const double ms = matvec_time(H, nrhs, mode, reps, s);
                ++n;
                if (ms < bt) { bt = ms; best = H.cfg; }
            }
    matvec_configure(H, best, s);
    if (best_ms) *best_ms = bt;
    if (trials) *trials = n;
    return best;
}

// workspace doubles per right-hand side: t, then the partial sums of chunked blocks
int64_t matvec_ws(const HMat &H, int band, int nrhs) { return ws_words(*H.mv[band], nrhs); }

void matvec_launch_ws(const HMat &H, int band, int nrhs, const double *x_c, double *y_c, const double *y0_c,
                      double *tbuf, hipStream_t s, int mode) {
    launch_plan(H, *H.mv[band], nrhs, x_c, y_c, y0_c, tbuf, s, mode);
}

void matvec_launch(const HMat &H, int band, int nrhs, const double *x_c, double *y_c, const double *y0_c,
                   hipStream_t s, int mode) {
    DevBuf tb(sizeof(double) * (size_t)matvec_ws(H, band, nrhs));
    poison(tb, s);
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
