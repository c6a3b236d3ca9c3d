// Assembly of one band of an H-matrix: dense near-field leaves and partially
// pivoted ACA of the admissible blocks (Section "Compression": only r rows
// and r columns of a block are computed, r being the rank reached for the
// relative Frobenius tolerance eps).
//
// Rank step k of a block A (m x n), with U_l, V_l the previous factors:
//   1. residual row  r_j = A(i*, j) - sum_l U_l(i*) V_l(j)
//   2. pivot j* = argmax |r_j| (ties: lowest j), v_k = r / r_{j*}
//   3. residual column u_k(i) = A(i, j*) - sum_l V_l(j*) U_l(i)
//   4. ||S_k||^2 += ||u_k||^2 ||v_k||^2 + 2 sum_l (u_l.u_k)(v_l.v_k)
//   5. stop when ||u_k|| ||v_k|| <= eps ||S_k||; next row i* = argmax |u_k| over unused rows.
// The first row is local row 0.  A zero residual row is marked used and the
// lowest unused row is taken instead.  A block that reaches
// k = floor(m n / (m + n)) without converging is stored dense.
//
// GPU organisation: all admissible blocks of a band advance together, one
// rank step at a time.  Steps 1 and 3 are flat launches with one lane per
// matrix entry over every active block (a lane finds its block by binary
// search in a prefix array), so the expensive entry evaluations keep every
// lane busy whatever the block sizes; steps 2, 4 and 5 run one workgroup per
// active block.  Reductions use wavefront shuffles and one LDS stage in a
// fixed order, so results are bitwise reproducible.
#include <algorithm>
#include <map>
#include <climits>
#include <numeric>

#include "entry_dev.h"
#include "kernels.h"

namespace rte {

namespace {

enum : int { kActive = 0, kConverged = 1, kFailed = 2 };

template <typename T>
struct AcaState {
    const AcaTask *task;
    int nb;
    int *k, *istar, *jstar, *status, *havepiv;
    int *hits;                  // per block: consecutive rank steps that met the stopping test
    int64_t *ents;              // per block: entries evaluated (rows and columns)
    T *pivot, *normS2;
    unsigned *used;             // row bitmaps
    const int64_t *ubase;       // first bitmap word of each block
    int64_t *rowoff, *coloff;   // [nb + 1] prefix sums of the active widths
    int64_t *chunkoff;          // [nb + 1] prefix sums of the update chunks of the pivoted blocks
    int *act, *act2;            // active block lists (row phase, column phase)
    int64_t *tot;               // [0] row entries, [1] active blocks, [2] column entries, [3] pivoted blocks,
                                // [4] update chunks
    T *Us, *Vs;                 // U^T [kcap][m] and V^T [kcap][n] per block
    T *part;                    // per chunk: [2][half] partial dot products (half > every kcap)
    int half;                   // partials per kind in a chunk
    T *pmax;                    // per chunk: |u| max and its signed value
    int *pidx;                  // per chunk: row of the max
    int *hint_r, *hint_c;       // per 256 row / column entries: position in act / act2 of the
                                // block holding the first one (set after every scan)
    int *cblock;                // per update chunk: its block (set after every scan)
};

// elements of the concatenated (u_k, v_k) range of a block handled by one update chunk
constexpr int kChunk = 1024;

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
__device__ __forceinline__ void block_argmax(T &a, int &idx, T &sv, T *sa, int *si, T *ss) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    wave_argmax(a, idx, sv);
    if (lane == 0) { sa[wid] = a; si[wid] = idx; ss[wid] = sv; }
    __syncthreads();
    a = sa[0]; idx = si[0]; sv = ss[0];
#pragma unroll
    for (int w = 1; w < 4; ++w)
        if (sa[w] > a || (sa[w] == a && si[w] < idx)) { a = sa[w]; idx = si[w]; sv = ss[w]; }
    __syncthreads();
}

__device__ __forceinline__ bool is_used(const unsigned *bits, int r) { return (bits[r >> 5] >> (r & 31)) & 1u; }


}  // namespace

template <typename T>
__global__ __launch_bounds__(256) void k_aca_init(AcaState<T> st) {
    const int b = blockIdx.x;
    if (threadIdx.x == 0) {
        st.k[b] = 0;
        st.istar[b] = 0;
        st.jstar[b] = 0;
        st.status[b] = kActive;
        st.havepiv[b] = 0;
        st.hits[b] = 0;
        st.normS2[b] = (T)0;
        st.pivot[b] = (T)0;
        st.ents[b] = 0;
    }
    const int words = (st.task[b].m + 31) / 32;
    for (int w = threadIdx.x; w < words; w += blockDim.x) st.used[st.ubase[b] + w] = 0u;
}

// Prefix sums of the widths (row phase: n, column phase: m and the update
// chunks) of the active blocks, and the list of those blocks.  The lists are
// rebuilt every few rank steps; in between, the kernels skip blocks that have
// stopped (or, in the column phase, have no pivot this step).  One workgroup
// of 1024 lanes.
template <typename T, bool COLS>
__global__ __launch_bounds__(1024) void k_aca_scan(AcaState<T> st) {
    __shared__ int64_t sw[1024], sq[1024];
    __shared__ int sc[1024];
    const int nb = st.nb, tid = threadIdx.x;
    const int per = (nb + 1023) / 1024;
    const int b0 = min(nb, tid * per), b1 = min(nb, b0 + per);
    int64_t w = 0, q = 0;
    int c = 0;
    for (int b = b0; b < b1; ++b) {
        const bool on = st.status[b] == kActive;
        if (on) {
            w += COLS ? st.task[b].m : st.task[b].n;
            q += (st.task[b].m + st.task[b].n + kChunk - 1) / kChunk;
            ++c;
        }
    }
    sw[tid] = w;
    sq[tid] = q;
    sc[tid] = c;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {   // inclusive scan
        const int64_t a = tid >= o ? sw[tid - o] : 0;
        const int64_t aq = tid >= o ? sq[tid - o] : 0;
        const int ac = tid >= o ? sc[tid - o] : 0;
        __syncthreads();
        sw[tid] += a;
        sq[tid] += aq;
        sc[tid] += ac;
        __syncthreads();
    }
    int64_t off = sw[tid] - w, qoff = sq[tid] - q;
    int cnt = sc[tid] - c;
    int64_t *offs = COLS ? st.coloff : st.rowoff;
    int *list = COLS ? st.act2 : st.act;
    for (int b = b0; b < b1; ++b) {
        offs[b] = off;
        if (COLS) st.chunkoff[b] = qoff;
        const bool on = st.status[b] == kActive;
        if (on) {
            off += COLS ? st.task[b].m : st.task[b].n;
            qoff += (st.task[b].m + st.task[b].n + kChunk - 1) / kChunk;
            list[cnt++] = b;
        }
    }
    if (tid == 1023) {
        offs[nb] = sw[1023];
        st.tot[COLS ? 2 : 0] = sw[1023];
        st.tot[COLS ? 3 : 1] = sc[1023];
        if (COLS) {
            st.chunkoff[nb] = sq[1023];
            st.tot[4] = sq[1023];
        }
    }
}

// For each run of 256 entries (one workgroup of the row or column launch):
// the position in the active list of the block holding its first entry, so
// that a lane finds its block by stepping forward over a few blocks instead
// of a binary search over all of them.
template <typename T, bool COLS>
__global__ __launch_bounds__(256) void k_aca_hint(AcaState<T> st, int64_t nwg, int nact) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= nwg) return;
    const int64_t e = c * 256;
    const int64_t *off = COLS ? st.coloff : st.rowoff;
    const int *list = COLS ? st.act2 : st.act;
    int lo = 0, hi = nact;   // first i with off[list[i] + 1] > e
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (off[list[mid] + 1] > e) hi = mid;
        else lo = mid + 1;
    }
    (COLS ? st.hint_c : st.hint_r)[c] = lo;
}

// the block of every update chunk (a workgroup of k_aca_dots)
template <typename T>
__global__ __launch_bounds__(256) void k_aca_chunk_block(AcaState<T> st, int64_t nchunk, int nact) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= nchunk) return;
    int lo = 0, hi = nact;   // first i with chunkoff[act2[i] + 1] > c
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (st.chunkoff[st.act2[mid] + 1] > c) hi = mid;
        else lo = mid + 1;
    }
    st.cblock[c] = st.act2[lo];
}

// the block of entry e (below the launch's total) from its workgroup's hint
__device__ __forceinline__ int hinted_block(const int64_t *__restrict__ off, const int *__restrict__ list,
                                            const int *__restrict__ hint, int64_t e) {
    int i = hint[blockIdx.x];
    int b = list[i];
    while (off[b + 1] <= e) b = list[++i];
    return b;
}

// Waves per SIMD the entry launches are compiled for: the register budget
// that keeps the march free of spills (the surface entry needs more
// registers than the volume one; measured per kind and precision).
template <typename T, int KIND, int NW>
constexpr int entry_waves() {
    if constexpr (sizeof(T) == 8) return KIND == RTE_VOLUME ? 4 : 3;
    else return KIND == RTE_VOLUME ? (NW != kNoWall ? 6 : 7) : 5;
}

// a - sum_l p[l * sp] q[l * sq], l < k, subtracted in order of l; the loads
// of 8 terms are issued before their products (the factors were written by
// earlier rank steps and come from L2 or HBM).  Terms past k are zero and
// subtracting them leaves a unchanged, so the result is that of the plain
// loop.
template <typename T>
__device__ __forceinline__ T residual(T a, const T *p, int64_t sp, const T *q, int64_t sq, int k) {
    constexpr int B = 8;
    for (int l = 0; l < k; l += B) {
        T x[B], y[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const bool in = l + u < k;
            x[u] = in ? p[(int64_t)(l + u) * sp] : (T)0;
            y[u] = in ? q[(int64_t)(l + u) * sq] : (T)0;
        }
#pragma unroll
        for (int u = 0; u < B; ++u) a -= x[u] * y[u];
    }
    return a;
}

// Step 1: residual rows of every active block, one lane per entry.
template <typename T, int KIND, int NW>
__global__ __launch_bounds__(256, (entry_waves<T, KIND, NW>())) void k_aca_rows(EntryCtx<T> c, AcaState<T> st, int64_t total,
                                                  const int64_t *__restrict__ tgt_nat,
                                                  const int64_t *__restrict__ src_nat) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= total) return;
    const int b = hinted_block(st.rowoff, st.act, st.hint_r, e);
    if (st.status[b] != kActive) return;
    const int j = (int)(e - st.rowoff[b]);
    T a;
    {
        const AcaTask tk = st.task[b];
        a = entry<T, KIND, NW>(c, tgt_nat[tk.t0 + st.istar[b]], src_nat[tk.s0 + j]);
    }
    // the block's state is read again after the march (only b and j stay
    // live through it; the barrier keeps the compiler from reusing the loads)
    asm volatile("" ::: "memory");
    const AcaTask tk = st.task[b];
    const int k = st.k[b], is = st.istar[b];
    const T *U = st.Us + tk.uoff;
    T *V = st.Vs + tk.voff;
    a = residual(a, U + is, tk.m, V + j, tk.n, k);
    V[(int64_t)k * tk.n + j] = a;
}

// Step 2: pivot column of each active block, or the next row after a zero row.
template <typename T>
__global__ __launch_bounds__(256) void k_aca_pivot(AcaState<T> st) {
    __shared__ T sa[4], ss[4];
    __shared__ int si[4];
    const int b = st.act[blockIdx.x];
    if (st.status[b] != kActive) return;
    const AcaTask tk = st.task[b];
    const int k = st.k[b];
    const T *V = st.Vs + tk.voff + (int64_t)k * tk.n;
    if (threadIdx.x == 0) st.ents[b] += tk.n;
    unsigned *bits = st.used + st.ubase[b];
    T best = (T)-1, sv = (T)0;
    int bj = INT_MAX;
    for (int j = threadIdx.x; j < tk.n; j += 256) {
        const T v = V[j], av = fabs(v);
        if (av > best) { best = av; bj = j; sv = v; }
    }
    block_argmax(best, bj, sv, sa, si, ss);
    if (threadIdx.x == 0) {
        const int is = st.istar[b];
        bits[is >> 5] |= 1u << (is & 31);
    }
    if (best > (T)0) {
        if (threadIdx.x == 0) {
            st.jstar[b] = bj;
            st.pivot[b] = sv;
            st.havepiv[b] = 1;
        }
        return;
    }
    // zero residual row: the lowest unused row is next
    __syncthreads();   // the bit of i* is visible
    int cand = INT_MAX;
    for (int r = threadIdx.x; r < tk.m; r += 256)
        if (!is_used(bits, r)) { cand = r; break; }
    T key = cand == INT_MAX ? (T)-1 : (T)1, dv = (T)0;
    block_argmax(key, cand, dv, sa, si, ss);
    if (threadIdx.x == 0) {
        st.havepiv[b] = 0;
        if (key < (T)0) st.status[b] = kConverged;   // every row used: the residual is zero
        else st.istar[b] = cand;
    }
}

// Step 3: residual columns of the pivoted blocks, one lane per entry.
template <typename T, int KIND, int NW>
__global__ __launch_bounds__(256, (entry_waves<T, KIND, NW>())) void k_aca_cols(EntryCtx<T> c, AcaState<T> st, int64_t total,
                                                  const int64_t *__restrict__ tgt_nat,
                                                  const int64_t *__restrict__ src_nat) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= total) return;
    const int b = hinted_block(st.coloff, st.act2, st.hint_c, e);
    if (st.status[b] != kActive || !st.havepiv[b]) return;
    const int i = (int)(e - st.coloff[b]);
    T a;
    {
        const AcaTask tk = st.task[b];
        a = entry<T, KIND, NW>(c, tgt_nat[tk.t0 + i], src_nat[tk.s0 + st.jstar[b]]);
    }
    asm volatile("" ::: "memory");   // as in k_aca_rows
    const AcaTask tk = st.task[b];
    const int k = st.k[b], js = st.jstar[b];
    T *U = st.Us + tk.uoff;
    const T *V = st.Vs + tk.voff;
    // V_l(j*) for l < k is already scaled; V_k is scaled in step 4
    a = residual(a, V + js, tk.n, U + i, tk.m, k);
    U[(int64_t)k * tk.m + i] = a;
}

// Steps 4-5, first part: scale v_k and form the partial dot products
// (u_l.u_k), (v_l.v_k), l <= k, and the partial argmax of |u_k| over unused
// rows, on one chunk of the concatenated (u_k, v_k) range of a block.  The
// chunk of (u_k, v_k) is staged in LDS (v_k scaled there and in memory).  For
// l < k a group of P consecutive lanes owns rank index l: its lanes read
// every P-th element of row l (contiguous across the group), and one
// butterfly over the group ends the sum, for all groups of a wavefront at
// once.  P is the largest power of two with 256 / P groups covering the k
// indices (at most 64), but at least 8 (64 contiguous bytes of a row per
// load; the 32 groups then take the k indices in passes).  The squares of
// u_k and v_k (l = k) come from the staging pass.
template <typename T>
__global__ __launch_bounds__(256) void k_aca_dots(AcaState<T> st) {
    __shared__ T ck[kChunk];
    __shared__ T sq[2][4];
    __shared__ T sa[4], ss[4];
    __shared__ int si[4];
    const int64_t c = blockIdx.x;
    const int b = st.cblock[c];
    if (st.status[b] != kActive || !st.havepiv[b]) return;   // uniform over the workgroup
    const AcaTask tk = st.task[b];
    const int k = st.k[b], m = tk.m, n = tk.n;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int e0 = (int)(c - st.chunkoff[b]) * kChunk;
    const int e1 = min(e0 + kChunk, m + n);
    const T *U = st.Us + tk.uoff;
    T *V = st.Vs + tk.voff;
    const unsigned *bits = st.used + st.ubase[b];
    const T inv = (T)1 / st.pivot[b];
    T bu = (T)-1, busv = (T)0, su = (T)0, sv = (T)0;
    int bi = INT_MAX;
    for (int e = e0 + tid; e < e1; e += 256) {
        if (e < m) {
            const T u = U[(int64_t)k * m + e];
            ck[e - e0] = u;
            su += u * u;
            if (!is_used(bits, e) && fabs(u) > bu) { bu = fabs(u); bi = e; busv = u; }
        } else {
            T *vp = V + (int64_t)k * n + (e - m);
            const T v = *vp * inv;
            *vp = v;
            ck[e - e0] = v;
            sv += v * v;
        }
    }
    su = wave_sum(su);
    sv = wave_sum(sv);
    if (lane == 0) { sq[0][wid] = su; sq[1][wid] = sv; }
    block_argmax(bu, bi, busv, sa, si, ss);   // its barriers publish ck and sq
    T *part = st.part + c * 2 * (int64_t)st.half;
    if (k > 0) {
        int P = 64;
        while (P > 8 && 256 / P < k) P >>= 1;
        const int G = 256 / P, g = tid / P, q = tid - g * P;
        const int eu1 = min(e1, m), ev0 = max(e0, m);
        for (int l0 = 0; l0 < k; l0 += G) {
            const int l = l0 + g;
            T pu = (T)0, pv = (T)0;
            if (l < k) {
                const T *ur = U + (int64_t)l * m;
                const T *vr = V + (int64_t)l * n - m;
#pragma unroll 8
                for (int e = e0 + q; e < eu1; e += P) pu += ur[e] * ck[e - e0];
#pragma unroll 8
                for (int e = ev0 + q; e < e1; e += P) pv += vr[e] * ck[e - e0];
            }
            for (int o = P >> 1; o > 0; o >>= 1) {
                pu += __shfl_xor(pu, o, 64);
                pv += __shfl_xor(pv, o, 64);
            }
            if (l < k && q == 0) {
                part[l] = pu;
                part[st.half + l] = pv;
            }
        }
    }
    if (tid == 0) {
        part[k] = ((sq[0][0] + sq[0][1]) + sq[0][2]) + sq[0][3];
        part[st.half + k] = ((sq[1][0] + sq[1][1]) + sq[1][2]) + sq[1][3];
        st.pmax[2 * c] = bu;
        st.pmax[2 * c + 1] = busv;
        st.pidx[c] = bi;
    }
}

// Steps 4-5, second part: add the chunk partials in order, update ||S_k||,
// test convergence and pick the next row.  One wavefront per pivoted block.
template <typename T>
__global__ __launch_bounds__(64) void k_aca_finish(AcaState<T> st, T eps, int need) {
    const int b = st.act2[blockIdx.x];
    if (st.status[b] != kActive || !st.havepiv[b]) return;
    const AcaTask tk = st.task[b];
    const int k = st.k[b], lane = threadIdx.x;
    if (lane == 0) st.ents[b] += tk.m;
    const int64_t c0 = st.chunkoff[b], c1 = st.chunkoff[b + 1];
    T cross = (T)0, u2 = (T)0, v2 = (T)0;
    for (int l = lane; l <= k; l += 64) {
        T su = (T)0, sv = (T)0;
        for (int64_t c = c0; c < c1; ++c) {
            su += st.part[c * 2 * st.half + l];
            sv += st.part[c * 2 * st.half + st.half + l];
        }
        if (l < k) cross += su * sv;
        else { u2 = su; v2 = sv; }
    }
    cross = wave_sum(cross);
    u2 = wave_sum(u2);
    v2 = wave_sum(v2);
    if (lane != 0) return;
    T bu = (T)-1, busv = (T)0;
    int bi = INT_MAX;
    for (int64_t c = c0; c < c1; ++c) {
        const T a = st.pmax[2 * c];
        const int i = st.pidx[c];
        if (a > bu || (a == bu && i < bi)) { bu = a; bi = i; busv = st.pmax[2 * c + 1]; }
    }
    (void)busv;
    const T s2 = st.normS2[b] + u2 * v2 + (T)2 * cross;
    st.normS2[b] = s2;
    // the stopping test, met by `need` consecutive rank steps
    const int hits = sqrt(u2 * v2) <= eps * sqrt(fabs(s2)) ? st.hits[b] + 1 : 0;
    st.hits[b] = hits;
    const bool stop = hits >= need;
    const int kn = k + 1;
    st.k[b] = kn;
    st.havepiv[b] = 0;
    if (stop) st.status[b] = kConverged;
    else if (kn >= tk.kcap) st.status[b] = kFailed;
    else if (bi == INT_MAX) st.status[b] = kConverged;   // every row used
    else st.istar[b] = bi;
}

__global__ void k_aca_ranks(const int *__restrict__ k, const int *__restrict__ status, int nb, int *__restrict__ out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) out[b] = status[b] == kConverged ? k[b] : -1;
}

// One piece of a block's compaction: rows [r0, r1) of U (part 0) or a range
// [r0, r1) of V (part 1: sources for FP64 / FP32 storage, groups of 8 stored
// source coordinates for BF16), so that the large blocks are spread over
// many workgroups instead of setting the length of the launch.
struct CompactTask {
    const void *su, *sv;
    void *du, *dv;
    void *dul, *dvl;      // BF16 lo parts (mixed precision)
    int64_t t0, s0;       // first target row and first source of the block
    int32_t m, n, k, li0; // li0: target leaf of t0
    int32_t part, r0, r1, pad;
};
constexpr int kCompactRows = 512;   // U rows per piece
constexpr int kCompactCols = 256;   // V sources per piece (FP64 / FP32)
constexpr int kCompactGroups = 32;  // V groups of 8 stored coordinates per piece (BF16)

// Final layout of a low-rank block (FP64 / FP32 storage): U in target-leaf
// slices, each column-major [k][rp], and V row-major [n][kp], kp = pad4(k).
// U: a thread owns 8 consecutive columns of one row (one slice lookup, 8
// loads issued before any store; reads of the U^T rows and writes of the
// slice columns are contiguous across threads).  V: [k][n] -> [n][kp] is a
// transpose, taken through an LDS tile of 32 ranks x 64 sources so that both
// the reads and the writes are contiguous.  Padding is written as zero.
template <typename T>
__global__ __launch_bounds__(256) void k_compact(const CompactTask *__restrict__ tasks, SliceMap sm) {
    __shared__ T tile[32][65];
    const CompactTask t = tasks[blockIdx.x];
    const T *__restrict__ su = static_cast<const T *>(t.su);
    const T *__restrict__ sv = static_cast<const T *>(t.sv);
    T *__restrict__ du = static_cast<T *>(t.du);
    T *__restrict__ dv = static_cast<T *>(t.dv);
    const int m = t.m, n = t.n, k = t.k, tid = threadIdx.x;
    if (t.part == 0) {
        const int rows = t.r1 - t.r0;
        const int64_t nu = (int64_t)((k + 7) / 8) * rows;
        for (int64_t e = tid; e < nu; e += blockDim.x) {
            const int lg = (int)(e / rows), i = t.r0 + (int)(e - (int64_t)lg * rows);
            const SliceRow sr = slice_row(sm, t.li0, t.t0 + i, k, t.li0 + i + 1);
            const int l0 = 8 * lg;
            T v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = l0 + u < k ? su[(int64_t)(l0 + u) * m + i] : (T)0;
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (l0 + u < k) du[sr.base + (int64_t)(l0 + u) * sr.rp + sr.r] = v[u];
        }
        return;
    }
    const int kp = (int)pad4(k);   // the branch is uniform over the workgroup: the barriers below are safe
    for (int j0 = t.r0; j0 < t.r1; j0 += 64)
        for (int l0 = 0; l0 < kp; l0 += 32) {
            const int jl = tid & 63;
            for (int p = tid >> 6; p < 32; p += 4) {
                const int l = l0 + p, j = j0 + jl;
                tile[p][jl] = l < k && j < t.r1 ? sv[(int64_t)l * n + j] : (T)0;
            }
            __syncthreads();
            const int ll = tid & 31;
            for (int q = tid >> 5; q < 64; q += 8) {
                const int l = l0 + ll, j = j0 + q;
                if (j < t.r1 && l < kp) dv[(int64_t)j * kp + l] = tile[ll][q];
            }
            __syncthreads();
        }
}

// Mixed precision (K-grouped BF16 storage): each factor element x (FP32) is
// stored as hi = bf16(x) and lo = bf16(x - hi).  U: slice rows of 8
// consecutive rank columns ([k8/8][r][8]); V: [nP/8][k][8] over the stored
// source coordinates (src_p), whose padding stays zero.  A thread writes one
// 16-byte group of 8 elements of each array.
__global__ __launch_bounds__(256) void k_compact_bf16(const CompactTask *__restrict__ tasks, SliceMap sm,
                                                      const int64_t *__restrict__ pmap) {
    const CompactTask t = tasks[blockIdx.x];
    const float *su = static_cast<const float *>(t.su), *sv = static_cast<const float *>(t.sv);
    uint16_t *uh = static_cast<uint16_t *>(t.du), *vh = static_cast<uint16_t *>(t.dv);
    uint16_t *ul = static_cast<uint16_t *>(t.dul), *vl = static_cast<uint16_t *>(t.dvl);
    auto put8 = [](uint16_t *hi, uint16_t *lo, int64_t o, const float x[8]) {
        uint32_t h[4], l[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint16_t h0 = f2bf(x[2 * e]), h1 = f2bf(x[2 * e + 1]);
            h[e] = (uint32_t)h0 | ((uint32_t)h1 << 16);
            l[e] = (uint32_t)f2bf(x[2 * e] - bf2f(h0)) | ((uint32_t)f2bf(x[2 * e + 1] - bf2f(h1)) << 16);
        }
        *reinterpret_cast<uint4 *>(hi + o) = make_uint4(h[0], h[1], h[2], h[3]);
        *reinterpret_cast<uint4 *>(lo + o) = make_uint4(l[0], l[1], l[2], l[3]);
    };
    if (t.part == 0) {
        const int kg = (t.k + 7) / 8, rows = t.r1 - t.r0;
        const int64_t nu = (int64_t)kg * rows;
        for (int64_t e = threadIdx.x; e < nu; e += blockDim.x) {
            const int64_t lg = e / rows, i = t.r0 + (e - lg * rows);
            const SliceRow sr = slice_row(sm, t.li0, t.t0 + i, t.k, t.li0 + (int)i + 1);
            float x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = 8 * lg + u < t.k ? su[(8 * lg + u) * t.m + i] : 0.0f;
            put8(uh, ul, sr.base + (lg * sr.rp + sr.r) * 8, x);
        }
        return;
    }
    const int64_t p0 = sm.src_p[t.s0];
    const int64_t nv = (int64_t)(t.r1 - t.r0) * t.k;
    for (int64_t e = threadIdx.x; e < nv; e += blockDim.x) {
        const int64_t jg = t.r0 + e / t.k, l = e % t.k;
        float x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t j = pmap[p0 + 8 * jg + u];
            x[u] = j >= 0 ? sv[l * t.n + (j - t.s0)] : 0.0f;
        }
        put8(vh, vl, (jg * t.k + l) * 8, x);
    }
}

// ---------------------------------------------------------------- host side

namespace {

SliceMap slice_map(const HMat &H) {
    return {H.leaf_start.as<int64_t>(), H.leaf_prp.as<int64_t>(), H.src_p.as<int64_t>(),
            (int)H.plan->tgt_leaves.size(), H.kgroup};
}

int64_t round8(int64_t e) { return (e + 7) & ~(int64_t)7; }

// padded rows of the target leaves covered by rows [t0, t1)
int64_t padded_rows(const HMat &H, int64_t t0, int64_t t1) {
    const Plan &P = *H.plan;
    return H.leaf_prp_h[P.leaf_of(t1 - 1) + 1] - H.leaf_prp_h[P.leaf_of(t0)];
}

// stored elements of the row side (K columns over rows [t0, t1)) and of V
int64_t stored_u(const HMat &H, int64_t t0, int64_t t1, int64_t K) {
    const int64_t g = H.kgroup;
    return (K + g - 1) / g * g * padded_rows(H, t0, t1);
}
int64_t stored_v(const HMat &H, int64_t s0, int64_t s1, int64_t k) {
    return H.kgroup > 1 ? H.pwidth(s0, s1) * k : (s1 - s0) * pad4(k);
}

template <typename T>
void fill_dense_blocks(HMat &H, BandStore &B, BandKappa<T> kap, const std::vector<Block> &blocks, bool pair,
                       hipStream_t s) {
    if (blocks.empty()) return;
    const Plan &P = *H.plan;
    const bool split = H.precision == RTE_MIXED_BF16;
    const size_t esz = split ? sizeof(uint16_t) : sizeof(T);
    int64_t total = 0, stored = 0;
    for (auto &b : blocks) {
        total += (b.t1 - b.t0) * (b.s1 - b.s0);
        stored += round8(stored_u(H, b.t0, b.t1, H.pwidth(b.s0, b.s1)));
    }
    DevBuf buf(esz * (size_t)stored), lo(split ? esz * (size_t)stored : 0);
    HIP_CHECK(hipMemsetAsync(buf.p, 0, buf.bytes, s));   // the row padding stays zero
    if (split) HIP_CHECK(hipMemsetAsync(lo.p, 0, lo.bytes, s));
    std::vector<char *> ptr(blocks.size()), ptrl(blocks.size());
    int64_t off = 0;
    for (size_t d = 0; d < blocks.size(); ++d) {
        const Block &b = blocks[d];
        ptr[d] = static_cast<char *>(buf.p) + off * esz;
        ptrl[d] = split ? static_cast<char *>(lo.p) + off * esz : nullptr;
        B.dense_blocks.push_back(b);
        B.dense_ptr.push_back(ptr[d]);
        B.dense_lo.push_back(ptrl[d]);
        off += round8(stored_u(H, b.t0, b.t1, H.pwidth(b.s0, b.s1)));
    }
    // volume operator: an off-diagonal block and its transpose are filled by
    // one set of tasks (each lane computes G(i, j) and G(j, i) on one march)
    std::map<std::pair<int64_t, int64_t>, size_t> at;
    if (pair)
        for (size_t d = 0; d < blocks.size(); ++d) at[{blocks[d].t0, blocks[d].s0}] = d;
    std::vector<FillTask> tasks;
    for (size_t d = 0; d < blocks.size(); ++d) {
        const Block &b = blocks[d];
        const int m = (int)(b.t1 - b.t0), n = (int)(b.s1 - b.s0), li0 = P.leaf_of(b.t0);
        const int32_t kw = (int32_t)H.pwidth(b.s0, b.s1);
        FillTask t{ptr[d], ptrl[d], b.t0, b.s0, m, n, li0, kw, 0, nullptr, nullptr, 0, 0};
        if (pair && b.t0 != b.s0) {
            auto it = at.find({b.s0, b.t0});
            if (it != at.end() && blocks[it->second].t1 == b.s1 && blocks[it->second].s1 == b.t1) {
                if (b.t0 > b.s0) continue;   // filled with its transpose
                t.out_t = ptr[it->second];
                t.outlo_t = ptrl[it->second];
                t.li0_t = P.leaf_of(b.s0);
                t.kw_t = (int32_t)H.pwidth(b.t0, b.t1);
            }
        }
        for (int64_t f = 0; f < (int64_t)m * n; f += kFillChunk) {
            t.first = f;
            tasks.push_back(t);
        }
    }
    dense_fill_launch<T>(*H.mesh, H.kind, kap, tasks, H.tgt_nat.as<int64_t>(), H.src_nat.as<int64_t>(), slice_map(H),
                         split, B, s);
    B.fill_launches += 1;
    B.dense_entries += total;
    B.evaluated += total;
    B.bytes += (int64_t)(buf.bytes + lo.bytes);
    B.bufs.push_back(std::move(buf));
    if (split) B.bufs.push_back(std::move(lo));
}

// One batch of blocks through the step-synchronous ACA.  A block that stops
// at its cap goes to `retry` when its storage break-even rank exceeds the cap
// (the next pass runs it again with a larger one), else to `fallback` (dense).
template <typename T>
void aca_batch(HMat &H, BandStore &B, BandKappa<T> kap, const std::vector<AcaTask> &tasks, const std::vector<size_t> &ids,
               int64_t uo, int64_t vo, std::vector<Block> &fallback, std::vector<size_t> &retry, hipStream_t s) {
    {   // an earlier batch's scratch is freed first (a fill's task list may stay queued)
        size_t pending = 0;
        for (const DevBuf &d : B.retire) pending += d.bytes;
        if (pending > ((size_t)256 << 20)) band_settle(B, s);
    }
    const Plan &P = *H.plan;
    const int nb = (int)tasks.size();
    int kmax = 1;
    for (auto &t : tasks) kmax = std::max(kmax, t.kcap);
    std::vector<int64_t> ubase(nb);
    int64_t words = 0;
    for (int b = 0; b < nb; ++b) {
        ubase[b] = words;
        words += (tasks[b].m + 31) / 32;
    }
    // every buffer of the batch comes from the scratch pool and goes back to it
    // once the band's stream has drained (band_settle)
    auto scratch = [](size_t b) { return DevBuf::scratch(b); };
    DevBuf Us = scratch(sizeof(T) * (size_t)uo), Vs = scratch(sizeof(T) * (size_t)vo);
    DevBuf dt = upload_scratch(tasks, s), dub = upload_scratch(ubase, s);
    int64_t max_chunks = 0;
    for (auto &t : tasks) max_chunks += (t.m + t.n + kChunk - 1) / kChunk;
    DevBuf ents = scratch(sizeof(int64_t) * (size_t)nb);
    DevBuf ints = scratch(sizeof(int) * (size_t)nb * 8), reals = scratch(sizeof(T) * (size_t)nb * 2),
           used = scratch(sizeof(unsigned) * (size_t)words), offs = scratch(sizeof(int64_t) * (size_t)(nb + 1) * 3),
           tot = scratch(sizeof(int64_t) * 5),
           part = scratch(sizeof(T) * (size_t)max_chunks * 2 * (size_t)(kmax + 1)),
           pmax = scratch(sizeof(T) * (size_t)max_chunks * 2), pidx = scratch(sizeof(int) * (size_t)max_chunks);
    int64_t sum_m = 0, sum_n = 0;
    for (auto &t : tasks) {
        sum_m += t.m;
        sum_n += t.n;
    }
    DevBuf hints = scratch(sizeof(int) * (size_t)((sum_n + 255) / 256 + (sum_m + 255) / 256 + 2));
    AcaState<T> st;
    st.task = dt.as<AcaTask>();
    st.nb = nb;
    int *ip = ints.as<int>();
    st.k = ip;
    st.istar = ip + nb;
    st.jstar = ip + 2 * nb;
    st.status = ip + 3 * nb;
    st.havepiv = ip + 4 * nb;
    st.act = ip + 5 * nb;
    st.act2 = ip + 6 * nb;
    st.hits = ip + 7 * nb;
    st.ents = ents.as<int64_t>();
    st.pivot = reals.as<T>();
    st.normS2 = reals.as<T>() + nb;
    st.used = used.as<unsigned>();
    st.ubase = dub.as<int64_t>();
    st.rowoff = offs.as<int64_t>();
    st.coloff = offs.as<int64_t>() + nb + 1;
    st.chunkoff = offs.as<int64_t>() + 2 * (nb + 1);
    st.tot = tot.as<int64_t>();
    st.part = part.as<T>();
    st.half = kmax + 1;
    st.pmax = pmax.as<T>();
    st.pidx = pidx.as<int>();
    st.hint_r = hints.as<int>();
    st.hint_c = hints.as<int>() + (sum_n + 255) / 256 + 1;
    DevBuf cblock = scratch(sizeof(int) * (size_t)std::max<int64_t>(max_chunks, 1));
    // pooled scratch holds what an earlier batch left: the checking aid fills it with NaN bytes
    for (DevBuf *d : {&Us, &Vs, &ents, &ints, &reals, &used, &offs, &tot, &part, &pmax, &pidx, &hints, &cblock})
        poison(*d, s);
    st.cblock = cblock.as<int>();
    st.Us = Us.as<T>();
    st.Vs = Vs.as<T>();
    auto c = make_ctx<T>(*H.mesh, kap);
    const T eps = (T)H.opts.aca_eps;
    const int64_t *tn = H.tgt_nat.as<int64_t>(), *sn = H.src_nat.as<int64_t>();
    // every step raises a rank or consumes a zero row, so this bounds the steps
    int max_steps = 0;
    for (auto &t : tasks) max_steps = std::max(max_steps, t.kcap + t.m);

    EventTimer whole(s);
    // HIP events around the entry launches, read once after the batch
    std::vector<hipEvent_t> evs;
    auto mark = [&]() {
        hipEvent_t e;
        HIP_CHECK(hipEventCreate(&e));
        HIP_CHECK(hipEventRecord(e, s));
        evs.push_back(e);
    };
    int launches = 0;
    whole.start();
    k_aca_init<T><<<nb, 256, 0, s>>>(st);
    HIP_LAUNCH_CHECK();
    // The active lists are rebuilt every kCompact steps (one host read of the
    // totals); in between, every step reuses them and the kernels skip the
    // blocks that have stopped, so a step costs five launches and no host
    // synchronisation.
    constexpr int kCompact = 8;
    int64_t ht[5];
    for (int step = 0; step <= max_steps;) {
        k_aca_scan<T, false><<<1, 1024, 0, s>>>(st);
        k_aca_scan<T, true><<<1, 1024, 0, s>>>(st);
        HIP_LAUNCH_CHECK();
        HIP_CHECK(hipMemcpyAsync(ht, st.tot, sizeof(int64_t) * 5, hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        if (ht[1] == 0) break;
        const int64_t nrow = ht[0], nact = ht[1], ncol = ht[2], nchunk = ht[4];
        const int64_t wr = (nrow + 255) / 256, wc = (ncol + 255) / 256;
        k_aca_hint<T, false><<<(unsigned)((wr + 255) / 256), 256, 0, s>>>(st, wr, (int)nact);
        k_aca_hint<T, true><<<(unsigned)((wc + 255) / 256), 256, 0, s>>>(st, wc, (int)ht[3]);
        k_aca_chunk_block<T><<<(unsigned)((nchunk + 255) / 256), 256, 0, s>>>(st, nchunk, (int)ht[3]);
        HIP_LAUNCH_CHECK();
        // the entry launches, compiled for the mesh's wall mode (no wall, one, several)
        const int wm = wall_mode(c.g);
        auto rows = [&](auto kernel) { kernel<<<(unsigned)((nrow + 255) / 256), 256, 0, s>>>(c, st, nrow, tn, sn); };
        auto cols = [&](auto kernel) { kernel<<<(unsigned)((ncol + 255) / 256), 256, 0, s>>>(c, st, ncol, tn, sn); };
        auto launch_rows = [&]() {
            if (H.kind == RTE_VOLUME) {
                if (wm == kNoWall) rows(k_aca_rows<T, RTE_VOLUME, kNoWall>);
                else if (wm == kOneWall) rows(k_aca_rows<T, RTE_VOLUME, kOneWall>);
                else rows(k_aca_rows<T, RTE_VOLUME, kAnyWalls>);
            } else {
                if (wm == kNoWall) rows(k_aca_rows<T, RTE_SURFACE, kNoWall>);
                else if (wm == kOneWall) rows(k_aca_rows<T, RTE_SURFACE, kOneWall>);
                else rows(k_aca_rows<T, RTE_SURFACE, kAnyWalls>);
            }
        };
        auto launch_cols = [&]() {
            if (H.kind == RTE_VOLUME) {
                if (wm == kNoWall) cols(k_aca_cols<T, RTE_VOLUME, kNoWall>);
                else if (wm == kOneWall) cols(k_aca_cols<T, RTE_VOLUME, kOneWall>);
                else cols(k_aca_cols<T, RTE_VOLUME, kAnyWalls>);
            } else {
                if (wm == kNoWall) cols(k_aca_cols<T, RTE_SURFACE, kNoWall>);
                else if (wm == kOneWall) cols(k_aca_cols<T, RTE_SURFACE, kOneWall>);
                else cols(k_aca_cols<T, RTE_SURFACE, kAnyWalls>);
            }
        };
        for (int r = 0; r < kCompact && step <= max_steps; ++r, ++step) {
            mark();
            launch_rows();
            HIP_LAUNCH_CHECK();
            mark();
            k_aca_pivot<T><<<(unsigned)nact, 256, 0, s>>>(st);
            HIP_LAUNCH_CHECK();
            mark();
            launch_cols();
            HIP_LAUNCH_CHECK();
            mark();
            k_aca_dots<T><<<(unsigned)nchunk, 256, 0, s>>>(st);
            k_aca_finish<T><<<(unsigned)nact, 64, 0, s>>>(st, eps, std::max(1, H.opts.aca_hits));
            HIP_LAUNCH_CHECK();
            launches += 2;
        }
    }
    whole.stop();
    const double whole_ms = whole.ms();   // synchronises: every event below has completed
    double entry_ms = 0.0;
    for (size_t e = 0; e + 1 < evs.size(); e += 2) {
        float ms = 0.0f;
        HIP_CHECK(hipEventElapsedTime(&ms, evs[e], evs[e + 1]));
        entry_ms += ms;
    }
    for (hipEvent_t e : evs) (void)hipEventDestroy(e);
    // exact count of the entries evaluated (per-block counters)
    int64_t entries = 0;
    {
        std::vector<int64_t> he(nb);
        HIP_CHECK(hipMemcpyAsync(he.data(), st.ents, sizeof(int64_t) * nb, hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        for (int64_t v : he) entries += v;
    }
    B.aca_ms += whole_ms;
    B.aca_entry_ms += entry_ms;
    B.aca_entry_launches += launches;
    B.aca_launches += 1;
    B.aca_entries += entries;
    B.evaluated += entries;

    DevBuf dr = scratch(sizeof(int) * (size_t)nb);
    k_aca_ranks<<<(nb + 255) / 256, 256, 0, s>>>(st.k, st.status, nb, dr.as<int>());
    HIP_LAUNCH_CHECK();
    std::vector<int> rk(nb);
    HIP_CHECK(hipMemcpyAsync(rk.data(), dr.p, sizeof(int) * rk.size(), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (H.opts.recompress) recompress_batch<T>(tasks, rk, Us.as<T>(), Vs.as<T>(), H.opts.aca_eps, B, s);
    int64_t total = 0;
    for (int t = 0; t < nb; ++t)
        if (rk[t] > 0)
            total += round8(stored_u(H, tasks[t].t0, tasks[t].t0 + tasks[t].m, rk[t])) +
                     round8(stored_v(H, tasks[t].s0, tasks[t].s0 + tasks[t].n, rk[t]));
    const bool split = H.precision == RTE_MIXED_BF16;
    const size_t esz = split ? sizeof(uint16_t) : sizeof(T);
    DevBuf out(esz * (size_t)total), outlo(split ? esz * (size_t)total : 0);
    HIP_CHECK(hipMemsetAsync(out.p, 0, out.bytes, s));   // slice and row padding stays zero
    if (split) HIP_CHECK(hipMemsetAsync(outlo.p, 0, outlo.bytes, s));
    std::vector<CompactTask> ct;
    ct.reserve((size_t)nb * 2);
    int64_t off = 0;
    for (int t = 0; t < nb; ++t) {
        const size_t b = ids[t];
        if (rk[t] <= 0) {
            const int64_t m = tasks[t].m, n = tasks[t].n;
            if (m * n / (m + n) > tasks[t].kcap && tasks[t].kcap < kAcaRetryRank) retry.push_back(b);
            else fallback.push_back(P.lowrank[b]);
            continue;
        }
        const int64_t nu = round8(stored_u(H, tasks[t].t0, tasks[t].t0 + tasks[t].m, rk[t])),
                      nv = round8(stored_v(H, tasks[t].s0, tasks[t].s0 + tasks[t].n, rk[t]));
        char *du = static_cast<char *>(out.p) + off * esz, *dv = du + nu * esz;
        char *dul = split ? static_cast<char *>(outlo.p) + off * esz : nullptr;
        char *dvl = split ? dul + nu * esz : nullptr;
        const CompactTask whole{Us.as<T>() + tasks[t].uoff, Vs.as<T>() + tasks[t].voff, du, dv, dul, dvl,
                                tasks[t].t0, tasks[t].s0, tasks[t].m, tasks[t].n, rk[t], P.leaf_of(tasks[t].t0),
                                0, 0, 0, 0};
        for (int r0 = 0; r0 < whole.m; r0 += kCompactRows) {
            CompactTask piece = whole;
            piece.r0 = r0;
            piece.r1 = (int)std::min<int64_t>(whole.m, r0 + kCompactRows);
            ct.push_back(piece);
        }
        const int64_t vend = split ? H.pwidth(tasks[t].s0, tasks[t].s0 + tasks[t].n) / 8 : tasks[t].n;
        const int vstep = split ? kCompactGroups : kCompactCols;
        for (int64_t r0 = 0; r0 < vend; r0 += vstep) {
            CompactTask piece = whole;
            piece.part = 1;
            piece.r0 = (int)r0;
            piece.r1 = (int)std::min<int64_t>(vend, r0 + vstep);
            ct.push_back(piece);
        }
        B.rank[b] = rk[t];
        B.U[b] = du;
        B.V[b] = dv;
        if (split) {
            B.Ulo[b] = dul;
            B.Vlo[b] = dvl;
        }
        B.lr_entries += (int64_t)rk[t] * (tasks[t].m + tasks[t].n);
        off += nu + nv;   // U and V each start 16-byte aligned for BF16, 32-byte for FP64
    }
    if (!ct.empty()) {
        DevBuf dct = upload_scratch(ct, s);
        if (split)
            k_compact_bf16<<<(unsigned)ct.size(), 256, 0, s>>>(dct.as<CompactTask>(), slice_map(H),
                                                              H.src_pmap.as<int64_t>());
        else k_compact<T><<<(unsigned)ct.size(), 256, 0, s>>>(dct.as<CompactTask>(), slice_map(H));
        HIP_LAUNCH_CHECK();
        B.retire.push_back(std::move(dct));
    }
    // The compaction reads the scratch while the host goes on (dense fallback,
    // matvec plan): every buffer of the batch is freed by band_settle().
    for (DevBuf *d : {&Us, &Vs, &dt, &dub, &ents, &ints, &reals, &used, &offs, &tot, &part, &pmax, &pidx, &hints,
                      &cblock, &dr})
        B.retire.push_back(std::move(*d));
    B.bytes += (int64_t)(out.bytes + outlo.bytes);
    B.bufs.push_back(std::move(out));
    if (split) B.bufs.push_back(std::move(outlo));
}

template <typename T>
void run_aca(HMat &H, BandStore &B, BandKappa<T> kap, hipStream_t s) {
    const Plan &P = *H.plan;
    const size_t nlr = P.lowrank.size();
    B.rank.assign(nlr, -1);
    B.U.assign(nlr, nullptr);
    B.V.assign(nlr, nullptr);
    B.Ulo.assign(nlr, nullptr);
    B.Vlo.assign(nlr, nullptr);
    std::vector<Block> fallback;
    // bytes of U/V scratch per batch: a quarter of the free memory, within
    // [2, 48] GiB (one batch for the common sizes: every batch has its own
    // set-up and its own tail of a few high-rank blocks)
    size_t free_b = 0, total_b = 0;
    HIP_CHECK(hipMemGetInfo(&free_b, &total_b));
    free_b += pool_idle_bytes();   // idle pooled scratch is free for this purpose
    const size_t scratch_limit = std::clamp(free_b / 4, (size_t)2 << 30, (size_t)48 << 30);
    // First pass: every admissible block with the rank cap kAcaMaxRank.  Second
    // pass: the blocks that reached it while their break-even rank is larger
    // (large, barely admissible blocks, common with a reflective wall, whose
    // two kernel terms add their ranks), again from the start with the cap
    // kAcaRetryRank; only what still reaches its cap is stored dense.
    // Checking aid: RTE_ACA_FIRST_CAP in the environment lowers the first
    // pass's cap (1 .. kAcaMaxRank), so that small problems exercise the
    // second pass; the stored operator does not depend on it.
    int64_t first_cap = kAcaMaxRank;
    if (const char *e = std::getenv("RTE_ACA_FIRST_CAP"))
        first_cap = std::min<int64_t>(kAcaMaxRank, std::max<int64_t>(1, std::atoll(e)));
    std::vector<size_t> todo(nlr), retry;
    for (size_t b = 0; b < nlr; ++b) todo[b] = b;
    for (int pass = 0; pass < 2 && !todo.empty(); ++pass) {
        const int64_t cap = pass == 0 ? first_cap : kAcaRetryRank;
        if (pass == 1) B.aca_retried += (int64_t)todo.size();
        std::vector<AcaTask> tasks;
        std::vector<size_t> ids;
        int64_t uo = 0, vo = 0;
        for (size_t b : todo) {
            const Block &bl = P.lowrank[b];
            const int32_t m = (int32_t)(bl.t1 - bl.t0), n = (int32_t)(bl.s1 - bl.s0);
            const int32_t kcap = (int32_t)std::min<int64_t>((int64_t)m * n / (m + n), cap);
            if (kcap < 1) {
                fallback.push_back(bl);
                continue;
            }
            const int64_t need = (int64_t)kcap * (m + n);
            if (!tasks.empty() && (size_t)(uo + vo + need) * sizeof(T) > scratch_limit) {
                aca_batch<T>(H, B, kap, tasks, ids, uo, vo, fallback, retry, s);
                tasks.clear();
                ids.clear();
                uo = vo = 0;
            }
            tasks.push_back({bl.t0, bl.s0, m, n, kcap, 0, uo, vo});
            ids.push_back(b);
            uo += (int64_t)kcap * m;
            vo += (int64_t)kcap * n;
        }
        if (!tasks.empty()) aca_batch<T>(H, B, kap, tasks, ids, uo, vo, fallback, retry, s);
        todo.swap(retry);
        retry.clear();
    }
    for (size_t b : todo) fallback.push_back(P.lowrank[b]);
    fill_dense_blocks<T>(H, B, kap, fallback, false, s);
}

template <typename T>
void assemble_typed(HMat &H, int band, BandKappa<T> kap, hipStream_t s) {
    BandStore &B = H.bands[band];
    fill_dense_blocks<T>(H, B, kap, H.plan->dense, H.kind == RTE_VOLUME, s);
    run_aca<T>(H, B, kap, s);
}

}  // namespace

void assemble_band(HMat &H, int band, const double *kappa_band, hipStream_t s) {
    // the band's kappa buffers go to B.retire only after every launch reading
    // them is queued (band_settle, which an ACA batch may call, releases what
    // B.retire holds)
    BandStore &B = H.bands[band];
    if (H.precision == RTE_FP64) {
        DevBuf kt = tet_table<double>(*H.mesh, kappa_band, s);
        assemble_typed<double>(H, band, BandKappa<double>{kappa_band, kt.as<double>()}, s);
        B.retire.push_back(std::move(kt));
    } else {
        DevBuf kf = DevBuf::scratch(sizeof(float) * (size_t)H.mesh->N);
        to_float(kappa_band, kf.as<float>(), H.mesh->N, s);
        DevBuf kt = tet_table<float>(*H.mesh, kf.as<float>(), s);
        assemble_typed<float>(H, band, BandKappa<float>{kf.as<float>(), kt.as<float>()}, s);
        B.retire.push_back(std::move(kf));
        B.retire.push_back(std::move(kt));
    }
}

void band_settle(BandStore &B, hipStream_t s) {
    HIP_CHECK(hipStreamSynchronize(s));
    for (const EventPair &e : B.fill_events) {
        float ms = 0.0f;
        HIP_CHECK(hipEventElapsedTime(&ms, e.a, e.b));
        B.fill_ms += ms;
    }
    B.fill_events.clear();
    for (DevBuf &d : B.retire) d.settled = true;   // the stream has drained: pooled scratch may be reused
    B.retire.clear();
}

}  // namespace rte
