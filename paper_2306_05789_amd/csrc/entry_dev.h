// Device evaluation of the kernel entries of the P1 collocation.
//
// Volume entry (Section "FEM discretization", with the Corollary's mirror term):
//   G^{ij} = exp(-tau(x_i,x_j)) g(x_i, j) + R exp(-tau_bar(x_i,x_j)) g(x_bar_i, j)
//   g(x, j) = |e|/(4 pi) sum_{e ni j} sum_q w_q kappa(y_q) lambda_j(y_q) / |x - y_q|^2
// Surface entry (eq. SE1 and its mirror, Proposition 2):
//   S^{il}  = exp(-tau(x_i,x_l)) s(x_i, l) + R exp(-tau_bar(x_i,x_l)) s(x_bar_i, l)
//   s(x, l) = |t|/(4 pi) sum_{t ni l} sum_q w_q lambda_l(y_q) |(x - y_q).n| / |x - y_q|^3
// with the coplanar limit theta_F/(4 pi) on the diagonal.  tau is the exact
// line integral of the P1 kappa, tau_bar the same along the path reflected
// at the wall.  One optical depth per vertex pair; near rule (degree 5)
// when the grid Chebyshev distance is <= 2, degree 2 otherwise.
//
// tau is computed by a march over the six plane families that bound the
// Kuhn tetrahedra (x_a = const and x_a - x_b = const in grid units): the
// next crossing of every family is kept, the smallest one ends the current
// piece, and kappa is linear on each piece, so the piece contributes its
// length times kappa at its midpoint.
#pragma once

#include <type_traits>
#include <utility>

#include "rte_internal.h"

namespace rte {

template <typename T>
struct EntryCtx {
    GridDev g;
    const T *__restrict__ kappa;   // [N] P1 vertex values of one band
    const T *__restrict__ ktet;    // the march's table of kappa (k_tet_table): FP32 [N][6][4], per cell
                                   // base and Kuhn tetrahedron its four vertex values; FP64 [N][8], per
                                   // cell base its eight corner values
    StencilDev<T> st;
    const T *__restrict__ near;    // quadrature tables of the mesh: near [125][8][8], then far [24][4][8]
};

// ---------------------------------------------------------------- compile-time Kuhn star
struct TetInfo { int slot[4]; int bits; };
struct TriInfo { int ob, oc; };

struct KuhnStar {
    TetInfo tet[kTets];
    TriInfo tri[kTris];
};

// Same enumeration as the host stencil tables: cell corner bits o (cell = j - o),
// then the axis orders in lexicographic order; keep the tetrahedra that contain j.
constexpr KuhnStar make_star() {
    KuhnStar S{};
    const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int n = 0;
    for (int bits = 0; bits < 8; ++bits) {
        int o[3] = {bits & 1, (bits >> 1) & 1, (bits >> 2) & 1};
        for (int p = 0; p < 6; ++p) {
            int w[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {1, 1, 1}};
            w[1][perm[p][0]] = 1;
            w[2][perm[p][0]] = 1;
            w[2][perm[p][1]] = 1;
            bool has = false;
            for (int k = 0; k < 4; ++k)
                if (w[k][0] == o[0] && w[k][1] == o[1] && w[k][2] == o[2]) has = true;
            if (!has) continue;
            for (int k = 0; k < 4; ++k)
                S.tet[n].slot[k] = (w[k][0] - o[0] + 1) * 9 + (w[k][1] - o[1] + 1) * 3 + (w[k][2] - o[2] + 1);
            S.tet[n].bits = bits;
            ++n;
        }
    }
    const int corners[2][3][2] = {{{0, 0}, {1, 0}, {1, 1}}, {{0, 0}, {0, 1}, {1, 1}}};
    int m = 0;
    for (int ob = 0; ob < 2; ++ob)
        for (int oc = 0; oc < 2; ++oc)
            for (int t = 0; t < 2; ++t) {
                bool has = false;
                for (int k = 0; k < 3; ++k)
                    if (corners[t][k][0] == ob && corners[t][k][1] == oc) has = true;
                if (!has) continue;
                S.tri[m].ob = ob;
                S.tri[m].oc = oc;
                ++m;
            }
    return S;
}

constexpr KuhnStar kStar = make_star();

// ---------------------------------------------------------------- P1 kappa and the march
// Minimum of two finite values without the quieting of signalling NaNs that
// fmin() adds on this target (two extra instructions per call in the march).
__device__ __forceinline__ double fmin_finite(double a, double b) {
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ float fmin_finite(float a, float b) {
    float r;
    asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}


// The four vertex values of the Kuhn tetrahedron of a point in the cell with
// flat base index b, at local coordinates (u0, u1, u2) in [0, 1]^3 (grid
// units), and the coordinates sorted decreasingly: kappa there is the P1
// (Freudenthal) interpolant kb + u0 (k1 - kb) + u1 (k2 - k1) + u2 (k3 - k2).
template <typename T>
struct TetSample {
    T kb, k1, k2, k3, u0, u1, u2;
    __device__ __forceinline__ T value() const { return kb + u0 * (k1 - kb) + u1 * (k2 - k1) + u2 * (k3 - k2); }
};

// The Kuhn tetrahedron of the point is given by the decreasing order of its
// local coordinates: from the base corner it adds the axis of the largest
// coordinate, then that of the middle one.  Ties pick the lowest axis as the
// largest and the highest axis as the smallest, so the two never coincide
// (the value is continuous across the faces the ties lie on).
//
// The vertices are b, b + s_L, b + s0 + s1 + 1 - s_S and b + s0 + s1 + 1 (s_a
// the axis strides, L and S the largest and smallest axes).  src is what the
// march reads kappa from (KappaSrc<T>):
//   FP32: the table of every (cell base, tetrahedron) pair, the tetrahedron
//   numbered t = 2 L + (S > L ? S - 1 : S): one 16-byte load per piece
//   instead of four gathers over the grid (the ACA entry launches of the 41^3
//   operator 98.6 -> 78.0 ms).  A base outside the grid (only the unused
//   sample after a segment's last piece, or a piece of rounding length) reads
//   the nearest row.
//   FP64: the table of the eight corner values of every cell base, in the
//   order k(b), k(b + s0 + s1 + 1), then b + s0, b + s1, b + 1, b + s0 + s1,
//   b + s1 + 1, b + s0 + 1: three loads from one 64-byte row per piece (the
//   first two values together).  In FP64 this runs as fast as four gathers
//   over the grid and as 32-byte rows per tetrahedron (41^3: 123 ms of entry
//   launches either way): a lane needs more than one load there whatever the
//   layout.
template <typename T>
struct KappaSrc {
    const T *__restrict__ tab;   // FP32 [N][6][4], FP64 [N][8]
};
template <typename T>
__device__ __forceinline__ KappaSrc<T> kappa_src(const T *tab) {
    return {tab};
}

template <typename T>
__device__ __forceinline__ TetSample<T> tet_sample(const GridDev &g, const KappaSrc<T> &src, int b, T u0, T u1,
                                                   T u2) {
    const bool c01 = u0 >= u1, c02 = u0 >= u2, c12 = u1 >= u2;
    const T hi = fmax(fmax(u0, u1), u2), lo = fmin(fmin(u0, u1), u2);
    const T mid = fmax(fmin(u0, u1), fmin(fmax(u0, u1), u2));
    if constexpr (sizeof(T) == 4) {
        const int L = (c01 && c02) ? 0 : (c12 ? 1 : 2);
        const int S = (c02 && c12) ? 2 : (c01 ? 1 : 0);
        const int t = 2 * L + (S > L ? S - 1 : S);
        const int nv = g.n[0] * g.n[1] * g.n[2];
        const int bc = min(max(b, 0), nv - 1);
        const float4 q = *reinterpret_cast<const float4 *>(src.tab + ((int64_t)bc * 6 + t) * 4);
        return {q.x, q.y, q.z, q.w, hi, mid, lo};
    } else {
        // row slots: v1 = b + s_L at 2 + L; v2 = b + s0 + s1 + 1 - s_S at 6, 7, 5 for S = 0, 1, 2
        const int i1 = (c01 && c02) ? 2 : (c12 ? 3 : 4);
        const int i2 = (c02 && c12) ? 5 : (c01 ? 7 : 6);
        const int nv = g.n[0] * g.n[1] * g.n[2];
        const int bc = min(max(b, 0), nv - 1);
        const double *r = src.tab + (int64_t)bc * 8;
        const double2 q = *reinterpret_cast<const double2 *>(r);
        return {q.x, r[i1], r[i2], q.y, hi, mid, lo};
    }
}

// The state of the march along one segment: start() sets it up for P -> Q
// and samples the tetrahedron of its first piece; piece() moves the families
// crossed at the end of the current piece on, samples the next piece's
// tetrahedron into nxt (its loads run while this piece is added) and adds the
// current one, true once that piece ends the segment; tau() is the optical
// depth.
template <typename T>
struct March {
    T D[3], tn[6], dt[6], w[3], ws[3];
    T len, tp, t, acc;
    int b, db[3];

    __device__ __forceinline__ T next_end() const {
        return fmin_finite(fmin_finite(fmin_finite(tn[0], tn[1]), fmin_finite(tn[2], tn[3])),
                           fmin_finite(fmin_finite(tn[4], tn[5]), (T)1));
    }

    // false when the segment has zero length (tau = 0, nothing sampled)
    __device__ __forceinline__ bool start(const GridDev &g, const KappaSrc<T> &kt, const T P[3], const T Q[3],
                                          TetSample<T> &first) {
#pragma unroll
        for (int a = 0; a < 3; ++a) D[a] = Q[a] - P[a];
        const T wx = D[0] * (T)g.h[0], wy = D[1] * (T)g.h[1], wz = D[2] * (T)g.h[2];
        len = sqrt(wx * wx + wy * wy + wz * wz);
        if (len == (T)0) return false;
        const T F0[6] = {P[0], P[1], P[2], P[0] - P[1], P[1] - P[2], P[0] - P[2]};
        const T dF[6] = {D[0], D[1], D[2], D[0] - D[1], D[1] - D[2], D[0] - D[2]};
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            if (dF[f] != (T)0) {
                const T next = dF[f] > (T)0 ? floor(F0[f]) + (T)1 : ceil(F0[f]) - (T)1;
                dt[f] = (T)1 / fabs(dF[f]);
                tn[f] = (next - F0[f]) / dF[f];
            } else {
                dt[f] = (T)0;
                tn[f] = (T)2;   // never before the end of the segment
            }
        }
        // cell of the first piece: along a, the one the segment enters from P
        // (the top cell when the segment lies in the top plane of a)
        b = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int sa = D[a] > (T)0 ? 1 : (D[a] < (T)0 ? -1 : 0);
            int ca = D[a] < (T)0 ? (int)ceil(P[a]) - 1 : (int)floor(P[a]);
            ca = min(max(ca, 0), g.n[a] - 2);
            b += ca * g.stride[a];
            db[a] = sa * g.stride[a];
            w[a] = P[a] - (T)ca;
            ws[a] = (T)sa;
        }
        tp = (T)0;
        t = next_end();
        acc = (T)0;
        const T tm0 = (T)0.5 * t;
        first = tet_sample(g, kt, b, w[0] + tm0 * D[0], w[1] + tm0 * D[1], w[2] + tm0 * D[2]);
        return true;
    }

    __device__ __forceinline__ bool piece(const GridDev &g, const KappaSrc<T> &kt, const TetSample<T> &cur,
                                          TetSample<T> &nxt) {
        const bool last = t >= (T)1;
#pragma unroll
        for (int f = 0; f < 3; ++f)
            if (tn[f] <= t) {
                tn[f] += dt[f];
                b += db[f];
                w[f] -= ws[f];
            }
#pragma unroll
        for (int f = 3; f < 6; ++f)
            if (tn[f] <= t) tn[f] += dt[f];
        const T tq = next_end();
        const T tm = (T)0.5 * (t + tq);
        nxt = tet_sample(g, kt, b, w[0] + tm * D[0], w[1] + tm * D[1], w[2] + tm * D[2]);
        acc += (t - tp) * cur.value();
        tp = t;
        t = tq;
        return last;
    }

    __device__ __forceinline__ T tau() const { return len * acc; }
};

// every piece advances at least one family: a segment has at most
// sum_f |dF_f| + 7 <= 3 (|D0|+|D1|+|D2|) + 7 pieces
__device__ __forceinline__ int march_cap(const GridDev &g) { return 3 * (g.n[0] + g.n[1] + g.n[2]) + 16; }

// tau along the segment P -> Q given in grid coordinates, both in the closed
// box.  The P1 kappa is linear between consecutive crossings of the six plane
// families, so each piece contributes its length times kappa at its midpoint
// (exact).  The next crossing time of family f advances by the constant
// 1/|dF_f| per crossing; a crossing of family a (a < 3) moves the cell by one
// along axis a, which updates its flat index and P's coordinates relative to
// the cell corner.  Only the last crossing of a family can be taken a few
// rounding units early (the segment ends on a vertex, that is on a plane of
// every family); the piece that follows is of rounding length, and its
// loads stay in bounds through the buffer resource.  The loop is software
// pipelined: the kappa values of the next piece are loaded while the current
// one is added (a piece of zero length, where two families cross together,
// adds zero; after the last piece one more sample is loaded and unused).
template <typename T>
__device__ T tau_segment(const GridDev &g, const KappaSrc<T> &kt, const T P[3], const T Q[3]) {
    March<T> m;
    // two named samples in turn, so that no copy closes the loop
    TetSample<T> sa, sb;
    if (!m.start(g, kt, P, Q, sa)) return (T)0;
    const int cap = march_cap(g);
    for (int it = 0; it < cap; it += 2) {
        if (m.piece(g, kt, sa, sb)) break;
        if (m.piece(g, kt, sb, sa)) break;
    }
    return m.tau();
}

// Wall w's axis, side and coefficient, picked by selects over the constant
// indices: an index into the grid's arrays that is not a compile-time constant
// would copy the whole kernel argument to scratch memory.
struct WallInfo {
    int axis, side;
    double R;
};
__device__ __forceinline__ WallInfo wall_info(const GridDev &g, int w) {
    WallInfo r{g.wall_axis[0], g.wall_side[0], g.R[0]};
#pragma unroll
    for (int k = 1; k < 6; ++k)
        if (w == k) r = WallInfo{g.wall_axis[k], g.wall_side[k], g.R[k]};
    return r;
}

// Optical depth of the path from x (grid coords P) to wall w and on to y (Q),
// the wall point being where the segment from the mirror image of x to y meets it.
template <typename T>
__device__ T tau_mirror(const GridDev &g, int w, const KappaSrc<T> &kt, const T P[3], const T Q[3]) {
    const WallInfo wi = wall_info(g, w);
    const int a = wi.axis;
    const T C = wi.side ? (T)(g.n[a] - 1) : (T)0;
    T Pb[3] = {P[0], P[1], P[2]};
    Pb[a] = (T)2 * C - P[a];
    T X[3];
    const T den = Q[a] - Pb[a];
    if (den == (T)0) {
        X[0] = Q[0]; X[1] = Q[1]; X[2] = Q[2];
    } else {
        const T t = (C - Pb[a]) / den;
#pragma unroll
        for (int b = 0; b < 3; ++b) X[b] = Pb[b] + t * (Q[b] - Pb[b]);
        X[a] = C;
    }
    return tau_segment(g, kt, P, X) + tau_segment(g, kt, X, Q);
}

// grid index of the mirror image of vertex xi in wall w
__device__ __forceinline__ void mirror_index(const GridDev &g, int w, const int xi[3], int mi[3]) {
    const WallInfo wi = wall_info(g, w);
    const int a = wi.axis;
    const int Ci = wi.side ? g.n[a] - 1 : 0;
    mi[0] = xi[0];
    mi[1] = xi[1];
    mi[2] = xi[2];
    mi[a] = 2 * Ci - xi[a];
}

// ---------------------------------------------------------------- the hole (non-convex domain)
// A path is blocked when it runs a positive length through the removed box of
// cells (kappa = +infinity there, Remark rem1) or over a part of a box face
// that the box covers.  Both ends of a segment are grid vertices (integer
// coordinates; a mirror image of one too), so the test is exact: the slab
// method with the parameters of the box planes kept as fractions n / d, d > 0,
// compared by cross multiplication.  An axis open on one side (bit 2a: below,
// 2a+1: above) has no plane there.
__device__ __forceinline__ bool frac_lt(int64_t an, int64_t ad, int64_t bn, int64_t bd) { return an * bd < bn * ad; }

__device__ __forceinline__ bool seg_meets_box(const int P[3], const int Q[3], const int lo[3], const int hi[3],
                                              unsigned open) {
    int64_t t0n = 0, t0d = 1, t1n = 1, t1d = 1;   // the segment's own [0, 1]
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int D = Q[a] - P[a];
        const bool ol = (open >> (2 * a)) & 1u, oh = (open >> (2 * a + 1)) & 1u;
        if (D == 0) {
            if (!((ol || P[a] > lo[a]) && (oh || P[a] < hi[a]))) return false;
            continue;
        }
        const int64_t ad = D > 0 ? D : -D;
        if (D > 0 ? !ol : !oh) {   // enters through the plane below (D > 0) or above
            const int64_t en = D > 0 ? lo[a] - P[a] : P[a] - hi[a];
            if (frac_lt(t0n, t0d, en, ad)) { t0n = en; t0d = ad; }
        }
        if (D > 0 ? !oh : !ol) {   // leaves through the plane above (D > 0) or below
            const int64_t ex = D > 0 ? hi[a] - P[a] : P[a] - lo[a];
            if (frac_lt(ex, ad, t1n, t1d)) { t1n = ex; t1d = ad; }
        }
    }
    return frac_lt(t0n, t0d, t1n, t1d);
}

// the straight path between grid vertices P and Q crosses the hole
__device__ __forceinline__ bool hole_blocks(const GridDev &g, const int P[3], const int Q[3]) {
    return seg_meets_box(P, Q, g.hole_lo, g.hole_hi, g.hole_open);
}

// the path from P reflected at wall w to Q crosses the hole.  Unfolded, it is
// the straight segment from P's mirror image to Q; its part beyond the wall
// is the mirror image of the first leg, so the blocking region there is the
// mirror image of the hole.  A hole that reaches the wall merges with its
// image into one box twice as long; otherwise the two boxes are tested apart.
__device__ __forceinline__ bool hole_blocks_mirror(const GridDev &g, int w, const int P[3], const int Q[3]) {
    const WallInfo wi = wall_info(g, w);
    const int a = wi.axis;
    // the wall axis' values by selects (a is not a compile-time constant)
    int Pb[3], lo[3], hi[3], C = 0, la = 0, ha = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        lo[k] = g.hole_lo[k];
        hi[k] = g.hole_hi[k];
        Pb[k] = P[k];
        if (k == a) {
            C = wi.side ? g.n[k] - 1 : 0;
            Pb[k] = 2 * C - P[k];
            la = g.hole_lo[k];
            ha = g.hole_hi[k];
        }
    }
    const unsigned ol = (g.hole_open >> (2 * a)) & 1u, oh = (g.hole_open >> (2 * a + 1)) & 1u;
    const unsigned others = g.hole_open & ~(3u << (2 * a));
    int blo[3], bhi[3];
    if (wi.side == 0 ? ol : oh) {
        // merged: (2C - hi, hi) at the low wall, (lo, 2C - lo) at the high one,
        // unbounded at both ends when the hole also reaches the far face
        const unsigned far = wi.side == 0 ? oh : ol;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            blo[k] = k == a ? (wi.side == 0 ? 2 * C - ha : la) : lo[k];
            bhi[k] = k == a ? (wi.side == 0 ? ha : 2 * C - la) : hi[k];
        }
        return seg_meets_box(Pb, Q, blo, bhi, others | (far ? 3u << (2 * a) : 0u));
    }
    if (seg_meets_box(Pb, Q, lo, hi, g.hole_open)) return true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        blo[k] = k == a ? 2 * C - ha : lo[k];
        bhi[k] = k == a ? 2 * C - la : hi[k];
    }
    return seg_meets_box(Pb, Q, blo, bhi, others | (oh << (2 * a)) | (ol << (2 * a + 1)));
}

// bit o of the 8 cells around vertex v (cell v - o) is set for the hole's cells
__device__ __forceinline__ int hole_cells(const GridDev &g, const int v[3]) {
    int m = 0;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        bool in = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int c = v[a] - ((o >> a) & 1);
            in = in && c >= g.hole_lo[a] && c < g.hole_hi[a];
        }
        m |= in ? (1 << o) : 0;
    }
    return m;
}

// a vertex of the closed domain: one of its cells inside the grid is no hole cell
__device__ __forceinline__ bool vertex_active(const GridDev &g, const int v[3]) {
    if (!g.has_hole) return true;
    int grid = 0;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        bool ok = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int c = v[a] - ((o >> a) & 1);
            ok = ok && c >= 0 && c <= g.n[a] - 2;
        }
        grid |= ok ? (1 << o) : 0;
    }
    return (grid & ~hole_cells(g, v)) != 0;
}

__device__ __forceinline__ int cheb3(const int a[3], const int b[3]) {
    return max(max(abs(a[0] - b[0]), abs(a[1] - b[1])), abs(a[2] - b[2]));
}

// grid index of vertex v (fewer than 2^28 vertices: 32-bit unsigned division)
__device__ __forceinline__ void vtx_index(const GridDev &g, int64_t v, int idx[3]) {
    const unsigned u = (unsigned)v, s0 = (unsigned)g.stride[0], s1 = (unsigned)g.stride[1];
    const unsigned i0 = u / s0, r = u - i0 * s0, i1 = r / s1;
    idx[0] = (int)i0;
    idx[1] = (int)i1;
    idx[2] = (int)(r - i1 * s1);
}

// ---------------------------------------------------------------- quadrature helpers
// 1/x for the positive, normal distances of the quadrature: the hardware
// reciprocal refined by two Newton steps (FP64: the seed's relative error e
// becomes e^4, below one ulp), or the hardware reciprocal alone (FP32, one
// ulp): cheaper than the IEEE division sequence.
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    r = fma(fma(-x, r, 1.0), r, r);
    return r;
}
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// ---------------------------------------------------------------- volume quadrature
// Near field (grid offset d = x - x_j with |d_a| <= 2): the degree-5 rule's
// sums, tabulated per mesh by cell and corner, so g is 64 products with the
// star's kappa values (cells outside the grid skipped).
template <typename T>
__device__ __forceinline__ T vol_near(const T *__restrict__ tab, const T kn[27], int cellmask, const int d[3]) {
    const T *row = tab + ((d[0] + 2) * 25 + (d[1] + 2) * 5 + (d[2] + 2)) * 64;
    T acc = (T)0;
#pragma unroll
    for (int bits = 0; bits < 8; ++bits) {
        if (!((cellmask >> bits) & 1)) continue;
        const int o0 = bits & 1, o1 = (bits >> 1) & 1, o2 = (bits >> 2) & 1;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int slot = ((e & 1) - o0 + 1) * 9 + (((e >> 1) & 1) - o1 + 1) * 3 + (((e >> 2) & 1) - o2 + 1);
            acc += row[bits * 8 + e] * kn[slot];
        }
    }
    return acc;
}

// Far field, one tetrahedron of the star: its 4 points' terms a_q / r_q added
// over a common denominator, so one reciprocal serves the 4 points.
template <typename T, int t>
__device__ __forceinline__ void vol_far_tet(const T *__restrict__ ft, const T kn[27], int cellmask, T D2,
                                            const T dg[3], T &acc) {
    constexpr TetInfo ti = kStar.tet[t];
    if (!((cellmask >> ti.bits) & 1)) return;
    const T k0 = kn[ti.slot[0]], k1 = kn[ti.slot[1]], k2 = kn[ti.slot[2]], k3 = kn[ti.slot[3]];
    const T *e = ft + t * 32;
    T a[4], r[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        r[q] = D2 + e[8 * q + 3] + e[8 * q + 0] * dg[0] + e[8 * q + 1] * dg[1] + e[8 * q + 2] * dg[2];
        a[q] = e[8 * q + 4] * k0 + e[8 * q + 5] * k1 + e[8 * q + 6] * k2 + e[8 * q + 7] * k3;
    }
    const T n01 = a[0] * r[1] + a[1] * r[0], d01 = r[0] * r[1];
    const T n23 = a[2] * r[3] + a[3] * r[2], d23 = r[2] * r[3];
    acc += (n01 * d23 + n23 * d01) * recip(d01 * d23);
}

template <typename T, int... ts>
__device__ __forceinline__ T vol_far_all(std::integer_sequence<int, ts...>, const T *__restrict__ ft, const T kn[27],
                                         int cellmask, T D2, const T dg[3]) {
    T acc = (T)0;
    (vol_far_tet<T, ts>(ft, kn, cellmask, D2, dg, acc), ...);
    return acc;
}

// g(x, j) without the 1/(4 pi)|e| factor; d = (x - x_j) in grid units
template <typename T>
__device__ __forceinline__ T vol_quad(const EntryCtx<T> &c, const T kn[27], int cellmask, const int d[3],
                                      const T h2[3], bool near) {
    if (near) return vol_near(c.near, kn, cellmask, d);
    const T dg[3] = {(T)d[0], (T)d[1], (T)d[2]};
    const T D2 = h2[0] * dg[0] * dg[0] + h2[1] * dg[1] * dg[1] + h2[2] * dg[2] * dg[2];
    return vol_far_all<T>(std::make_integer_sequence<int, kTets>{}, c.near + kNearSize, kn, cellmask, D2, dg);
}

template <typename T>
__device__ __forceinline__ void load_star(const EntryCtx<T> &c, const int jj[3], T kn[27], int &cellmask) {
    const GridDev &g = c.g;
    cellmask = 0;
#pragma unroll
    for (int bits = 0; bits < 8; ++bits) {
        bool ok = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int o = (bits >> a) & 1;
            ok = ok && (o ? jj[a] >= 1 : jj[a] <= g.n[a] - 2);
        }
        cellmask |= ok ? (1 << bits) : 0;
    }
#pragma unroll
    for (int s = 0; s < 27; ++s) {
        const int dx = s / 9 - 1, dy = (s / 3) % 3 - 1, dz = s % 3 - 1;
        const int x = min(max(jj[0] + dx, 0), g.n[0] - 1);
        const int y = min(max(jj[1] + dy, 0), g.n[1] - 1);
        const int z = min(max(jj[2] + dz, 0), g.n[2] - 1);
        kn[s] = c.kappa[x * g.stride[0] + y * g.stride[1] + z];
    }
}

// Wall modes the entry code is compiled for: no wall, exactly one wall (the
// common reflective case, kept as straight-line code), or the general mode:
// any number of walls read from the grid (a loop; its per-wall attenuations go
// through a small array in scratch memory) and the hole of a non-convex domain.
constexpr int kNoWall = 0, kOneWall = 1, kAnyWalls = 6;
inline int wall_mode(const GridDev &g) {
    return (g.has_hole || g.n_walls > 1) ? kAnyWalls : (g.n_walls == 0 ? kNoWall : kOneWall);
}

// sum over the direct path and the walls of attenuation times the quadrature
// of the source star of ss seen from target tt (or from its mirror image in
// each wall); att_w[w] = R_w exp(-tau_w)
template <typename T, int NW>
__device__ __forceinline__ T vol_sum(const EntryCtx<T> &c, T att, const T att_w[6], const int tt[3],
                                     const int ss[3]) {
    const GridDev &g = c.g;
    const T h2[3] = {(T)(g.h[0] * g.h[0]), (T)(g.h[1] * g.h[1]), (T)(g.h[2] * g.h[2])};
    T kn[27];
    int cellmask;
    load_star(c, ss, kn, cellmask);
    if constexpr (NW == kAnyWalls)
        if (g.has_hole) cellmask &= ~hole_cells(g, ss);   // the hole's cells are in no star
    const int dg[3] = {tt[0] - ss[0], tt[1] - ss[1], tt[2] - ss[2]};
    T G = att * vol_quad(c, kn, cellmask, dg, h2, cheb3(tt, ss) <= kNearCheb);
    if constexpr (NW != kNoWall) {
        const int nw = NW == kOneWall ? 1 : g.n_walls;
        for (int w = 0; w < nw; ++w) {
            int mt[3];
            mirror_index(g, w, tt, mt);
            const int dgm[3] = {mt[0] - ss[0], mt[1] - ss[1], mt[2] - ss[2]};
            G += att_w[w] * vol_quad(c, kn, cellmask, dgm, h2, cheb3(mt, ss) <= kNearCheb);
        }
    }
    return G * (T)g.vol_scale;
}

// The optical depths of a pair: direct, and R_w exp(-tau_w) per wall; a path
// that the hole blocks has tau = +infinity (no march).  Pi, Qi: the vertices'
// grid indices, P, Q the same as reals.
template <typename T, int NW>
__device__ __forceinline__ T attenuations(const GridDev &g, const KappaSrc<T> &kt, const int Pi[3],
                                          const int Qi[3], const T P[3], const T Q[3], T att_w[6]) {
    if constexpr (NW == kAnyWalls) {
        const bool hole = g.has_hole;
        const T att = (hole && hole_blocks(g, Pi, Qi)) ? (T)0 : exp(-tau_segment(g, kt, P, Q));
        for (int w = 0; w < g.n_walls; ++w)
            att_w[w] = (hole && hole_blocks_mirror(g, w, Pi, Qi))
                           ? (T)0
                           : (T)wall_info(g, w).R * exp(-tau_mirror(g, w, kt, P, Q));
        return att;
    } else {
        const T att = exp(-tau_segment(g, kt, P, Q));
        if constexpr (NW == kOneWall) att_w[0] = (T)g.R[0] * exp(-tau_mirror(g, 0, kt, P, Q));
        return att;
    }
}

// G(i, j).  Every wall adds its own mirror-image term (one reflection per
// ray).  The optical depths come first: the star of j is loaded after the
// marches, so its 27 values do not stay live through them.
template <typename T, int NW = kAnyWalls>
__device__ T volume_entry(const EntryCtx<T> &c, int64_t i, int64_t j) {
    const GridDev &g = c.g;
    int ii[3], jj[3];
    vtx_index(g, i, ii);
    vtx_index(g, j, jj);
    if constexpr (NW == kAnyWalls)
        if (!vertex_active(g, ii)) return (T)0;   // a removed vertex (its column: an empty star)
    const T P[3] = {(T)ii[0], (T)ii[1], (T)ii[2]};
    const T Q[3] = {(T)jj[0], (T)jj[1], (T)jj[2]};
    T att_w[6];
    const T att = attenuations<T, NW>(g, kappa_src(c.ktet), ii, jj, P, Q, att_w);
    return vol_sum<T, NW>(c, att, att_w, ii, jj);
}

// G(i, j) and G(j, i) together: the optical depth along the segment (and along
// each reflected path, whose wall point is the same seen from either end) is
// shared; each entry takes its own source star and quadrature.
template <typename T, int NW = kAnyWalls>
__device__ __forceinline__ void volume_entry_pair(const EntryCtx<T> &c, int64_t i, int64_t j, T &gij, T &gji) {
    const GridDev &g = c.g;
    int ii[3], jj[3];
    vtx_index(g, i, ii);
    vtx_index(g, j, jj);
    const T P[3] = {(T)ii[0], (T)ii[1], (T)ii[2]};
    const T Q[3] = {(T)jj[0], (T)jj[1], (T)jj[2]};
    T att_w[6];
    const T att = attenuations<T, NW>(g, kappa_src(c.ktet), ii, jj, P, Q, att_w);
    gij = vol_sum<T, NW>(c, att, att_w, ii, jj);
    gji = vol_sum<T, NW>(c, att, att_w, jj, ii);
    if constexpr (NW == kAnyWalls) {   // removed vertices have zero rows
        if (!vertex_active(g, ii)) gij = (T)0;
        if (!vertex_active(g, jj)) gji = (T)0;
    }
}

// ---------------------------------------------------------------- surface quadrature
// The wall kernel without its normal-distance factor: 1 / r^3 for the
// isotropic source (eq. SE1, times |d|), 1 / r^4 for the cosine-weighted one
// of Section "Example" (C2, times d^2).
template <typename T, bool C2>
__device__ __forceinline__ T wall_kernel(T r2) {
    if constexpr (C2) return recip(r2 * r2);
    else return recip(r2 * sqrt(r2));
}

template <typename T, int NQ, bool C2, int t>
__device__ __forceinline__ void tri_term(const T *__restrict__ tab, const int lb, const int lc, const int nb,
                                         const int nc, const T db, const T dc, const T da2, const T hb2,
                                         const T hc2, T &acc) {
    constexpr TriInfo ti = kStar.tri[t];
    const int sb = lb - ti.ob, sc = lc - ti.oc;
    if (sb < 0 || sb > nb - 2 || sc < 0 || sc > nc - 2) return;
    const T *e = tab + t * NQ * 4;
    T s = (T)0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const T eb = db - e[4 * q + 0], ec = dc - e[4 * q + 1];
        const T r2 = da2 + hb2 * eb * eb + hc2 * ec * ec;
        s += e[4 * q + 2] * wall_kernel<T, C2>(r2);
    }
    acc += s;
}

template <typename T, int NQ, bool C2, int... ts>
__device__ __forceinline__ T tri_all(std::integer_sequence<int, ts...>, const T *__restrict__ tab, int lb, int lc,
                                     int nb, int nc, T db, T dc, T da2, T hb2, T hc2) {
    T acc = (T)0;
    (tri_term<T, NQ, C2, ts>(tab, lb, lc, nb, nc, db, dc, da2, hb2, hc2, acc), ...);
    return acc;
}

// s(x, l) including 1/(4 pi) and the element areas; x given by its grid
// coordinates (possibly outside the box for a mirror image) and index.
template <typename T>
__device__ T surf_quad(const EntryCtx<T> &c, const int xi[3], const int ll[3], bool near) {
    const GridDev &g = c.g;
    T acc = (T)0;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        if (!((g.emit_faces >> f) & 1u)) continue;
        const int a = f / 2;
        const int pf = (f & 1) ? g.n[a] - 1 : 0;
        if (ll[a] != pf) continue;
        const int b = (a == 0) ? 1 : 0;
        const int cc = (a == 2) ? 1 : 2;
        if (xi[a] == pf) {
            // coplanar limit: theta_F(x)/(4 pi) on the diagonal (isotropic), half
            // that for the cosine-weighted source
            if (xi[0] == ll[0] && xi[1] == ll[1] && xi[2] == ll[2]) {
                T frac = (T)1;
                const int axes[2] = {b, cc};
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const int p = xi[axes[k]];
                    if (p < 0 || p > g.n[axes[k]] - 1) frac = (T)0;
                    else if (p == 0 || p == g.n[axes[k]] - 1) frac *= (T)0.5;
                }
                acc += (g.emission ? (T)0.25 : (T)0.5) * frac;
            }
            continue;
        }
        const T da = (T)(xi[a] - pf) * (T)g.h[a];
        const T da2 = da * da;
        const T hb2 = (T)(g.h[b] * g.h[b]), hc2 = (T)(g.h[cc] * g.h[cc]);
        const T db = (T)(xi[b] - ll[b]), dc = (T)(xi[cc] - ll[cc]);
        constexpr auto seq = std::make_integer_sequence<int, kTris>{};
        T s;
        if (g.emission) {
            s = near ? tri_all<T, 7, true>(seq, c.st.tri_near, ll[b], ll[cc], g.n[b], g.n[cc], db, dc, da2, hb2, hc2)
                     : tri_all<T, 3, true>(seq, c.st.tri_far, ll[b], ll[cc], g.n[b], g.n[cc], db, dc, da2, hb2, hc2);
            s *= da2;
        } else {
            s = near ? tri_all<T, 7, false>(seq, c.st.tri_near, ll[b], ll[cc], g.n[b], g.n[cc], db, dc, da2, hb2, hc2)
                     : tri_all<T, 3, false>(seq, c.st.tri_far, ll[b], ll[cc], g.n[b], g.n[cc], db, dc, da2, hb2, hc2);
            s *= fabs(da);
        }
        acc += s * (T)g.area_scale[a];
    }
    return acc;
}

// The general mode's surface quadrature: the emitting rectangles are the
// emitting box faces (f < 6) and the hole's emitting faces (f >= 6); a square
// emits when it lies in its rectangle and the cell it bounds on the domain
// side is no hole cell (bit ob + 2 oc of sqmask: the square l - (ob, oc)).  A
// rectangle seen from behind adds nothing; on the diagonal in the rectangle's
// plane the planar angle of the emitting squares, pi/2 each, over 4 pi.  For
// the box faces of a mesh without a hole this is surf_quad, term for term.
template <typename T, int NQ, bool C2, int t>
__device__ __forceinline__ void tri_term_m(const T *__restrict__ tab, int sqmask, const T db, const T dc, const T da2,
                                           const T hb2, const T hc2, T &acc) {
    constexpr TriInfo ti = kStar.tri[t];
    if (!((sqmask >> (ti.ob + 2 * ti.oc)) & 1)) return;
    const T *e = tab + t * NQ * 4;
    T s = (T)0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const T eb = db - e[4 * q + 0], ec = dc - e[4 * q + 1];
        const T r2 = da2 + hb2 * eb * eb + hc2 * ec * ec;
        s += e[4 * q + 2] * wall_kernel<T, C2>(r2);
    }
    acc += s;
}

template <typename T, int NQ, bool C2, int... ts>
__device__ __forceinline__ T tri_all_m(std::integer_sequence<int, ts...>, const T *__restrict__ tab, int sqmask, T db,
                                       T dc, T da2, T hb2, T hc2) {
    T acc = (T)0;
    (tri_term_m<T, NQ, C2, ts>(tab, sqmask, db, dc, da2, hb2, hc2, acc), ...);
    return acc;
}

template <typename T>
__device__ T surf_quad_rects(const EntryCtx<T> &c, const int xi[3], const int ll[3], bool near) {
    const GridDev &g = c.g;
    T acc = (T)0;
    for (int f = 0; f < 12; ++f) {
        const bool box = f < 6;
        const int fb = box ? f : f - 6;
        if (!(((box ? g.emit_faces : g.hole_emit) >> fb) & 1u)) continue;
        const int a = fb / 2, hi_side = fb & 1;
        const int b = (a == 0) ? 1 : 0;
        const int cc = (a == 2) ? 1 : 2;
        // the rectangle's plane, inward normal sign and square ranges [lo, hi), by selects
        int pf = 0, rlo[2] = {0, 0}, rhi[2] = {0, 0};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int lo_k = box ? 0 : g.hole_lo[k], hi_k = box ? g.n[k] - 1 : g.hole_hi[k];
            if (k == a) pf = hi_side ? hi_k : lo_k;
            if (k == b) { rlo[0] = lo_k; rhi[0] = hi_k; }
            if (k == cc) { rlo[1] = lo_k; rhi[1] = hi_k; }
        }
        const int sign = box ? (hi_side ? -1 : 1) : (hi_side ? 1 : -1);
        if (ll[a] != pf) continue;
        int sqmask = 0;
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const int sb = ll[b] - (o & 1), sc = ll[cc] - (o >> 1);
            if (sb < rlo[0] || sb >= rhi[0] || sc < rlo[1] || sc >= rhi[1]) continue;
            bool covered = false;
            if (box && g.has_hole) {
                int cell[3];
                cell[0] = a == 0 ? (sign > 0 ? pf : pf - 1) : (b == 0 ? sb : sc);
                cell[1] = a == 1 ? (sign > 0 ? pf : pf - 1) : (b == 1 ? sb : sc);
                cell[2] = a == 2 ? (sign > 0 ? pf : pf - 1) : sc;
                covered = cell[0] >= g.hole_lo[0] && cell[0] < g.hole_hi[0] && cell[1] >= g.hole_lo[1] &&
                          cell[1] < g.hole_hi[1] && cell[2] >= g.hole_lo[2] && cell[2] < g.hole_hi[2];
            }
            sqmask |= covered ? 0 : (1 << o);
        }
        if (xi[a] == pf) {
            // coplanar limit: theta(x)/(4 pi) on the diagonal, pi/2 per emitting square
            // (isotropic), half that for the cosine-weighted source
            if (xi[0] == ll[0] && xi[1] == ll[1] && xi[2] == ll[2])
                acc += (g.emission ? (T)0.0625 : (T)0.125) * (T)__builtin_popcount(sqmask);
            continue;
        }
        const int d = (xi[a] - pf) * sign;
        if (d <= 0) continue;
        T ha = (T)0, hb2 = (T)0, hc2 = (T)0, as = (T)0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (k == a) { ha = (T)g.h[k]; as = (T)g.area_scale[k]; }
            if (k == b) hb2 = (T)(g.h[k] * g.h[k]);
            if (k == cc) hc2 = (T)(g.h[k] * g.h[k]);
        }
        const T da = (T)d * ha;
        const T da2 = da * da;
        const T db = (T)(xi[b] - ll[b]), dc = (T)(xi[cc] - ll[cc]);
        constexpr auto seq = std::make_integer_sequence<int, kTris>{};
        T s;
        if (g.emission) {
            s = near ? tri_all_m<T, 7, true>(seq, c.st.tri_near, sqmask, db, dc, da2, hb2, hc2)
                     : tri_all_m<T, 3, true>(seq, c.st.tri_far, sqmask, db, dc, da2, hb2, hc2);
            s *= da2;
        } else {
            s = near ? tri_all_m<T, 7, false>(seq, c.st.tri_near, sqmask, db, dc, da2, hb2, hc2)
                     : tri_all_m<T, 3, false>(seq, c.st.tri_far, sqmask, db, dc, da2, hb2, hc2);
            s *= da;
        }
        acc += s * as;
    }
    return acc;
}

template <typename T, int NW = kAnyWalls>
__device__ T surface_entry(const EntryCtx<T> &c, int64_t i, int64_t l) {
    const GridDev &g = c.g;
    int ii[3], ll[3];
    vtx_index(g, i, ii);
    vtx_index(g, l, ll);
    const T P[3] = {(T)ii[0], (T)ii[1], (T)ii[2]};
    const T Q[3] = {(T)ll[0], (T)ll[1], (T)ll[2]};
    if constexpr (NW == kAnyWalls) {
        if (!vertex_active(g, ii)) return (T)0;   // a removed vertex
        T att_w[6];
        const T att = attenuations<T, NW>(g, kappa_src(c.ktet), ii, ll, P, Q, att_w);
        T S = att == (T)0 ? (T)0 : att * surf_quad_rects(c, ii, ll, cheb3(ii, ll) <= kNearCheb);
        for (int w = 0; w < g.n_walls; ++w) {
            if (att_w[w] == (T)0) continue;
            int mi[3];
            mirror_index(g, w, ii, mi);
            S += att_w[w] * surf_quad_rects(c, mi, ll, cheb3(mi, ll) <= kNearCheb);
        }
        return S;
    } else {
        const KappaSrc<T> ks = kappa_src(c.ktet);
        T S = exp(-tau_segment(g, ks, P, Q)) * surf_quad(c, ii, ll, cheb3(ii, ll) <= kNearCheb);
        if constexpr (NW == kOneWall) {
            int mi[3];
            mirror_index(g, 0, ii, mi);
            S += (T)g.R[0] * exp(-tau_mirror(g, 0, ks, P, Q)) * surf_quad(c, mi, ll, cheb3(mi, ll) <= kNearCheb);
        }
        return S;
    }
}

template <typename T, int KIND, int NW = kAnyWalls>
__device__ __forceinline__ T entry(const EntryCtx<T> &c, int64_t i, int64_t j) {
    if constexpr (KIND == RTE_VOLUME) return volume_entry<T, NW>(c, i, j);
    else return surface_entry<T, NW>(c, i, j);
}

}  // namespace rte
