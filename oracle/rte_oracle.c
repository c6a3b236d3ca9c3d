/*
 * FP64 CPU oracle for the kernel entries of the integral-form radiative
 * transfer method with a planar reflective wall (Pironneau & Tournier,
 * arXiv 2306.05789).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is part of the oracle that the tests,
 * the smoke check and the benchmark's CPU-baseline leg use to check the GPU
 * library.  It shares no code with the library, and the library never calls
 * it.  Everything here is plain, slow and written to be read against the paper:
 *
 *   - Integral form, eq. (gen1): the volume kernel is
 *       exp(-int_[x,y] kappa) / (4 pi |x-y|^2),
 *     with int_[x,y] f = |y-x| int_0^1 f(s y + (1-s) x) ds.
 *   - Propositions 1-2 and the Corollary: with a planar reflective wall the
 *     kernel gains R * exp(-int over [x,x'] u [x',y]) / (|x-x'|+|x'-y|)^2,
 *     where x' is where the segment from the mirror image of x to y meets the
 *     wall; for the boundary source the kernel is the solid-angle density
 *     |(x-y).n| / |x-y|^3 (eq. SE1), seen from x and from its mirror image.
 *     With several planar walls (the three planes of the academic test) and at
 *     most one reflection per ray (Hypothesis 1), every wall adds its own
 *     mirror-image term.
 *   - Section "FEM discretization": P1 collocation, G^{ij} integrates
 *     kappa * kernel * w^j over the tetrahedra around vertex j with a
 *     degree-5 (14 point) rule near x^i and degree-2 (4 point) rule
 *     otherwise; the surface matrix replaces Q^0 by the boundary hat w~^l.
 *
 * The mesh is a structured box grid; each cell is split into the six Kuhn
 * tetrahedra that share the cell's (0,0,0)-(1,1,1) diagonal.  For the
 * mirror-doubled domain used as an independent check of the reflective term,
 * cells on one side of a plane may be the mirror images of Kuhn cells.
 *
 * A non-convex domain is the box minus a box of grid cells (the inner cube of
 * the academic test); following Remark rem1 the method is applied to the box
 * with kappa = +infinity in the hole: a segment whose path crosses the hole's
 * interior has an infinite optical depth, the hole's cells are in no vertex's
 * star, and the hole's faces may emit into the domain.
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - one optical depth per vertex pair ("frozen tau"): the quadrature acts on
 *     kappa * w^j / r^2 only, and tau is the exact line integral of the P1
 *     kappa between the two vertices;
 *   - near rule iff the grid-index Chebyshev distance is <= near_cheb (2);
 *   - a target on the plane of an emitting face receives theta_F/(4 pi) from
 *     that face on the diagonal (the coplanar limit of the solid angle);
 *   - kappa(y) multiplies both the direct and the reflected volume terms;
 *   - hole: a segment is blocked only when a positive length of it lies
 *     outside the closed domain: in the hole's open interior or on a part of
 *     a box face the hole covers (one grazing the hole's faces or edges inside
 *     the box is not);
 *     vertices with no non-hole cell have zero rows and columns (for them the
 *     iteration gives J = 0 and T = 0); a face square is emitting when the
 *     cell it bounds on the domain side is no hole cell, and theta_F on the
 *     diagonal is pi/2 per emitting square at the vertex.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n[3];          /* vertex counts per axis */
    double lo[3];          /* box corner */
    double h[3];           /* spacing */
    int32_t flip_axis;     /* -1: plain Kuhn grid; else mirrored cells below flip_cells */
    int32_t flip_cells;
    const double *kappa;   /* [N] P1 vertex values, natural order */
    int32_t n_walls;       /* planar reflective walls, each a whole box face */
    int32_t wall_axis[6];
    int32_t wall_side[6];  /* 0: plane at lo, 1: plane at hi */
    double R[6];           /* reflection coefficients */
    uint32_t emit_faces;   /* bit f: face (axis f/2, side f%2) emits */
    int32_t hole_lo[3];    /* non-convex domain: the box minus the cells [hole_lo, hole_hi), where */
    int32_t hole_hi[3];    /* kappa is +infinity (no hole when hole_lo[0] >= hole_hi[0]) */
    uint32_t hole_emit;    /* bit f: the hole's face on side f%2 of axis f/2 emits into the domain */
    uint32_t emission;     /* 0: isotropic wall, kernel [(x-y).n]_+ / |x-y|^3 (eq. SE1); 1: the Example's
                              Q = [omega.n]_- Q0, kernel ([(x-y).n]_+)^2 / |x-y|^4 */
    int32_t near_cheb;
    int32_t nq_tet_far, nq_tet_near, nq_tri_far, nq_tri_near;
    const double *tet_far_p, *tet_far_w;     /* [nq][4], [nq] */
    const double *tet_near_p, *tet_near_w;
    const double *tri_far_p, *tri_far_w;     /* [nq][3], [nq] */
    const double *tri_near_p, *tri_near_w;
} og_problem_t;

#define OG_PI 3.14159265358979323846

/* ---------------------------------------------------------------- grid */

static int64_t vid(const og_problem_t *P, const int idx[3])
{
    return ((int64_t)idx[0] * P->n[1] + idx[1]) * P->n[2] + idx[2];
}

static void vidx(const og_problem_t *P, int64_t v, int idx[3])
{
    idx[2] = (int)(v % P->n[2]);
    v /= P->n[2];
    idx[1] = (int)(v % P->n[1]);
    idx[0] = (int)(v / P->n[1]);
}

static void vpos(const og_problem_t *P, const int idx[3], double x[3])
{
    for (int a = 0; a < 3; ++a) x[a] = P->lo[a] + idx[a] * P->h[a];
}

static double kap(const og_problem_t *P, const int idx[3]) { return P->kappa[vid(P, idx)]; }

static int has_hole(const og_problem_t *P)
{
    return P->hole_lo[0] < P->hole_hi[0] && P->hole_lo[1] < P->hole_hi[1] && P->hole_lo[2] < P->hole_hi[2];
}

/* is cell c one of the hole's cells */
static int hole_cell(const og_problem_t *P, const int c[3])
{
    if (!has_hole(P)) return 0;
    for (int a = 0; a < 3; ++a)
        if (c[a] < P->hole_lo[a] || c[a] >= P->hole_hi[a]) return 0;
    return 1;
}

/* a vertex belongs to the closed domain when one of its cells is not a hole
 * cell; the others (inside the hole, or on a box face the hole covers) have
 * zero rows and columns */
static int vertex_active(const og_problem_t *P, const int v[3])
{
    if (!has_hole(P)) return 1;
    for (int o = 0; o < 8; ++o) {
        int c[3], ok = 1;
        for (int a = 0; a < 3; ++a) {
            c[a] = v[a] - ((o >> a) & 1);
            if (c[a] < 0 || c[a] > P->n[a] - 2) ok = 0;
        }
        if (ok && !hole_cell(P, c)) return 1;
    }
    return 0;
}

/* is the point X (grid coordinates) outside the closed domain: strictly
 * inside the hole, or on a part of a box face that the hole covers (along an
 * axis where the hole reaches the box face, the open range extends past it) */
static int in_hole(const og_problem_t *P, const double X[3])
{
    if (!has_hole(P)) return 0;
    for (int a = 0; a < 3; ++a) {
        const int open_lo = P->hole_lo[a] == 0, open_hi = P->hole_hi[a] == P->n[a] - 1;
        if (!((open_lo || X[a] > P->hole_lo[a]) && (open_hi || X[a] < P->hole_hi[a]))) return 0;
    }
    return 1;
}

/* The tetrahedron of cell c for axis order sig[]: its vertices are
 * base, base+s0 e_sig0, base+s0 e_sig0+s1 e_sig1, base+s.  For a plain Kuhn cell
 * base = c and every step is +1; in a mirrored cell the flip axis starts at
 * c+1 and steps by -1. */
static void cell_frame(const og_problem_t *P, const int c[3], int base[3], int step[3])
{
    for (int a = 0; a < 3; ++a) {
        base[a] = c[a];
        step[a] = 1;
    }
    if (P->flip_axis >= 0 && c[P->flip_axis] < P->flip_cells) {
        base[P->flip_axis] = c[P->flip_axis] + 1;
        step[P->flip_axis] = -1;
    }
}

static void tet_vertices(const int base[3], const int step[3], const int sig[3], int v[4][3])
{
    for (int a = 0; a < 3; ++a) v[0][a] = base[a];
    for (int a = 0; a < 3; ++a) v[1][a] = v[0][a];
    v[1][sig[0]] += step[sig[0]];
    for (int a = 0; a < 3; ++a) v[2][a] = v[1][a];
    v[2][sig[1]] += step[sig[1]];
    for (int a = 0; a < 3; ++a) v[3][a] = base[a] + step[a];
}

static const int PERMS[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

/* P1 interpolation of kappa at a point (Freudenthal/Kuhn barycentrics). */
double og_kappa_at(const og_problem_t *P, const double x[3])
{
    double X[3], u[3];
    int c[3], base[3], step[3];
    for (int a = 0; a < 3; ++a) {
        X[a] = (x[a] - P->lo[a]) / P->h[a];
        int f = (int)floor(X[a]);
        if (f < 0) f = 0;
        if (f > P->n[a] - 2) f = P->n[a] - 2;
        c[a] = f;
    }
    cell_frame(P, c, base, step);
    for (int a = 0; a < 3; ++a) u[a] = (X[a] - base[a]) * step[a];
    /* axes ordered by decreasing local coordinate */
    int s[3] = {0, 1, 2};
    for (int p = 0; p < 3; ++p)
        for (int q = p + 1; q < 3; ++q)
            if (u[s[q]] > u[s[p]]) {
                int t = s[p];
                s[p] = s[q];
                s[q] = t;
            }
    int v[4][3];
    tet_vertices(base, step, s, v);
    double lam[4] = {1.0 - u[s[0]], u[s[0]] - u[s[1]], u[s[1]] - u[s[2]], u[s[2]]};
    double k = 0.0;
    for (int m = 0; m < 4; ++m) k += lam[m] * kap(P, v[m]);
    return k;
}

/* ---------------------------------------------------------------- optical depth */

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* tau(p,q) = |q-p| * integral over [0,1] of the P1 kappa along the segment.
 * Brute force: every parameter where the segment crosses a plane of a family
 * that bounds the tetrahedra is collected and sorted; kappa is linear between
 * consecutive breakpoints, so the trapezoid rule on those pieces is exact. */
double og_tau(const og_problem_t *P, const double p[3], const double q[3])
{
    double Pg[3], Qg[3], len2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        Pg[a] = (p[a] - P->lo[a]) / P->h[a];
        Qg[a] = (q[a] - P->lo[a]) / P->h[a];
        len2 += (q[a] - p[a]) * (q[a] - p[a]);
    }
    if (len2 == 0.0) return 0.0;
    /* plane families a . X in Z */
    double fam[9][3];
    int nf = 0;
    for (int a = 0; a < 3; ++a) {
        double e[3] = {0, 0, 0};
        e[a] = 1;
        memcpy(fam[nf++], e, sizeof e);
    }
    for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b) {
            double e[3] = {0, 0, 0};
            e[a] = 1;
            e[b] = -1;
            memcpy(fam[nf++], e, sizeof e);
        }
    if (P->flip_axis >= 0)
        for (int b = 0; b < 3; ++b)
            if (b != P->flip_axis) {
                double e[3] = {0, 0, 0};
                e[P->flip_axis] = 1;
                e[b] = 1;
                memcpy(fam[nf++], e, sizeof e);
            }
    size_t cap = 64, cnt = 0;
    for (int f = 0; f < nf; ++f) {
        double F0 = fam[f][0] * Pg[0] + fam[f][1] * Pg[1] + fam[f][2] * Pg[2];
        double F1 = fam[f][0] * Qg[0] + fam[f][1] * Qg[1] + fam[f][2] * Qg[2];
        cap += (size_t)(fabs(F1 - F0) + 2.0);
    }
    double *t = (double *)malloc(cap * sizeof(double));
    t[cnt++] = 0.0;
    for (int f = 0; f < nf; ++f) {
        double F0 = fam[f][0] * Pg[0] + fam[f][1] * Pg[1] + fam[f][2] * Pg[2];
        double F1 = fam[f][0] * Qg[0] + fam[f][1] * Qg[1] + fam[f][2] * Qg[2];
        if (F0 == F1) continue;
        double lo = F0 < F1 ? F0 : F1, hi = F0 < F1 ? F1 : F0;
        for (double m = floor(lo) + 1.0; m < hi; m += 1.0) {
            double tm = (m - F0) / (F1 - F0);
            if (tm > 0.0 && tm < 1.0) t[cnt++] = tm;
        }
    }
    t[cnt++] = 1.0;
    qsort(t, cnt, sizeof(double), cmp_double);
    /* kappa is +infinity in the hole: a piece (the hole's boundary planes are
     * among the breakpoints) whose midpoint lies outside the closed domain
     * blocks the segment.  Pieces of rounding length, where two families
     * cross at the same point, carry no length and are passed over (between
     * grid vertices a piece of positive length is longer than 1/n^2). */
    for (size_t m = 1; m < cnt; ++m) {
        if (t[m] - t[m - 1] <= 1e-12) continue;
        double X[3], tm = 0.5 * (t[m - 1] + t[m]);
        for (int a = 0; a < 3; ++a) X[a] = Pg[a] + tm * (Qg[a] - Pg[a]);
        if (in_hole(P, X)) {
            free(t);
            return INFINITY;
        }
    }
    double sum = 0.0, kprev = 0.0;
    for (size_t m = 0; m < cnt; ++m) {
        double x[3];
        for (int a = 0; a < 3; ++a) x[a] = p[a] + t[m] * (q[a] - p[a]);
        double k = og_kappa_at(P, x);
        if (m > 0) sum += (t[m] - t[m - 1]) * 0.5 * (kprev + k);
        kprev = k;
    }
    free(t);
    return sqrt(len2) * sum;
}

static double wall_plane(const og_problem_t *P, int w)
{
    int a = P->wall_axis[w];
    return P->wall_side[w] == 0 ? P->lo[a] : P->lo[a] + (P->n[a] - 1) * P->h[a];
}

static void mirror_point(const og_problem_t *P, int w, const double x[3], double xb[3])
{
    double c = wall_plane(P, w);
    for (int a = 0; a < 3; ++a) xb[a] = x[a];
    xb[P->wall_axis[w]] = 2.0 * c - x[P->wall_axis[w]];
}

static void mirror_index(const og_problem_t *P, int w, const int idx[3], int mb[3])
{
    int a = P->wall_axis[w];
    for (int b = 0; b < 3; ++b) mb[b] = idx[b];
    mb[a] = P->wall_side[w] == 0 ? -idx[a] : 2 * (P->n[a] - 1) - idx[a];
}

/* Optical depth along the broken path x -> x' -> y, where x' is the point of
 * wall w on the segment from the mirror image of x to y. */
double og_tau_mirror(const og_problem_t *P, int w, const double x[3], const double y[3])
{
    double xb[3], xp[3];
    int a = P->wall_axis[w];
    mirror_point(P, w, x, xb);
    double den = y[a] - xb[a];
    if (den == 0.0) {
        for (int b = 0; b < 3; ++b) xp[b] = y[b];
    } else {
        double t = (wall_plane(P, w) - xb[a]) / den;
        for (int b = 0; b < 3; ++b) xp[b] = xb[b] + t * (y[b] - xb[b]);
        xp[a] = wall_plane(P, w);
    }
    return og_tau(P, x, xp) + og_tau(P, xp, y);
}

/* ---------------------------------------------------------------- entries */

static int cheb(const int a[3], const int b[3])
{
    int m = 0;
    for (int k = 0; k < 3; ++k) {
        int d = abs(a[k] - b[k]);
        if (d > m) m = d;
    }
    return m;
}

/* (1/4pi) sum over tets e around vertex j of |e| sum_q w_q kappa(y_q) lambda_j(y_q) / |x-y_q|^2 */
static double volume_quad(const og_problem_t *P, const double x[3], const int j[3], int near)
{
    int nq = near ? P->nq_tet_near : P->nq_tet_far;
    const double *bp = near ? P->tet_near_p : P->tet_far_p;
    const double *bw = near ? P->tet_near_w : P->tet_far_w;
    double vol = P->h[0] * P->h[1] * P->h[2] / 6.0;
    double sum = 0.0;
    for (int o = 0; o < 8; ++o) {
        int c[3] = {j[0] - (o & 1), j[1] - ((o >> 1) & 1), j[2] - ((o >> 2) & 1)};
        int ok = 1;
        for (int a = 0; a < 3; ++a)
            if (c[a] < 0 || c[a] > P->n[a] - 2) ok = 0;
        if (!ok || hole_cell(P, c)) continue;   /* the hole is not part of the domain */
        int base[3], step[3];
        cell_frame(P, c, base, step);
        for (int s = 0; s < 6; ++s) {
            int v[4][3];
            tet_vertices(base, step, PERMS[s], v);
            int loc = -1;
            for (int m = 0; m < 4; ++m)
                if (v[m][0] == j[0] && v[m][1] == j[1] && v[m][2] == j[2]) loc = m;
            if (loc < 0) continue;
            double pos[4][3], kv[4];
            for (int m = 0; m < 4; ++m) {
                vpos(P, v[m], pos[m]);
                kv[m] = kap(P, v[m]);
            }
            for (int qi = 0; qi < nq; ++qi) {
                const double *b = bp + 4 * qi;
                double y[3] = {0, 0, 0}, ky = 0.0;
                for (int m = 0; m < 4; ++m) {
                    for (int a = 0; a < 3; ++a) y[a] += b[m] * pos[m][a];
                    ky += b[m] * kv[m];
                }
                double r2 = 0.0;
                for (int a = 0; a < 3; ++a) r2 += (x[a] - y[a]) * (x[a] - y[a]);
                sum += vol * bw[qi] * ky * b[loc] / r2;
            }
        }
    }
    return sum / (4.0 * OG_PI);
}

double og_volume_entry(const og_problem_t *P, int64_t i, int64_t j)
{
    int ii[3], jj[3];
    double xi[3], xj[3];
    vidx(P, i, ii);
    vidx(P, j, jj);
    vpos(P, ii, xi);
    vpos(P, jj, xj);
    if (!vertex_active(P, ii) || !vertex_active(P, jj)) return 0.0;
    double G = exp(-og_tau(P, xi, xj)) * volume_quad(P, xi, jj, cheb(ii, jj) <= P->near_cheb);
    for (int w = 0; w < P->n_walls; ++w) {
        if (P->R[w] == 0.0) continue;
        double xb[3];
        int mb[3];
        mirror_point(P, w, xi, xb);
        mirror_index(P, w, ii, mb);
        G += P->R[w] * exp(-og_tau_mirror(P, w, xi, xj)) *
             volume_quad(P, xb, jj, cheb(mb, jj) <= P->near_cheb);
    }
    return G;
}

/* An emitting rectangle of the boundary: the plane x_a = pf (grid index), the
 * normal pointing into the domain (sign * e_a), and the vertex index ranges
 * [lo, hi] along the face's two other axes b < c.  The box's emitting faces,
 * then the hole's. */
typedef struct {
    int a, pf, sign, lo[2], hi[2];
} og_rect_t;

static int emit_rects(const og_problem_t *P, og_rect_t r[12])
{
    int n = 0;
    for (int f = 0; f < 6; ++f) {
        if (!((P->emit_faces >> f) & 1u)) continue;
        int a = f / 2, b = (a == 0) ? 1 : 0, c = (a == 2) ? 1 : 2;
        og_rect_t q = {a, (f & 1) ? P->n[a] - 1 : 0, (f & 1) ? -1 : 1, {0, 0}, {P->n[b] - 1, P->n[c] - 1}};
        r[n++] = q;
    }
    if (has_hole(P))
        for (int f = 0; f < 6; ++f) {
            if (!((P->hole_emit >> f) & 1u)) continue;
            int a = f / 2, b = (a == 0) ? 1 : 0, c = (a == 2) ? 1 : 2;
            og_rect_t q = {a, (f & 1) ? P->hole_hi[a] : P->hole_lo[a], (f & 1) ? 1 : -1,
                           {P->hole_lo[b], P->hole_lo[c]}, {P->hole_hi[b], P->hole_hi[c]}};
            r[n++] = q;
        }
    return n;
}

/* Does the grid square with lower corner (sq[0], sq[1]) (along the axes b < c
 * other than R's) belong to the emitting surface: it lies in R and the cell
 * it bounds on the domain side is not a hole cell (a box face is covered
 * where the hole touches it). */
static int emitting_square(const og_problem_t *P, const og_rect_t *R, const int sq[2])
{
    if (sq[0] < R->lo[0] || sq[0] > R->hi[0] - 1 || sq[1] < R->lo[1] || sq[1] > R->hi[1] - 1) return 0;
    int a = R->a, b = (a == 0) ? 1 : 0, c = (a == 2) ? 1 : 2, cell[3];
    cell[a] = R->sign > 0 ? R->pf : R->pf - 1;
    cell[b] = sq[0];
    cell[c] = sq[1];
    return !hole_cell(P, cell);
}

/* (1/4pi) sum over emitting rectangles R containing l of the integral over R's
 * emitting squares of w~^l(y) [(x-y).n_R]_+ / |x-y|^3 (a rectangle seen from
 * behind adds nothing); on the diagonal, when the point lies in the plane of
 * R, the planar angle theta of R's emitting squares at the point over 4pi
 * (pi/2 per square).  With the Example's cosine-weighted source (section
 * "Example": Q = [omega.n]_- Q0) the integrand is w~^l(y) ([(x-y).n_R]_+)^2 /
 * |x-y|^4 and the in-plane limit half as large: a quarter plane gives
 * int_0^inf d^2 rho / (d^2 + rho^2)^2 drho * pi/2 = pi/4 whatever d, so pi/4
 * per square over 4pi. */
static double surface_quad(const og_problem_t *P, const double x[3], const int xidx[3],
                           const int l[3], int near)
{
    int nq = near ? P->nq_tri_near : P->nq_tri_far;
    const double *bp = near ? P->tri_near_p : P->tri_far_p;
    const double *bw = near ? P->tri_near_w : P->tri_far_w;
    og_rect_t rects[12];
    int nr = emit_rects(P, rects);
    double sum = 0.0;
    for (int f = 0; f < nr; ++f) {
        const og_rect_t *R = &rects[f];
        int a = R->a, pf = R->pf;
        int b = (a == 0) ? 1 : 0;
        int c = (a == 2) ? 1 : 2;
        if (l[a] != pf) continue;
        double plane = P->lo[a] + pf * P->h[a];
        if (xidx[a] == pf) {
            if (xidx[0] == l[0] && xidx[1] == l[1] && xidx[2] == l[2])
                for (int o = 0; o < 4; ++o) {
                    int sq[2] = {l[b] - (o & 1), l[c] - ((o >> 1) & 1)};
                    if (emitting_square(P, R, sq)) sum += (P->emission ? 0.25 : 0.5) * OG_PI / (4.0 * OG_PI);
                }
            continue;
        }
        double d = (x[a] - plane) * R->sign;
        if (d <= 0.0) continue;
        double area = 0.5 * P->h[b] * P->h[c];
        for (int o = 0; o < 4; ++o) {
            int sq[2] = {l[b] - (o & 1), l[c] - ((o >> 1) & 1)};
            if (!emitting_square(P, R, sq)) continue;
            /* square frame, mirrored like the cells when the flip axis lies in the face */
            int B[2] = {sq[0], sq[1]}, S[2] = {1, 1};
            if (P->flip_axis == b && sq[0] < P->flip_cells) { B[0] = sq[0] + 1; S[0] = -1; }
            if (P->flip_axis == c && sq[1] < P->flip_cells) { B[1] = sq[1] + 1; S[1] = -1; }
            for (int t = 0; t < 2; ++t) {
                int tv[3][2];
                tv[0][0] = B[0];
                tv[0][1] = B[1];
                tv[2][0] = B[0] + S[0];
                tv[2][1] = B[1] + S[1];
                if (t == 0) { tv[1][0] = B[0] + S[0]; tv[1][1] = B[1]; }
                else        { tv[1][0] = B[0];        tv[1][1] = B[1] + S[1]; }
                int loc = -1;
                for (int m = 0; m < 3; ++m)
                    if (tv[m][0] == l[b] && tv[m][1] == l[c]) loc = m;
                if (loc < 0) continue;
                double pos[3][3];
                for (int m = 0; m < 3; ++m) {
                    int vi[3];
                    vi[a] = pf;
                    vi[b] = tv[m][0];
                    vi[c] = tv[m][1];
                    vpos(P, vi, pos[m]);
                }
                for (int qi = 0; qi < nq; ++qi) {
                    const double *bb = bp + 3 * qi;
                    double y[3] = {0, 0, 0};
                    for (int m = 0; m < 3; ++m)
                        for (int k = 0; k < 3; ++k) y[k] += bb[m] * pos[m][k];
                    double r2 = 0.0;
                    for (int k = 0; k < 3; ++k) r2 += (x[k] - y[k]) * (x[k] - y[k]);
                    const double k = P->emission ? d * d / (r2 * r2) : d / (r2 * sqrt(r2));
                    sum += area * bw[qi] * bb[loc] * k / (4.0 * OG_PI);
                }
            }
        }
    }
    return sum;
}

double og_surface_entry(const og_problem_t *P, int64_t i, int64_t l)
{
    int ii[3], ll[3];
    double xi[3], xl[3];
    vidx(P, i, ii);
    vidx(P, l, ll);
    vpos(P, ii, xi);
    vpos(P, ll, xl);
    if (!vertex_active(P, ii) || !vertex_active(P, ll)) return 0.0;
    double S = exp(-og_tau(P, xi, xl)) * surface_quad(P, xi, ii, ll, cheb(ii, ll) <= P->near_cheb);
    for (int w = 0; w < P->n_walls; ++w) {
        if (P->R[w] == 0.0) continue;
        double xb[3];
        int mb[3];
        mirror_point(P, w, xi, xb);
        mirror_index(P, w, ii, mb);
        S += P->R[w] * exp(-og_tau_mirror(P, w, xi, xl)) *
             surface_quad(P, xb, mb, ll, cheb(mb, ll) <= P->near_cheb);
    }
    return S;
}

/* ---------------------------------------------------------------- batched entry points */

void og_volume_block(const og_problem_t *P, int64_t nr, const int64_t *rows, int64_t nc,
                     const int64_t *cols, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nr; ++r)
        for (int64_t c = 0; c < nc; ++c) out[r * nc + c] = og_volume_entry(P, rows[r], cols[c]);
}

void og_surface_block(const og_problem_t *P, int64_t nr, const int64_t *rows, int64_t nc,
                      const int64_t *cols, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nr; ++r)
        for (int64_t c = 0; c < nc; ++c) out[r * nc + c] = og_surface_entry(P, rows[r], cols[c]);
}

void og_volume_pairs(const og_problem_t *P, int64_t n, const int64_t *rows, const int64_t *cols,
                     double *out)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < n; ++k) out[k] = og_volume_entry(P, rows[k], cols[k]);
}

void og_surface_pairs(const og_problem_t *P, int64_t n, const int64_t *rows, const int64_t *cols,
                      double *out)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < n; ++k) out[k] = og_surface_entry(P, rows[k], cols[k]);
}

/* mask[v] = 1 when vertex v is a corner of an emitting square (the surface
 * unknowns, in natural order), else 0 */
void og_emitting_mask(const og_problem_t *P, uint8_t *mask)
{
    og_rect_t rects[12];
    int nr = emit_rects(P, rects);
    int64_t N = (int64_t)P->n[0] * P->n[1] * P->n[2];
    for (int64_t v = 0; v < N; ++v) {
        int l[3];
        vidx(P, v, l);
        mask[v] = 0;
        for (int f = 0; f < nr && !mask[v]; ++f) {
            const og_rect_t *R = &rects[f];
            int a = R->a, b = (a == 0) ? 1 : 0, c = (a == 2) ? 1 : 2;
            if (l[a] != R->pf) continue;
            for (int o = 0; o < 4; ++o) {
                int sq[2] = {l[b] - (o & 1), l[c] - ((o >> 1) & 1)};
                if (emitting_square(P, R, sq)) mask[v] = 1;
            }
        }
    }
}

void og_kappa_points(const og_problem_t *P, int64_t n, const double *x, double *out)
{
    for (int64_t k = 0; k < n; ++k) out[k] = og_kappa_at(P, x + 3 * k);
}

/* wall < 0: the straight segment; else the path reflected by wall `wall` */
void og_tau_segments(const og_problem_t *P, int64_t n, const double *p, const double *q,
                     int32_t wall, double *out)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < n; ++k)
        out[k] = wall >= 0 ? og_tau_mirror(P, wall, p + 3 * k, q + 3 * k) : og_tau(P, p + 3 * k, q + 3 * k);
}
