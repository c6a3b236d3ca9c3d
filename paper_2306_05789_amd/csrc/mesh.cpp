// Structured Kuhn mesh of a box and the quadrature stencils of the P1
// collocation (Section "FEM discretization and Compressed H-Matrices").
//
// Each grid cell is split into the six tetrahedra that share its
// (0,0,0)-(1,1,1) diagonal, one per ordering of the three axes; a vertex of
// the interior belongs to 24 of them.  Boundary squares are split along the
// same diagonal direction, so a vertex inside a face belongs to 6 triangles.
// On a uniform grid the quadrature points of the elements around a vertex sit
// at fixed offsets from it, so one table per rule serves every vertex; the
// elements that fall outside the box are masked per vertex.
#include <cmath>
#include <map>
#include <mutex>

#include "rte_internal.h"

namespace rte {

std::vector<double> Mesh::positions() const {
    std::vector<double> p((size_t)N * 3);
    for (int64_t v = 0; v < N; ++v) {
        int64_t k = v % desc.n[2], j = (v / desc.n[2]) % desc.n[1], i = v / ((int64_t)desc.n[1] * desc.n[2]);
        p[3 * v + 0] = desc.lo[0] + i * h[0];
        p[3 * v + 1] = desc.lo[1] + j * h[1];
        p[3 * v + 2] = desc.lo[2] + k * h[2];
    }
    return p;
}

std::vector<double> Mesh::emitting_positions() const {
    auto all = positions();
    std::vector<double> p;
    p.reserve(emitting.size() * 3);
    for (int64_t v : emitting) p.insert(p.end(), all.begin() + 3 * v, all.begin() + 3 * v + 3);
    return p;
}

static const int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

static StencilHost make_stencil() {
    StencilHost S;
    const Rule &r_far = tet_rule(2), &r_near = tet_rule(5);
    const Rule &t_far = tri_rule(2), &t_near = tri_rule(5);
    S.nq_vol_far = r_far.nq;
    S.nq_vol_near = r_near.nq;
    S.nq_tri_far = t_far.nq;
    S.nq_tri_near = t_near.nq;
    // the device quadrature loops are specialised for these orbit sizes
    if (r_far.nq != 4 || r_near.nq != 14 || t_far.nq != 3 || t_near.nq != 7)
        throw Error(RTE_E_INTERNAL, "quadrature rule sizes differ from the device stencil sizes");
    struct Tet { int dv[4][3]; int loc; int bits; };
    std::vector<Tet> tets;
    for (int bits = 0; bits < 8; ++bits) {
        int o[3] = {bits & 1, (bits >> 1) & 1, (bits >> 2) & 1};
        for (auto &sg : kPerm) {
            int w[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {1, 1, 1}};
            w[1][sg[0]] = 1;
            w[2][sg[0]] = 1;
            w[2][sg[1]] = 1;
            int loc = -1;
            for (int k = 0; k < 4; ++k)
                if (w[k][0] == o[0] && w[k][1] == o[1] && w[k][2] == o[2]) loc = k;
            if (loc < 0) continue;
            Tet t;
            for (int k = 0; k < 4; ++k)
                for (int a = 0; a < 3; ++a) t.dv[k][a] = w[k][a] - o[a];
            t.loc = loc;
            t.bits = bits;
            tets.push_back(t);
        }
    }
    if ((int)tets.size() != kTets) throw Error(RTE_E_INTERNAL, "Kuhn star size");
    auto fill_vol = [&](const Rule &r, std::vector<double> &out) {
        out.assign((size_t)kTets * r.nq * 8, 0.0);
        for (int t = 0; t < kTets; ++t)
            for (int q = 0; q < r.nq; ++q) {
                double *e = &out[((size_t)t * r.nq + q) * 8];
                const double *b = &r.p[(size_t)q * 4];
                for (int a = 0; a < 3; ++a) {
                    double s = 0;
                    for (int k = 0; k < 4; ++k) s += b[k] * tets[t].dv[k][a];
                    e[a] = s;
                }
                e[3] = r.w[q] * b[tets[t].loc];
                for (int k = 0; k < 4; ++k) e[4 + k] = b[k];
            }
    };
    fill_vol(r_far, S.vol_far);
    fill_vol(r_near, S.vol_near);
    for (auto &t : tets) {
        for (int k = 0; k < 4; ++k)
            S.tet_meta.push_back((t.dv[k][0] + 1) * 9 + (t.dv[k][1] + 1) * 3 + (t.dv[k][2] + 1));
        S.tet_meta.push_back(t.bits);
    }
    // boundary triangles around a face vertex, in the face's axes (b, c)
    struct Tri { int dv[3][2]; int loc; int ob, oc; };
    std::vector<Tri> tris;
    const int corners[2][3][2] = {{{0, 0}, {1, 0}, {1, 1}}, {{0, 0}, {0, 1}, {1, 1}}};
    for (int ob = 0; ob < 2; ++ob)
        for (int oc = 0; oc < 2; ++oc)
            for (int t = 0; t < 2; ++t) {
                int loc = -1;
                for (int k = 0; k < 3; ++k)
                    if (corners[t][k][0] == ob && corners[t][k][1] == oc) loc = k;
                if (loc < 0) continue;
                Tri tr;
                for (int k = 0; k < 3; ++k) {
                    tr.dv[k][0] = corners[t][k][0] - ob;
                    tr.dv[k][1] = corners[t][k][1] - oc;
                }
                tr.loc = loc;
                tr.ob = ob;
                tr.oc = oc;
                tris.push_back(tr);
            }
    if ((int)tris.size() != kTris) throw Error(RTE_E_INTERNAL, "face star size");
    auto fill_tri = [&](const Rule &r, std::vector<double> &out) {
        out.assign((size_t)kTris * r.nq * 4, 0.0);
        for (int t = 0; t < kTris; ++t)
            for (int q = 0; q < r.nq; ++q) {
                double *e = &out[((size_t)t * r.nq + q) * 4];
                const double *b = &r.p[(size_t)q * 3];
                for (int a = 0; a < 2; ++a) {
                    double s = 0;
                    for (int k = 0; k < 3; ++k) s += b[k] * tris[t].dv[k][a];
                    e[a] = s;
                }
                e[2] = r.w[q] * b[tris[t].loc];
                e[3] = 0;
            }
    };
    fill_tri(t_far, S.tri_far);
    fill_tri(t_near, S.tri_near);
    for (auto &t : tris) {
        S.tri_meta.push_back(t.ob);
        S.tri_meta.push_back(t.oc);
    }
    return S;
}

const StencilHost &stencil_host() {
    static std::once_flag f;
    static StencilHost S;
    std::call_once(f, [] { S = make_stencil(); });
    return S;
}

namespace {
template <typename T>
const T *upload_forever(const std::vector<double> &v) {
    std::vector<T> c(v.begin(), v.end());
    void *p = nullptr;
    HIP_CHECK(hipMalloc(&p, c.size() * sizeof(T)));
    HIP_CHECK(hipMemcpy(p, c.data(), c.size() * sizeof(T), hipMemcpyHostToDevice));
    return static_cast<const T *>(p);
}
const int *upload_ints(const std::vector<int> &v) {
    void *p = nullptr;
    HIP_CHECK(hipMalloc(&p, v.size() * sizeof(int)));
    HIP_CHECK(hipMemcpy(p, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice));
    return static_cast<const int *>(p);
}
}  // namespace

// One copy per device, kept for the life of the process.
const StencilBuffers &stencil_device() {
    static std::mutex mu;
    static std::map<int, StencilBuffers> per_dev;
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = per_dev.find(dev);
    if (it != per_dev.end()) return it->second;
    const StencilHost &H = stencil_host();
    StencilBuffers B;
    const int *tm = upload_ints(H.tet_meta);
    const int *rm = upload_ints(H.tri_meta);
    B.d = {upload_forever<double>(H.tri_far), upload_forever<double>(H.tri_near), H.nq_tri_far, H.nq_tri_near, tm, rm};
    B.f = {upload_forever<float>(H.tri_far), upload_forever<float>(H.tri_near), H.nq_tri_far, H.nq_tri_near, tm, rm};
    return per_dev.emplace(dev, B).first->second;
}

// Weights of the near table (see NearTables): the same sums as the device's
// degree-5 loop, grouped by the cell and corner whose kappa they multiply.
static std::vector<double> make_near_table(const double h[3]) {
    static_assert(kNearCheb == 2 && kNearOffsets == 125, "the near table covers offsets in [-2, 2]^3");
    const StencilHost &S = stencil_host();
    const int nq = S.nq_vol_near;
    std::vector<double> T((size_t)kNearOffsets * 64, 0.0);
    for (int dx = -2; dx <= 2; ++dx)
        for (int dy = -2; dy <= 2; ++dy)
            for (int dz = -2; dz <= 2; ++dz) {
                const int d[3] = {dx, dy, dz};
                double *row = &T[(size_t)((dx + 2) * 25 + (dy + 2) * 5 + (dz + 2)) * 64];
                for (int t = 0; t < kTets; ++t) {
                    const int bits = S.tet_meta[5 * t + 4];
                    const int o[3] = {bits & 1, (bits >> 1) & 1, (bits >> 2) & 1};
                    for (int q = 0; q < nq; ++q) {
                        const double *e = &S.vol_near[((size_t)t * nq + q) * 8];
                        double r2 = 0.0;
                        for (int a = 0; a < 3; ++a) r2 += h[a] * h[a] * (d[a] - e[a]) * (d[a] - e[a]);
                        const double w = e[3] / r2;
                        for (int k = 0; k < 4; ++k) {
                            const int slot = S.tet_meta[5 * t + k];
                            const int s3[3] = {slot / 9 - 1, (slot / 3) % 3 - 1, slot % 3 - 1};
                            const int corner = (s3[0] + o[0]) + 2 * (s3[1] + o[1]) + 4 * (s3[2] + o[2]);
                            row[bits * 8 + corner] += w * e[4 + k];
                        }
                    }
                }
            }
    // far field
    T.resize((size_t)kNearSize + kFarSize, 0.0);
    const int nf = S.nq_vol_far;
    if (nf != 4) throw Error(RTE_E_INTERNAL, "far rule size");
    for (int t = 0; t < kTets; ++t)
        for (int q = 0; q < nf; ++q) {
            const double *e = &S.vol_far[((size_t)t * nf + q) * 8];
            double *f = &T[(size_t)kNearSize + ((size_t)t * 4 + q) * 8];
            double c = 0.0;
            for (int a = 0; a < 3; ++a) {
                f[a] = -2.0 * h[a] * h[a] * e[a];
                c += h[a] * h[a] * e[a] * e[a];
            }
            f[3] = c;
            for (int k = 0; k < 4; ++k) f[4 + k] = e[3] * e[4 + k];
        }
    return T;
}

NearTables::~NearTables() {
    for (auto &kv : dev) {
        (void)hipFree(kv.second.first);
        (void)hipFree(kv.second.second);
    }
}

const void *Mesh::near_table(bool fp64) const {
    int d = 0;
    HIP_CHECK(hipGetDevice(&d));
    std::lock_guard<std::mutex> lk(near->mu);
    auto it = near->dev.find(d);
    if (it == near->dev.end()) {
        const std::vector<double> &H = near->host;
        std::vector<float> F(H.begin(), H.end());
        void *pd = nullptr, *pf = nullptr;
        HIP_CHECK(hipMalloc(&pd, H.size() * sizeof(double)));
        HIP_CHECK(hipMalloc(&pf, F.size() * sizeof(float)));
        HIP_CHECK(hipMemcpy(pd, H.data(), H.size() * sizeof(double), hipMemcpyHostToDevice));
        HIP_CHECK(hipMemcpy(pf, F.data(), F.size() * sizeof(float), hipMemcpyHostToDevice));
        it = near->dev.emplace(d, std::make_pair(pd, pf)).first;
    }
    return fp64 ? it->second.first : it->second.second;
}

// The emitting rectangles of a mesh: the emitting box faces, then the hole's
// emitting faces; square index ranges [lo, hi) along the two other axes.
std::vector<EmitRect> emit_rects(const rte_mesh_desc_t &d) {
    std::vector<EmitRect> r;
    for (int f = 0; f < 6; ++f) {
        if (!((d.emit_faces >> f) & 1u)) continue;
        const int a = f / 2, b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
        r.push_back({a, (f & 1) ? d.n[a] - 1 : 0, (f & 1) ? -1 : 1, {0, 0}, {d.n[b] - 1, d.n[c] - 1}});
    }
    for (int f = 0; f < 6; ++f) {
        if (!((d.hole_emit >> f) & 1u)) continue;
        const int a = f / 2, b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
        r.push_back({a, (f & 1) ? d.hole_hi[a] : d.hole_lo[a], (f & 1) ? 1 : -1, {d.hole_lo[b], d.hole_lo[c]},
                     {d.hole_hi[b], d.hole_hi[c]}});
    }
    return r;
}

void mesh_init(Mesh &M, const rte_mesh_desc_t &d) {
    for (int a = 0; a < 3; ++a) {
        RTE_REQUIRE(d.n[a] >= 2, "mesh: every axis needs at least 2 vertices");
        RTE_REQUIRE(d.n[a] <= (1 << 20), "mesh: axis too long");
        RTE_REQUIRE(std::isfinite(d.lo[a]) && std::isfinite(d.hi[a]) && d.lo[a] < d.hi[a],
                    "mesh: need finite lo < hi on every axis");
    }
    // the device kernels index vertices (and kappa bytes) with 32-bit integers
    RTE_REQUIRE((int64_t)d.n[0] * d.n[1] * d.n[2] < ((int64_t)1 << 28), "mesh: at most 2^28 vertices");
    RTE_REQUIRE(d.reflect_axis >= -1 && d.reflect_axis <= 2, "mesh: reflect_axis must be -1, 0, 1 or 2");
    RTE_REQUIRE(d.reflect_side == 0 || d.reflect_side == 1, "mesh: reflect_side must be 0 or 1");
    RTE_REQUIRE(d.reflect_axis < 0 || (std::isfinite(d.R) && d.R >= 0.0 && d.R <= 1.0),
                "mesh: R must lie in [0, 1]");
    RTE_REQUIRE(d.emit_faces < 64u, "mesh: emit_faces has 6 bits");
    RTE_REQUIRE(d.reflect_faces < 64u, "mesh: reflect_faces has 6 bits");
    // the reflective walls: the single one of reflect_axis, then those of reflect_faces
    std::vector<std::pair<int, double>> walls;   // (face, R)
    if (d.reflect_axis >= 0) walls.push_back({2 * d.reflect_axis + d.reflect_side, d.R});
    for (int f = 0; f < 6; ++f)
        if ((d.reflect_faces >> f) & 1u) {
            RTE_REQUIRE(d.reflect_axis < 0 || f != 2 * d.reflect_axis + d.reflect_side,
                        "mesh: a face is given as reflective twice");
            RTE_REQUIRE(std::isfinite(d.R_faces[f]) && d.R_faces[f] >= 0.0 && d.R_faces[f] <= 1.0,
                        "mesh: R_faces must lie in [0, 1]");
            walls.push_back({f, d.R_faces[f]});
        }
    for (auto &w : walls)
        RTE_REQUIRE(!((d.emit_faces >> w.first) & 1u), "mesh: a reflective face cannot also emit");
    RTE_REQUIRE(d.emission <= 1u, "mesh: emission must be 0 (isotropic) or 1 (cosine-weighted)");
    // the removed box of cells (all-zero fields: none)
    const bool hole = d.hole_lo[0] < d.hole_hi[0] || d.hole_lo[1] < d.hole_hi[1] || d.hole_lo[2] < d.hole_hi[2];
    if (hole) {
        for (int a = 0; a < 3; ++a)
            RTE_REQUIRE(0 <= d.hole_lo[a] && d.hole_lo[a] < d.hole_hi[a] && d.hole_hi[a] <= d.n[a] - 1,
                        "mesh: the hole must be a non-empty box of cells inside the grid");
        RTE_REQUIRE(d.hole_emit < 64u, "mesh: hole_emit has 6 bits");
        for (int f = 0; f < 6; ++f)
            if ((d.hole_emit >> f) & 1u) {
                const int a = f / 2;
                RTE_REQUIRE((f & 1) ? d.hole_hi[a] < d.n[a] - 1 : d.hole_lo[a] > 0,
                            "mesh: an emitting hole face must lie inside the box");
            }
    } else {
        for (int a = 0; a < 3; ++a)
            RTE_REQUIRE(d.hole_lo[a] == 0 && d.hole_hi[a] == 0, "mesh: the hole must be a non-empty box of cells");
        RTE_REQUIRE(d.hole_emit == 0u, "mesh: hole_emit without a hole");
    }
    int64_t N = (int64_t)d.n[0] * d.n[1] * d.n[2];
    RTE_REQUIRE(N < (int64_t)1 << 31, "mesh: more than 2^31 vertices");
    M.desc = d;
    M.N = N;
    for (int a = 0; a < 3; ++a) M.h[a] = (d.hi[a] - d.lo[a]) / (d.n[a] - 1);
    M.near = std::make_shared<NearTables>();
    M.plans = new_plan_cache();
    M.near->host = make_near_table(M.h);
    // the surface unknowns: corners of the emitting squares (a box-face square
    // whose cell is a hole cell is covered and does not emit)
    auto hole_cell = [&](const int c[3]) {
        if (!hole) return false;
        for (int a = 0; a < 3; ++a)
            if (c[a] < d.hole_lo[a] || c[a] >= d.hole_hi[a]) return false;
        return true;
    };
    std::vector<EmitRect> rects = emit_rects(d);
    M.emitting.clear();
    for (int64_t v = 0; v < N; ++v) {
        int idx[3] = {(int)(v / ((int64_t)d.n[1] * d.n[2])), (int)((v / d.n[2]) % d.n[1]), (int)(v % d.n[2])};
        bool on = false;
        for (const EmitRect &r : rects) {
            if (idx[r.a] != r.plane) continue;
            const int b = r.a == 0 ? 1 : 0, c = r.a == 2 ? 1 : 2;
            for (int o = 0; o < 4 && !on; ++o) {
                const int sb = idx[b] - (o & 1), sc = idx[c] - (o >> 1);
                if (sb < r.lo[0] || sb >= r.hi[0] || sc < r.lo[1] || sc >= r.hi[1]) continue;
                int cell[3];
                cell[r.a] = r.sign > 0 ? r.plane : r.plane - 1;
                cell[b] = sb;
                cell[c] = sc;
                on = !hole_cell(cell);
            }
            if (on) break;
        }
        if (on) M.emitting.push_back(v);
    }
    M.L = (int64_t)M.emitting.size();
    GridDev &g = M.dev;
    for (int a = 0; a < 3; ++a) {
        g.n[a] = d.n[a];
        g.lo[a] = d.lo[a];
        g.h[a] = M.h[a];
    }
    g.stride[0] = d.n[1] * d.n[2];
    g.stride[1] = d.n[2];
    g.stride[2] = 1;
    // walls with R = 0 add nothing and are left out
    g.n_walls = 0;
    for (auto &w : walls) {
        if (!(w.second > 0.0)) continue;
        g.wall_axis[g.n_walls] = w.first / 2;
        g.wall_side[g.n_walls] = w.first % 2;
        g.R[g.n_walls] = w.second;
        ++g.n_walls;
    }
    for (int k = g.n_walls; k < 6; ++k) {
        g.wall_axis[k] = 0;
        g.wall_side[k] = 0;
        g.R[k] = 0.0;
    }
    g.emit_faces = d.emit_faces;
    g.has_hole = hole ? 1 : 0;
    g.hole_open = 0u;
    for (int a = 0; a < 3; ++a) {
        g.hole_lo[a] = hole ? d.hole_lo[a] : 0;
        g.hole_hi[a] = hole ? d.hole_hi[a] : 0;
        if (hole && d.hole_lo[a] == 0) g.hole_open |= 1u << (2 * a);
        if (hole && d.hole_hi[a] == d.n[a] - 1) g.hole_open |= 1u << (2 * a + 1);
    }
    g.hole_emit = hole ? d.hole_emit : 0u;
    g.emission = d.emission;
    const double four_pi = 4.0 * M_PI;
    g.vol_scale = M.h[0] * M.h[1] * M.h[2] / 6.0 / four_pi;
    g.area_scale[0] = 0.5 * M.h[1] * M.h[2] / four_pi;
    g.area_scale[1] = 0.5 * M.h[0] * M.h[2] / four_pi;
    g.area_scale[2] = 0.5 * M.h[0] * M.h[1] / four_pi;
}

}  // namespace rte
