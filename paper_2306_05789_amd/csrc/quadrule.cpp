// Symmetric quadrature rules on the tetrahedron and the triangle, derived at
// run time from their moment equations.
//
// Section "FEM discretization" integrates against P1 hat functions with points
// inside the elements: degree 5 (M_q = 14) near the target vertex and degree 2
// (M_q = 4) elsewhere.  The boundary source matrix uses the triangle rules of
// the same degrees (3 and 7 points).  Each rule is fixed by its symmetry
// orbits; the orbit parameters solve "the rule integrates every barycentric
// monomial of degree <= d exactly", where the exact simplex mean of
// lambda^alpha is d! prod(alpha_i!) / (d + |alpha|)!.  The system is solved
// by damped Gauss-Newton from a deterministic set of starts and the unique
// interior positive-weight solution is kept.
#include <algorithm>
#include <array>
#include <cmath>
#include <functional>
#include <mutex>

#include "rte_internal.h"

namespace rte {
namespace {

double factorial(int k) {
    double f = 1;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

struct Moments {
    int nvert, degree;
    std::vector<std::vector<int>> alpha;
    std::vector<double> exact;
    Moments(int nv, int deg) : nvert(nv), degree(deg) {
        std::vector<int> a(nv, 0);
        std::function<void(int, int)> rec = [&](int pos, int left) {
            if (pos == nv - 1) {
                a[pos] = left;
                alpha.push_back(a);
                return;
            }
            for (int k = 0; k <= left; ++k) {
                a[pos] = k;
                rec(pos + 1, left - k);
            }
        };
        for (int total = 0; total <= degree; ++total) rec(0, total);
        for (auto &al : alpha) {
            double num = factorial(nv - 1);
            int s = 0;
            for (int x : al) { num *= factorial(x); s += x; }
            exact.push_back(num / factorial(nv - 1 + s));
        }
    }
};

// All distinct permutations of a barycentric tuple.
std::vector<std::vector<double>> orbit(std::vector<double> base) {
    std::sort(base.begin(), base.end());
    std::vector<std::vector<double>> out;
    do { out.push_back(base); } while (std::next_permutation(base.begin(), base.end()));
    return out;
}

using Builder = std::function<void(const std::vector<double> &, std::vector<std::vector<double>> &,
                                   std::vector<double> &)>;

std::vector<double> residual(const Moments &M, const Builder &b, const std::vector<double> &x) {
    std::vector<std::vector<double>> pts;
    std::vector<double> w;
    b(x, pts, w);
    // integer powers of every barycentric coordinate, up to the rule degree
    const int D = M.degree + 1;
    std::vector<double> pw(pts.size() * M.nvert * D);
    for (size_t q = 0; q < pts.size(); ++q)
        for (int d = 0; d < M.nvert; ++d) {
            double *p = &pw[(q * M.nvert + d) * D];
            p[0] = 1.0;
            for (int e = 1; e < D; ++e) p[e] = p[e - 1] * pts[q][d];
        }
    std::vector<double> r(M.alpha.size());
    for (size_t k = 0; k < M.alpha.size(); ++k) {
        double v = 0;
        for (size_t q = 0; q < pts.size(); ++q) {
            double m = w[q];
            for (int d = 0; d < M.nvert; ++d) m *= pw[(q * M.nvert + d) * D + M.alpha[k][d]];
            v += m;
        }
        r[k] = v - M.exact[k];
    }
    return r;
}

double norm2(const std::vector<double> &r) {
    double s = 0;
    for (double v : r) s += v * v;
    return s;
}

// Solve the small normal equations (J^T J + mu I) dx = -J^T r by Gaussian elimination.
std::vector<double> solve_small(std::vector<std::vector<double>> A, std::vector<double> b) {
    int n = (int)b.size();
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
        std::swap(A[c], A[piv]);
        std::swap(b[c], b[piv]);
        if (A[c][c] == 0) return std::vector<double>(n, 0.0);
        for (int r = c + 1; r < n; ++r) {
            double f = A[r][c] / A[c][c];
            for (int k = c; k < n; ++k) A[r][k] -= f * A[c][k];
            b[r] -= f * b[c];
        }
    }
    std::vector<double> x(n);
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int k = r + 1; k < n; ++k) s -= A[r][k] * x[k];
        x[r] = s / A[r][r];
    }
    return x;
}

bool gauss_newton(const Moments &M, const Builder &b, std::vector<double> &x) {
    int n = (int)x.size();
    double mu = 1e-3;
    auto r = residual(M, b, x);
    double f = norm2(r);
    for (int it = 0; it < 300 && f > 1e-31; ++it) {
        std::vector<std::vector<double>> J(r.size(), std::vector<double>(n));
        for (int c = 0; c < n; ++c) {
            double eps = 1e-7 * std::max(1.0, std::fabs(x[c]));
            auto xp = x, xm = x;
            xp[c] += eps;
            xm[c] -= eps;
            auto rp = residual(M, b, xp), rm = residual(M, b, xm);
            for (size_t k = 0; k < r.size(); ++k) J[k][c] = (rp[k] - rm[k]) / (2 * eps);
        }
        std::vector<std::vector<double>> A(n, std::vector<double>(n, 0.0));
        std::vector<double> g(n, 0.0);
        for (size_t k = 0; k < r.size(); ++k)
            for (int a = 0; a < n; ++a) {
                g[a] -= J[k][a] * r[k];
                for (int c = 0; c < n; ++c) A[a][c] += J[k][a] * J[k][c];
            }
        bool improved = false;
        for (int tries = 0; tries < 20; ++tries) {
            auto Am = A;
            for (int a = 0; a < n; ++a) Am[a][a] *= (1 + mu);
            auto dx = solve_small(Am, g);
            auto xn = x;
            for (int a = 0; a < n; ++a) xn[a] += dx[a];
            auto rn = residual(M, b, xn);
            double fn = norm2(rn);
            if (std::isfinite(fn) && fn < f) {
                x = xn;
                r = rn;
                f = fn;
                mu = std::max(mu * 0.2, 1e-12);
                improved = true;
                break;
            }
            mu *= 10;
        }
        if (!improved) break;
    }
    double worst = 0;
    for (double v : r) worst = std::max(worst, std::fabs(v));
    return worst < 1e-13;
}

Rule solve_rule(int nvert, int degree, int nparams, const Builder &b, const std::vector<double> &lo,
                const std::vector<double> &hi, const std::function<std::vector<double>(std::vector<double>)> &canon,
                int starts) {
    Moments M(nvert, degree);
    uint64_t state = 0x9E3779B97F4A7C15ull ^ (uint64_t)(nvert * 131 + degree);
    auto uni = [&]() {
        state = state * 6364136223846793005ull + 1442695040888963407ull;
        return (double)(state >> 11) * (1.0 / 9007199254740992.0);
    };
    std::vector<std::vector<double>> found;
    for (int s = 0; s < starts; ++s) {
        std::vector<double> x(nparams);
        for (int k = 0; k < nparams; ++k) x[k] = lo[k] + (hi[k] - lo[k]) * uni();
        if (!gauss_newton(M, b, x)) continue;
        std::vector<std::vector<double>> pts;
        std::vector<double> w;
        b(x, pts, w);
        bool ok = true;
        for (double v : w) ok &= v > 1e-12;
        for (auto &p : pts)
            for (double v : p) ok &= v > 1e-9;
        if (!ok) continue;
        auto key = canon(x);
        bool dup = false;
        for (auto &f : found) {
            double d = 0;
            for (int k = 0; k < nparams; ++k) d = std::max(d, std::fabs(f[k] - key[k]));
            dup |= d < 1e-9;
        }
        if (!dup) found.push_back(key);
    }
    if (found.size() != 1)
        throw Error(RTE_E_INTERNAL, "quadrature derivation: expected a unique interior rule, found " +
                                        std::to_string(found.size()));
    Rule R;
    std::vector<std::vector<double>> pts;
    b(found[0], pts, R.w);
    R.nvert = nvert;
    R.degree = degree;
    R.nq = (int)pts.size();
    for (auto &p : pts) R.p.insert(R.p.end(), p.begin(), p.end());
    return R;
}

void add_orbit(std::vector<double> base, double w, std::vector<std::vector<double>> &pts, std::vector<double> &ws) {
    for (auto &p : orbit(base)) {
        pts.push_back(p);
        ws.push_back(w);
    }
}

std::vector<double> canon_pairs(std::vector<double> x, int i, int j) {
    if (x[i] > x[j]) {
        std::swap(x[i], x[j]);
        std::swap(x[i + 1], x[j + 1]);
    }
    return x;
}

Rule make_tet(int degree) {
    if (degree == 2) {
        Builder b = [](const std::vector<double> &x, std::vector<std::vector<double>> &p, std::vector<double> &w) {
            double a = x[0], c = (1 - a) / 3;
            add_orbit({a, c, c, c}, 0.25, p, w);
        };
        return solve_rule(4, 2, 1, b, {-0.5}, {1.0}, [](std::vector<double> x) { return x; }, 32);
    }
    // two (a,b,b,b) orbits and one (c,c,d,d) orbit: 4 + 4 + 6 = 14 points
    Builder b = [](const std::vector<double> &x, std::vector<std::vector<double>> &p, std::vector<double> &w) {
        for (int o = 0; o < 2; ++o) {
            double a = x[2 * o], c = (1 - a) / 3;
            add_orbit({a, c, c, c}, x[2 * o + 1], p, w);
        }
        double c = x[4], d = 0.5 - c;
        add_orbit({c, c, d, d}, x[5], p, w);
    };
    auto canon = [](std::vector<double> x) {
        x[4] = std::min(x[4], 0.5 - x[4]);   // (c,c,d,d) and (d,d,c,c) are the same orbit
        return canon_pairs(x, 0, 2);
    };
    return solve_rule(4, 5, 6, b, {0, 0, 0, 0, 0, 0}, {1, 0.2, 1, 0.2, 0.5, 0.2}, canon, 48);
}

Rule make_tri(int degree) {
    if (degree == 2) {
        Builder b = [](const std::vector<double> &x, std::vector<std::vector<double>> &p, std::vector<double> &w) {
            double a = x[0], c = (1 - a) / 2;
            add_orbit({a, c, c}, 1.0 / 3.0, p, w);
        };
        return solve_rule(3, 2, 1, b, {-0.5}, {1.0}, [](std::vector<double> x) { return x; }, 32);
    }
    // centroid plus two (a,b,b) orbits: 1 + 3 + 3 = 7 points
    Builder b = [](const std::vector<double> &x, std::vector<std::vector<double>> &p, std::vector<double> &w) {
        p.push_back({1.0 / 3, 1.0 / 3, 1.0 / 3});
        w.push_back(x[0]);
        for (int o = 0; o < 2; ++o) {
            double a = x[1 + 2 * o], c = (1 - a) / 2;
            add_orbit({a, c, c}, x[2 + 2 * o], p, w);
        }
    };
    auto canon = [](std::vector<double> x) { return canon_pairs(x, 1, 3); };
    return solve_rule(3, 5, 5, b, {0, 0, 0, 0, 0}, {0.5, 1, 0.3, 1, 0.3}, canon, 48);
}

}  // namespace

const Rule &tet_rule(int degree) {
    static std::once_flag f2, f5;
    static Rule r2, r5;
    if (degree == 2) { std::call_once(f2, [] { r2 = make_tet(2); }); return r2; }
    if (degree == 5) { std::call_once(f5, [] { r5 = make_tet(5); }); return r5; }
    throw Error(RTE_E_INTERNAL, "tet rule degree");
}

const Rule &tri_rule(int degree) {
    static std::once_flag f2, f5;
    static Rule r2, r5;
    if (degree == 2) { std::call_once(f2, [] { r2 = make_tri(2); }); return r2; }
    if (degree == 5) { std::call_once(f5, [] { r5 = make_tri(5); }); return r5; }
    throw Error(RTE_E_INTERNAL, "tri rule degree");
}

}  // namespace rte
