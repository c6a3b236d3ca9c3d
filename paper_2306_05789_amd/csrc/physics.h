// Source terms and the per-vertex temperature balance shared by the fixed-point
// solver and the request server (Algorithm of Section "Fixed Point
// Iterations"; eq. grey for the one-band case).
#pragma once

#include <hip/hip_runtime.h>

namespace rte {

constexpr double kSigma = 6.493939402266829;   // pi^4 / 15

// rescaled Planck function B_nu(T) = nu^3 / (exp(nu / T) - 1), B(0) = 0
__device__ __forceinline__ double planck(double nu, double T) {
    if (!(T > 0.0)) return 0.0;
    const double x = nu / T;
    if (x > 700.0) return 0.0;
    return nu * nu * nu / expm1(x);
}


// The temperature T >= 0 solving sum_b c_b (J_b - B_{nu_b}(T)) = 0 with
// c_b >= 0 (c_b = w_b kappa_b (1 - a_b)), started from Told.  band(b, nu, c, J)
// gives nu_b, c_b and J_b.  f decreases in T and f(0) = sum c_b J_b > 0: a
// safeguarded Newton iteration.  Every evaluation narrows the bracket
// [lo, hi] by the sign of f (hi starts unbounded); a step that leaves it is
// replaced by bisection, or by doubling while hi is unbounded.  Newton
// converges quadratically from the previous sweep's temperature: once a
// Newton step s is below 1e-8 relative, the iterate after it is within about
// (nu / T) s^2 of the root, at the rounding level for the frequencies and
// temperatures here, and the iteration stops, whether or not that step lands
// strictly inside the bracket (near the root the step rounds to almost
// nothing, and rejecting it for a bisection would restart the search from the
// far end of the bracket).
//
// NB > 0: the loops over the bands are unrolled to NB iterations guarded by
// b < nb (nb <= NB), so that a caller can keep the bands' c_b and J_b in
// registers; the sums are taken in the same order either way.
template <int NB, typename F>
__device__ __forceinline__ void for_bands(int nb, F f) {
    if constexpr (NB > 0) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
            if (b < nb) f(b);
    } else {
        for (int b = 0; b < nb; ++b) f(b);
    }
}

template <int NB = 0, typename Band>
__device__ double solve_temperature(int nb, double Told, Band band) {
    double f0 = 0.0;
    for_bands<NB>(nb, [&](int b) {
        double nu, c, j;
        band(b, nu, c, j);
        f0 += c * j;
    });
    if (!(f0 > 0.0)) return 0.0;
    // f = f0 - sum c_b B_b(t) and f' at t > 0: B = nu^3 r, dB/dT = B (1 + r) x / t
    // with x = nu / t and r = 1 / (e^x - 1); one division per band.  The J_b enter
    // through f0 alone, so a caller holding the bands in registers keeps only c_b
    // live through the iteration.
    auto f = [&](double t, double &df) {
        double s = 0.0, d = 0.0;
        const double it = 1.0 / t;
        for_bands<NB>(nb, [&](int b) {
            double nu, c, j;
            band(b, nu, c, j);
            const double x = nu * it;
            double B = 0.0, dB = 0.0;
            if (x <= 700.0) {
                const double r = 1.0 / expm1(x);
                B = nu * nu * nu * r;
                dB = B * (1.0 + r) * (x * it);
            }
            s += c * B;
            d -= c * dB;
        });
        df = d;
        return f0 - s;
    };
    double lo = 0.0, hi = INFINITY, d;
    double x = Told > 0.0 ? Told : 1.0;
    for (int it = 0; it < 200; ++it) {
        const double fx = f(x, d);
        if (fx == 0.0) break;
        if (fx > 0.0) lo = x; else hi = x;
        double xn = (d < 0.0) ? x - fx / d : -1.0;
        if (xn > 0.0 && fabs(xn - x) <= 1e-8 * x) {   // the next iterate is at the rounding level
            x = xn;
            break;
        }
        if (!(xn > lo && xn < hi)) xn = isinf(hi) ? 2.0 * x : 0.5 * (lo + hi);
        x = xn;
        if (hi - lo <= 2.3e-16 * hi && !isinf(hi)) break;
    }
    return x;
}

}  // namespace rte
