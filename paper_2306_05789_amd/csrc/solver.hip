// The monotone fixed point (Algorithm of Section "Fixed Point Iterations",
// eq. algo) on the GPU, with J^0 = 0:
//   S_b   = (1 - a_b) B_{nu_b}(T) + a_b J_b              (collocated source, eq. eqS / P1)
//   J_b  <- S^E_b + G_b S_b,   S^E_b = S_hat_b Q_b,  Q_b = B_{nu_b}(T_wall)
//   T     : per vertex, root of sum_b w_b kappa_b (1 - a_b)(J_b - B_{nu_b}(T)) = 0
// The temperature root is a safeguarded FP64 Newton iteration (the paper uses
// Newton); in the grey case (eq. grey) B(T) = sigma T^4, sigma = pi^4/15, and
// T = (J/sigma)^{1/4}.  Rescaled Planck function B_nu(T) = nu^3/(exp(nu/T)-1).
// All vectors live in the cluster order of the volume H-matrix; the
// iteration stops when max over bands and right-hand sides of
// ||J^{k+1} - J^k||_2 / ||J^{k+1}||_2 <= tol.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>

#include "kernels.h"
#include "physics.h"

namespace rte {

namespace {

struct BandParams {
    int nb;
    int grey;
    const double *nu;   // device [nb]
    const double *w;    // device [nb]
    const double *a;    // device [nb]
};

__global__ void k_emission(BandParams bp, const double *__restrict__ Tw, int64_t L, int nrhs,
                           double *__restrict__ Q) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = L * nrhs;
    if (k >= tot) return;
    const double T = Tw[k];
    for (int b = 0; b < bp.nb; ++b)
        Q[(int64_t)b * tot + k] = bp.grey ? kSigma * (T * T) * (T * T) : planck(bp.nu[b], T);
}

// S = (1 - a) B(T) + a J, minus sub (the source an inner sweep takes the change from) when given
__global__ void k_source(BandParams bp, const double *__restrict__ T, const double *__restrict__ J, int64_t N,
                         int nrhs, const double *__restrict__ sub, double *__restrict__ S) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = N * nrhs;
    if (k >= tot) return;
    const double t = T[k];
    for (int b = 0; b < bp.nb; ++b) {
        const int64_t o = (int64_t)b * tot + k;
        const double ab = bp.a[b];
        const double e = bp.grey ? kSigma * (t * t) * (t * t) : planck(bp.nu[b], t);
        const double v = (1.0 - ab) * e + (ab != 0.0 ? ab * J[o] : 0.0);
        S[o] = sub ? v - sub[o] : v;
    }
}

// Partial sums of ||Jn - J||^2 and ||Jn||^2 per (band, rhs) vector; fixed
// assignment of elements to blocks, reduced in a fixed order by k_resid_final.
constexpr int kResidBlocks = 64;

__global__ __launch_bounds__(256) void k_resid_partial(const double *__restrict__ J, const double *__restrict__ Jn,
                                                       int64_t N, double *__restrict__ part) {
    __shared__ double s1[4], s2[4];
    const int vec = blockIdx.y;
    const double *a = J + (int64_t)vec * N, *b = Jn + (int64_t)vec * N;
    double d2 = 0.0, n2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)kResidBlocks * 256) {
        const double d = b[i] - a[i];
        d2 += d * d;
        n2 += b[i] * b[i];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        d2 += __shfl_xor(d2, o, 64);
        n2 += __shfl_xor(n2, o, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { s1[wid] = d2; s2[wid] = n2; }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[((int64_t)vec * kResidBlocks + blockIdx.x) * 2 + 0] = ((s1[0] + s1[1]) + s1[2]) + s1[3];
        part[((int64_t)vec * kResidBlocks + blockIdx.x) * 2 + 1] = ((s2[0] + s2[1]) + s2[2]) + s2[3];
    }
}

__global__ void k_resid_final(const double *__restrict__ part, int nvec, double *__restrict__ out) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvec) return;
    double d2 = 0.0, n2 = 0.0;
    for (int b = 0; b < kResidBlocks; ++b) {
        d2 += part[((int64_t)v * kResidBlocks + b) * 2 + 0];
        n2 += part[((int64_t)v * kResidBlocks + b) * 2 + 1];
    }
    out[2 * v] = d2;
    out[2 * v + 1] = n2;
}

// Per vertex and right-hand side: T solving sum_b c_b (J_b - B_b(T)) = 0,
// c_b = w_b kappa_b (1 - a_b).  Bracketed Newton: f decreases in T,
// f(0) = sum c_b J_b > 0; a step leaving the bracket is replaced by bisection.
// NB > 0 (nb <= NB): each thread reads its bands' c_b and J_b once into
// registers, and the Newton evaluations (every one a pass over the bands) run
// on them; NB = 0 reads them from memory at each evaluation, for any nb.
template <int NB>
__global__ __launch_bounds__(256) void k_newton(BandParams bp, const double *__restrict__ J,
                                                const double *__restrict__ kap, int64_t N, int nrhs,
                                                double *__restrict__ T, unsigned long long *__restrict__ viol) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = N * nrhs;
    if (k >= tot) return;
    const int64_t i = k % N;
    const double Told = T[k];
    double Tn;
    if (bp.grey) {
        const double j = J[k];
        Tn = j > 0.0 ? sqrt(sqrt(j / kSigma)) : 0.0;
    } else if constexpr (NB > 0) {
        double cc[NB], jj[NB];
        for_bands<NB>(bp.nb, [&](int b) {
            cc[b] = bp.w[b] * kap[(int64_t)b * N + i] * (1.0 - bp.a[b]);
            jj[b] = J[(int64_t)b * tot + k];
        });
        Tn = solve_temperature<NB>(bp.nb, Told, [&](int b, double &nu, double &c, double &j) {
            nu = bp.nu[b];
            c = cc[b];
            j = jj[b];
        });
    } else {
        Tn = solve_temperature(bp.nb, Told, [&](int b, double &nu, double &c, double &j) {
            nu = bp.nu[b];
            c = bp.w[b] * kap[(int64_t)b * N + i] * (1.0 - bp.a[b]);
            j = J[(int64_t)b * tot + k];
        });
    }
    // a decrease beyond the rounding of the root (8 units of 2^-52 relative): at the
    // converged state two sweeps' roots may differ in their last bits
    if (Tn < Told * (1.0 - 8.0 * 2.220446049250313e-16)) atomicAdd(viol, 1ull);
    T[k] = Tn;
}

void newton_launch(const BandParams &bp, const double *J, const double *kap, int64_t N, int nrhs, double *T,
                   unsigned long long *viol, hipStream_t s) {
    const unsigned g = (unsigned)((N * nrhs + 255) / 256);
    if (!bp.grey && bp.nb <= 8) k_newton<8><<<g, 256, 0, s>>>(bp, J, kap, N, nrhs, T, viol);
    else if (!bp.grey && bp.nb <= 32) k_newton<32><<<g, 256, 0, s>>>(bp, J, kap, N, nrhs, T, viol);
    else k_newton<0><<<g, 256, 0, s>>>(bp, J, kap, N, nrhs, T, viol);
    HIP_LAUNCH_CHECK();
}

// Captured sweeps of one solve, keyed by what the captured launches bake in:
// the operator, the Newton step, and the buffers (J and Jn swap every sweep).
struct GraphKey {
    int mode;
    bool newton;
    const void *y0, *sub, *J, *Jn, *S;
    int part;   // -1: the whole sweep; 0, 1, 2: before, the matvec, after (timed sweeps)
    bool operator==(const GraphKey &o) const {
        return mode == o.mode && newton == o.newton && y0 == o.y0 && sub == o.sub && J == o.J && Jn == o.Jn &&
               S == o.S && part == o.part;
    }
};

struct GraphCache {
    std::vector<std::pair<GraphKey, hipGraphExec_t>> items;
    hipGraphExec_t find(const GraphKey &k) const {
        for (auto &it : items)
            if (it.first == k) return it.second;
        return nullptr;
    }
    hipGraphExec_t add(const GraphKey &k, hipGraph_t g) {
        hipGraphExec_t ex = nullptr;
        const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) throw Error(RTE_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        items.push_back({k, ex});
        return ex;
    }
    int size() const { return (int)items.size(); }
    ~GraphCache() {
        for (auto &it : items) (void)hipGraphExecDestroy(it.second);
    }
};

void check_desc(const Mesh &m, const HMat &G, const HMat &S, const rte_solve_desc_t &d) {
    RTE_REQUIRE(G.kind == RTE_VOLUME && S.kind == RTE_SURFACE, "solve: need a volume and a surface H-matrix");
    RTE_REQUIRE(G.mesh == &m && S.mesh == &m, "solve: H-matrices were assembled on another mesh");
    RTE_REQUIRE(d.n_bands >= 1 && d.n_bands <= 4096, "solve: n_bands out of range");
    RTE_REQUIRE(G.n_bands == d.n_bands && S.n_bands == d.n_bands, "solve: band count differs from the matrices");
    RTE_REQUIRE(!d.grey || d.n_bands == 1, "solve: the grey formulation has one band");
    RTE_REQUIRE(d.nrhs >= 1 && d.nrhs <= 4096, "solve: nrhs out of range");
    RTE_REQUIRE(d.T_wall != nullptr, "solve: T_wall is required");
    RTE_REQUIRE(d.tol > 0.0 && std::isfinite(d.tol), "solve: tol must be > 0");
    RTE_REQUIRE(d.max_iter >= 1, "solve: max_iter must be >= 1");
    RTE_REQUIRE(d.precision == RTE_FP64 || d.precision == RTE_FP32 || d.precision == RTE_MIXED_BF16,
                "solve: unknown precision");
    RTE_REQUIRE(d.launch == RTE_LAUNCH_STREAM || d.launch == RTE_LAUNCH_GRAPH, "solve: unknown launch mode");
    RTE_REQUIRE(d.time_matvecs == 0 || d.time_matvecs == 1, "solve: time_matvecs must be 0 or 1");
    RTE_REQUIRE(d.precision != RTE_MIXED_BF16 || G.precision == RTE_MIXED_BF16,
                "solve: the mixed-precision iteration needs a volume matrix assembled with RTE_MIXED_BF16");
    if (!d.grey) {
        RTE_REQUIRE(d.nu != nullptr, "solve: nu is required for the band formulation");
        for (int b = 0; b < d.n_bands; ++b) {
            RTE_REQUIRE(std::isfinite(d.nu[b]) && d.nu[b] > 0, "solve: nu must be positive");
            if (b) RTE_REQUIRE(d.nu[b] > d.nu[b - 1], "solve: nu must increase");
            if (d.w) RTE_REQUIRE(std::isfinite(d.w[b]) && d.w[b] >= 0, "solve: w must be >= 0");
        }
    }
    if (d.a)
        for (int b = 0; b < d.n_bands; ++b)
            RTE_REQUIRE(std::isfinite(d.a[b]) && d.a[b] >= 0 && d.a[b] < 1, "solve: a must lie in [0, 1)");
}

}  // namespace

// Graph launch works on a stream of its own (non-blocking, default priority):
// capture is not allowed on the null stream.  It is ordered after the caller's
// stream on entry, and the caller's stream after it on exit.
struct SolveStream {
    hipStream_t user, own = nullptr;
    hipEvent_t ev = nullptr;
    SolveStream(hipStream_t u, bool separate) : user(u) {
        if (!separate) return;
        HIP_CHECK(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
        HIP_CHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        HIP_CHECK(hipEventRecord(ev, user));
        HIP_CHECK(hipStreamWaitEvent(own, ev, 0));
    }
    hipStream_t get() const { return own ? own : user; }
    ~SolveStream() {
        if (!own) return;
        (void)hipEventRecord(ev, own);
        (void)hipStreamWaitEvent(user, ev, 0);
        (void)hipStreamSynchronize(own);
        (void)hipEventDestroy(ev);
        (void)hipStreamDestroy(own);
    }
};

rte_status_t fixed_point_solve(const Mesh &m, const HMat &G, const HMat &S, const rte_solve_desc_t &d,
                               double *T_out, double *J_out, rte_solve_stats_t *st, hipStream_t s_user) {
    check_desc(m, G, S, d);
    SolveStream ss(s_user, d.launch == RTE_LAUNCH_GRAPH);
    const hipStream_t s = ss.get();
    const auto t_start = std::chrono::steady_clock::now();
    const int nb = d.n_bands, nr = d.nrhs;
    const int64_t N = m.N, L = m.L;
    // band constants
    std::vector<double> nu(nb, 1.0), w(nb, 1.0), a(nb, 0.0);
    if (!d.grey) {
        for (int b = 0; b < nb; ++b) nu[b] = d.nu[b];
        if (d.w) {
            for (int b = 0; b < nb; ++b) w[b] = d.w[b];
        } else if (nb > 1) {
            // trapezoid weights on the sorted band frequencies, no tails
            w[0] = 0.5 * (nu[1] - nu[0]);
            w[nb - 1] = 0.5 * (nu[nb - 1] - nu[nb - 2]);
            for (int b = 1; b + 1 < nb; ++b) w[b] = 0.5 * (nu[b + 1] - nu[b - 1]);
        }
    }
    if (d.a)
        for (int b = 0; b < nb; ++b) a[b] = d.a[b];
    std::vector<double> consts;
    consts.insert(consts.end(), nu.begin(), nu.end());
    consts.insert(consts.end(), w.begin(), w.end());
    consts.insert(consts.end(), a.begin(), a.end());
    DevBuf dconst = upload(consts, s);
    BandParams bp{nb, d.grey, dconst.as<double>(), dconst.as<double>() + nb, dconst.as<double>() + 2 * nb};

    const int64_t vecN = N * nr;
    DevBuf Tw(sizeof(double) * L * nr), Q(sizeof(double) * L * nr * nb), SE(sizeof(double) * vecN * nb),
        Sv(sizeof(double) * vecN * nb), J(sizeof(double) * vecN * nb), Jn(sizeof(double) * vecN * nb),
        T(sizeof(double) * vecN), part(sizeof(double) * 2 * kResidBlocks * nb * nr),
        res(sizeof(double) * 2 * nb * nr), viol(sizeof(unsigned long long));
    const int64_t kt = std::max<int64_t>({1, matvec_ws_all(G, nr), matvec_ws_all(S, nr)});
    DevBuf tbuf(sizeof(double) * kt);
    poison(tbuf, s);
    const unsigned gN = (unsigned)((vecN + 255) / 256), gL = (unsigned)((L * nr + 255) / 256);

    // boundary source: Q_b = B_b(T_wall) and S^E_b = S_hat_b Q_b
    permute_gather(S.src_pos.as<int64_t>(), L, nr, L, L, d.T_wall, Tw.as<double>(), s);
    k_emission<<<gL, 256, 0, s>>>(bp, Tw.as<double>(), L, nr, Q.as<double>());
    HIP_LAUNCH_CHECK();
    matvec_launch_all(S, nr, Q.as<double>(), SE.as<double>(), nullptr, tbuf.as<double>(), s);
    if (d.T0) permute_gather(G.tgt_nat.as<int64_t>(), N, nr, N, N, d.T0, T.as<double>(), s);
    else HIP_CHECK(hipMemsetAsync(T.p, 0, T.bytes, s));
    HIP_CHECK(hipMemsetAsync(J.p, 0, J.bytes, s));
    HIP_CHECK(hipMemsetAsync(viol.p, 0, viol.bytes, s));

    hipEvent_t e0, e1, m0, m1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    HIP_CHECK(hipEventCreate(&m0));
    HIP_CHECK(hipEventCreate(&m1));
    float mv_ms = 0.0f;
    // volume-matvec time per operator (time_matvecs): events around the matvec
    // launches; a graph-launched sweep is then captured as three graphs (before,
    // the matvec, after) with the events between them
    const bool mv_events = d.time_matvecs != 0;
    double op_ms[2] = {0.0, 0.0};
    int op_count[2] = {0, 0};
    std::vector<double> rv(2 * nb * nr);
    const bool mixed = d.precision == RTE_MIXED_BF16;
    DevBuf Jacc(mixed ? sizeof(double) * vecN * nb : 0), Sm(mixed ? sizeof(double) * vecN * nb : 0);

    // the parts of a sweep: before the matvec, the matvec, after it
    auto enqueue_pre = [&](const double *sub) {
        k_source<<<gN, 256, 0, s>>>(bp, T.as<double>(), J.as<double>(), N, nr, sub, Sv.as<double>());
        HIP_LAUNCH_CHECK();
    };
    auto enqueue_mv = [&](int mode, const double *y0) {
        matvec_launch_all(G, nr, Sv.as<double>(), Jn.as<double>(), y0, tbuf.as<double>(), s, mode);
    };
    auto enqueue_post = [&](bool newton) {
        k_resid_partial<<<dim3(kResidBlocks, nb * nr), 256, 0, s>>>(J.as<double>(), Jn.as<double>(), N,
                                                                     part.as<double>());
        k_resid_final<<<(nb * nr + 63) / 64, 64, 0, s>>>(part.as<double>(), nb * nr, res.as<double>());
        HIP_LAUNCH_CHECK();
        if (newton)
            newton_launch(bp, Jn.as<double>(), G.kappa_c.as<double>(), N, nr, T.as<double>(),
                          viol.as<unsigned long long>(), s);
    };
    // one sweep: S = S(T, J) (minus Sm when given); Jn = y0 + G S over all bands;
    // residual(J, Jn); T = T(Jn); J <- Jn.  The kernels only (no copies, no
    // memsets), so that a sweep can be captured in a graph.
    auto enqueue = [&](int mode, const double *y0, bool newton, const double *sub, int part_) {
        if (part_ < 0 || part_ == 0) enqueue_pre(sub);
        if (part_ < 0 || part_ == 1) enqueue_mv(mode, y0);
        if (part_ < 0 || part_ == 2) enqueue_post(newton);
    };
    GraphCache graphs;
    auto graph_of = [&](int mode, const double *y0, bool newton, const double *sub, int part_) {
        const GraphKey key{mode, newton, y0, sub, J.p, Jn.p, Sv.p, part_};
        hipGraphExec_t ex = graphs.find(key);
        if (!ex) {
            hipGraph_t g = nullptr;
            HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            try {
                enqueue(mode, y0, newton, sub, part_);
            } catch (...) {
                // leave the stream out of capture mode before reporting
                if (hipStreamEndCapture(s, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
                throw;
            }
            HIP_CHECK(hipStreamEndCapture(s, &g));
            ex = graphs.add(key, g);
        }
        return ex;
    };
    // The first sweep from T = 0 and J = 0 has a zero source (B(0) = 0): G S = 0
    // exactly, so Jn = y0 without streaming the operator (the result is the same
    // bit for bit: the products of zeros add +0)
    bool zero_source = !d.T0;
    int n_hist = 0;
    auto sweep = [&](int mode, const double *y0, bool newton, const double *sub) -> double {
        HIP_CHECK(hipEventRecord(e0, s));
        const bool skip = zero_source;
        zero_source = false;
        if (skip) {
            enqueue_pre(sub);   // S = 0 (the outer step keeps it as its source)
            HIP_CHECK(hipMemcpyAsync(Jn.p, y0, Jn.bytes, hipMemcpyDeviceToDevice, s));
            enqueue_post(newton);
        } else if (d.launch == RTE_LAUNCH_GRAPH && !mv_events) {
            HIP_CHECK(hipGraphLaunch(graph_of(mode, y0, newton, sub, -1), s));
        } else if (d.launch == RTE_LAUNCH_GRAPH) {
            HIP_CHECK(hipGraphLaunch(graph_of(mode, y0, newton, sub, 0), s));
            HIP_CHECK(hipEventRecord(m0, s));
            HIP_CHECK(hipGraphLaunch(graph_of(mode, y0, newton, sub, 1), s));
            HIP_CHECK(hipEventRecord(m1, s));
            HIP_CHECK(hipGraphLaunch(graph_of(mode, y0, newton, sub, 2), s));
        } else {
            enqueue_pre(sub);
            HIP_CHECK(hipEventRecord(m0, s));
            enqueue_mv(mode, y0);
            HIP_CHECK(hipEventRecord(m1, s));
            enqueue_post(newton);
        }
        HIP_CHECK(hipEventRecord(e1, s));
        HIP_CHECK(hipMemcpyAsync(rv.data(), res.p, sizeof(double) * rv.size(), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        float ms = 0.0f;
        HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
        mv_ms += ms;
        if (!skip && (mv_events || d.launch != RTE_LAUNCH_GRAPH)) {
            float mm = 0.0f;
            HIP_CHECK(hipEventElapsedTime(&mm, m0, m1));
            op_ms[mode == kMatvecLow ? 0 : 1] += mm;
            op_count[mode == kMatvecLow ? 0 : 1] += 1;
        }
        double q = 0.0;
        for (int v = 0; v < nb * nr; ++v) {
            const double num = rv[2 * v], den = rv[2 * v + 1];
            q = std::max(q, den > 0.0 ? std::sqrt(num / den) : (num > 0.0 ? INFINITY : 0.0));
        }
        if (d.residuals && n_hist < d.max_iter) d.residuals[n_hist++] = q;
        return q;
    };

    double r = INFINITY;
    int it = 0, outer = 0;
    bool conv = false;
    if (!mixed) {
        while (it < d.max_iter) {
            r = sweep(kMatvecAccurate, SE.as<double>(), true, nullptr);
            ++it;
            std::swap(J, Jn);
            if (!std::isfinite(r)) break;
            if (r <= d.tol) { conv = true; break; }
        }
    } else {
        // FP64 defect correction around sweeps on the BF16-hi operator G_lo:
        //   outer: J_acc = S^E + G S_m, S_m = S(T), with the hi+lo operator and FP64
        //          accumulation; its relative change is the residual that decides
        //          convergence;
        //   inner: J <- J_acc + G_lo (S(T(J)) - S_m), whose fixed point solves
        //          J = S^E + (G - G_lo) S_m + G_lo S(T(J)); BF16 only ever meets the
        //          change of the source, until the change of J is far below the outer one.
        while (it < d.max_iter) {
            r = sweep(kMatvecAccurate, SE.as<double>(), false, nullptr);
            ++it;
            ++outer;
            if (!std::isfinite(r)) break;
            std::swap(Sm, Sv);   // S_m = the source of this outer step
            HIP_CHECK(hipMemcpyAsync(Jacc.p, Jn.p, Jacc.bytes, hipMemcpyDeviceToDevice, s));
            newton_launch(bp, Jn.as<double>(), G.kappa_c.as<double>(), N, nr, T.as<double>(),
                          viol.as<unsigned long long>(), s);
            std::swap(J, Jn);
            if (r <= d.tol) { conv = true; break; }
            const double inner_tol = std::max(2e-3 * r, 0.25 * d.tol);
            double r_prev = r;
            for (int k = 0; k < 200 && it < d.max_iter; ++k) {
                const double ri = sweep(kMatvecLow, Jacc.as<double>(), true, Sm.as<double>());
                ++it;
                std::swap(J, Jn);
                if (!std::isfinite(ri) || ri <= inner_tol) break;
                // the sweeps contract J's change by rho = ri / r_prev each: when the
                // next change, rho ri, is predicted within half the tolerance, the
                // defect step (which decides convergence) comes next
                const double rho = ri / r_prev;
                if (rho < 1.0 && rho * ri <= 0.5 * d.tol) break;
                r_prev = ri;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(m0);
    (void)hipEventDestroy(m1);
    if (T_out) permute_scatter(G.tgt_nat.as<int64_t>(), N, nr, N, N, T.as<double>(), T_out, s);
    if (J_out)
        for (int b = 0; b < nb; ++b)
            // J_out is [nrhs][nb][N]: rhs stride nb*N, band offset b*N
            permute_scatter(G.tgt_nat.as<int64_t>(), N, nr, N, (int64_t)nb * N, J.as<double>() + (int64_t)b * vecN,
                            J_out + (int64_t)b * N, s);
    unsigned long long nviol = 0;
    HIP_CHECK(hipMemcpyAsync(&nviol, viol.p, sizeof(nviol), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (st) {
        st->iterations = it;
        st->outer_steps = outer;
        st->residual = r;
        st->monotone_violations = (int64_t)nviol;
        st->ms_matvec = (mv_events || d.launch != RTE_LAUNCH_GRAPH) ? op_ms[0] + op_ms[1] : mv_ms;
        st->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
        st->graphs = graphs.size();
        const bool timed = mv_events || d.launch != RTE_LAUNCH_GRAPH;
        st->ms_matvec_low = timed ? op_ms[0] : -1.0;
        st->matvecs_low = op_count[0];
        st->ms_matvec_acc = timed ? op_ms[1] : -1.0;
        st->matvecs_acc = op_count[1];
    }
    if (!std::isfinite(r)) throw Error(RTE_E_INTERNAL, "solve: the residual is not finite");
    return conv ? RTE_OK : RTE_E_NOT_CONVERGED;
}

}  // namespace rte
