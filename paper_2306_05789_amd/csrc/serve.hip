// Request server: fixed-point solves of many requests on resident meshes,
// continuously batched (the serving pattern around the fixed point of
// Section "Fixed Point Iterations").
//
// A request names a resident mesh, a subset of the band catalogue, a kappa
// multiplier per band (of the mesh's base field kappa(x)) and wall
// temperatures.  The absorption of a band is the base field times a level of
// the ladder m_l = 10^(l / levels_per_decade), the multiplier snapped to the
// nearest level in log space (ties to the lower level), following the
// paper's use of a few piecewise-constant absorption values per band; the
// snapped value defines the request.  Operators (volume G and boundary source
// S of one (mesh, level)) are assembled on first use, shared by every band
// of every request at that level, kept while the HBM budget allows and
// evicted least recently used when not in use.
//
// Requests wait in arrival order.  A waiting request whose operators are all
// resident is admitted as soon as its state fits the budget, in arrival order
// among such requests (one with missing operators does not hold up the ones
// behind it).  A background thread on its own stream assembles the missing
// operators of the oldest few waiting requests; only the oldest may evict
// unused operators to make room, the others are assembled into free room
// only, so the oldest request always makes progress.  Each step runs one
// sweep of every admitted request: the (request, band) columns
// that share an operator go through one multi-right-hand-side matvec, then
// one launch updates every request's temperatures.  A request that converges
// (or reaches its iteration cap) retires at once and frees its slot; the
// others keep iterating.  With mixed-precision storage every request runs the
// defect-corrected iteration of the single solve (FP64 defect steps on the hi
// + lo operator, inner sweeps on the BF16-hi one) with its own phase; its
// columns are reduced in a fixed order whatever else shares a launch, so a
// request gets the same numbers alone and in a mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <exception>
#include <condition_variable>
#include <map>
#include <mutex>
#include <thread>

#include "kernels.h"
#include "physics.h"
#include "serve.h"

namespace rte {

namespace {

constexpr int kSrvResidBlocks = 32;

// one (request, band) column of a sweep
struct SrvCol {
    double nu;
    double a;            // scattering coefficient of the band (eq. eqS)
    const double *T;     // request temperatures [N], cluster order
    double *Sm;          // source of the last defect step (mixed), else null
    const double *y0;    // S^E (plain sweep, defect step) or J_acc (inner sweep)
    double *J;           // radiation [N]
    double *Jacc;        // J_acc, written on defect steps (mixed), else null
    int32_t inner;       // inner sweep: the operand is S(T) - S_m
    int32_t save;        // defect step of the mixed iteration: keep S(T) and J_acc
};

// x[c] = S = (1 - a) B_nu(T) + a J (minus S_m on inner sweeps); a defect step
// keeps S in S_m
__global__ void k_srv_x(const SrvCol *__restrict__ cols, int64_t N, double *__restrict__ x) {
    const int c = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const SrvCol col = cols[c];
    const double e = planck(col.nu, col.T[i]);
    const double s = col.a != 0.0 ? (1.0 - col.a) * e + col.a * col.J[i] : e;
    x[(int64_t)c * N + i] = col.inner ? s - col.Sm[i] : s;
    if (col.save) col.Sm[i] = s;
}

// J_new = y0 + y; fixed-order partial sums of |J_new - J|^2 and |J_new|^2;
// J <- J_new (and J_acc <- J_new on defect steps)
__global__ __launch_bounds__(256) void k_srv_update(const SrvCol *__restrict__ cols, int64_t N,
                                                    const double *__restrict__ y, double *__restrict__ part) {
    __shared__ double s1[4], s2[4];
    const int c = blockIdx.y;
    const SrvCol col = cols[c];
    double d2 = 0.0, n2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)kSrvResidBlocks * 256) {
        const double jn = col.y0[i] + y[(int64_t)c * N + i];
        const double d = jn - col.J[i];
        d2 += d * d;
        n2 += jn * jn;
        col.J[i] = jn;
        if (col.save) col.Jacc[i] = jn;
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
        part[((int64_t)c * kSrvResidBlocks + blockIdx.x) * 2 + 0] = ((s1[0] + s1[1]) + s1[2]) + s1[3];
        part[((int64_t)c * kSrvResidBlocks + blockIdx.x) * 2 + 1] = ((s2[0] + s2[1]) + s2[2]) + s2[3];
    }
}

__global__ void k_srv_resid(const double *__restrict__ part, int ncol, double *__restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncol) return;
    double d2 = 0.0, n2 = 0.0;
    for (int b = 0; b < kSrvResidBlocks; ++b) {
        d2 += part[((int64_t)c * kSrvResidBlocks + b) * 2 + 0];
        n2 += part[((int64_t)c * kSrvResidBlocks + b) * 2 + 1];
    }
    out[2 * c] = d2;
    out[2 * c + 1] = n2;
}

// per request: its bands in the band table [b0, b0 + nb)
struct SrvNewt {
    double *T;
    const double *kap;   // base kappa at the vertices, cluster order [N]
    int64_t N;
    int32_t nb, b0;
};
struct SrvBand {
    double nu, w, mult, a;   // frequency, catalogue weight, snapped kappa multiplier, scattering
    const double *J;
};

__global__ void k_srv_newton(const SrvNewt *__restrict__ reqs, const SrvBand *__restrict__ bands) {
    const SrvNewt r = reqs[blockIdx.y];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= r.N) return;
    const double k = r.kap[i];
    r.T[i] = solve_temperature(r.nb, r.T[i], [&](int b, double &nu, double &c, double &j) {
        const SrvBand &bd = bands[r.b0 + b];
        nu = bd.nu;
        c = bd.w * bd.mult * k * (1.0 - bd.a);
        j = bd.J[i];
    });
}

// Q = B_nu(T_wall) for one band
__global__ void k_srv_emission(double nu, const double *__restrict__ Tw, int64_t L, double *__restrict__ Q) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < L) Q[i] = planck(nu, Tw[i]);
}

__global__ void k_scale(const double *__restrict__ in, double a, int64_t n, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a * in[i];
}

template <typename T>
void grow(DevBuf &b, int64_t count, hipStream_t s) {
    if ((int64_t)b.bytes < count * (int64_t)sizeof(T)) {
        b.alloc(sizeof(T) * (size_t)count);
        poison(b, s);
    }
}

// Pinned staging for the small per-step tables.
struct Pinned {
    void *p = nullptr;
    size_t bytes = 0;
    void reserve(size_t b) {
        if (b <= bytes) return;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        HIP_CHECK(hipHostMalloc(&p, b, hipHostMallocDefault));
        bytes = b;
    }
    ~Pinned() {
        if (p) (void)hipHostFree(p);
    }
};

}  // namespace

struct SrvOp {
    int mesh = 0, level = 0;
    std::unique_ptr<rte_hmat> G, S;
    int64_t bytes = 0;
    int64_t reserved = 0;   // bytes held for it while it was being assembled
    double ms = 0.0;        // assembly wall time
    int users = 0;
    uint64_t used = 0;
};

struct SrvMesh {
    Mesh mesh;
    DevBuf kappa;          // base field, natural order [N]
    DevBuf kap_c;          // base field, cluster order [N] (after the first operator)
    DevBuf tgt_nat;        // volume cluster position -> vertex
    DevBuf src_pos;        // surface cluster position -> position in the caller's wall vector
    bool have_order = false;
    std::mutex order_mu;     // the assembler that builds the first operator sets the tables above
    int64_t est_bytes = 0;   // operator bytes of one level (estimate, then the largest seen)
};

struct SrvReq {
    int64_t id = 0;
    int mesh = 0;
    std::vector<int> bands, levels;
    std::vector<double> a;      // scattering coefficient per band
    std::vector<SrvOp *> ops;   // per band
    double tol = 1e-6;
    int max_iter = 1000;
    int state = RTE_REQ_PENDING;
    DevBuf Tw;                  // [L], natural emitting order
    DevBuf st;                  // T [N] | J, SE, Jacc, Sm [nb][N]
    DevBuf out;                 // T [N], natural order, once finished
    int64_t state_bytes = 0;
    int phase = 0;              // 0: plain sweep or defect step; 1: inner sweep
    int inner = 0, iterations = 0, outer = 0;
    double residual = INFINITY, inner_tol = 0.0;
    bool converged = false;
    double *T() const { return st.as<double>(); }
    double *J(int64_t N, int b) const { return st.as<double>() + N + (int64_t)b * N; }
    double *SE(int64_t N, int b) const { return st.as<double>() + N + (int64_t)(bands.size() + b) * N; }
    double *Jacc(int64_t N, int b) const { return st.as<double>() + N + (int64_t)(2 * bands.size() + b) * N; }
    double *Sm(int64_t N, int b) const { return st.as<double>() + N + (int64_t)(3 * bands.size() + b) * N; }
};

struct Server {
    // requests scanned for admission in one pass, and the oldest waiting
    // requests whose missing operators are assembled ahead of their admission
    static constexpr int kWindow = 256, kLookahead = 4;

    rte_server_desc_t desc{};
    std::vector<double> nu, w;   // catalogue
    hipStream_t user = nullptr;  // the caller's stream (inputs are ordered after it)
    hipStream_t s = nullptr;     // sweeps (the server's own, non-blocking, default priority)
    // assemblers: each builds one operator at a time (the volume one on as[w],
    // the boundary-source one concurrently on as2[w]), so two operators are
    // assembled at once and one's ACA tail and host work overlap the other's
    static constexpr int kAssemblers = 2;
    hipStream_t as[kAssemblers] = {}, as2[kAssemblers] = {};
    int device = 0;
    std::vector<std::unique_ptr<SrvMesh>> meshes;
    std::vector<std::unique_ptr<SrvOp>> ops;   // resident operators (main thread only)
    std::map<int64_t, std::unique_ptr<SrvReq>> reqs;
    std::deque<SrvReq *> pending;
    std::vector<SrvReq *> active;
    int64_t next_id = 1;
    uint64_t clock = 0;
    int64_t resident = 0;        // operator and request-state bytes held
    int64_t reserved = 0;        // estimated bytes of the operators being assembled
    rte_server_stats_t stats{};
    // per-step device and pinned buffers
    DevBuf x, y, ws, cols, part, res, newt, bandt, q;
    Pinned hcols, hres, hnewt, hband;
    // the assembler thread
    struct Job { SrvMesh *m; int mesh, level; int64_t reserved; };
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable cv, done_cv;
    std::deque<Job> jobs;                        // waiting
    std::vector<std::pair<int, int>> inflight;   // queued or running (mesh, level)
    std::vector<std::unique_ptr<SrvOp>> built;   // finished, not yet published
    std::string worker_error;
    bool stopping = false;

    bool mixed() const { return desc.precision == RTE_MIXED_BF16; }

    rte_hmat_opts_t opts(int kind) const {
        rte_hmat_opts_t o{};
        o.kind = kind;
        o.dense = 0;
        o.leaf_size = desc.leaf_size;
        o.eta = desc.eta;
        o.aca_eps = desc.aca_eps;
        o.precision = desc.precision;
        o.recompress = kind == RTE_VOLUME ? desc.recompress : 0;
        return o;
    }

    // estimate of one level's operator bytes from the plans (no assembly):
    // dense leaves in full, admissible blocks at the first pass's rank cap
    // (a block stored dense after its ACA can exceed it; the largest level
    // assembled so far replaces the estimate)
    int64_t bound_bytes(const Mesh &m) const {
        const int64_t esz = mixed() ? 4 : 8;
        int64_t e = 0;
        for (int kind : {RTE_VOLUME, RTE_SURFACE}) {
            auto P = mesh_plan(m, opts(kind));
            for (auto &b : P->dense) e += (b.t1 - b.t0) * (b.s1 - b.s0);
            for (auto &b : P->lowrank) {
                const int64_t mm = b.t1 - b.t0, nn = b.s1 - b.s0;
                const int64_t cap = std::min<int64_t>(mm * nn / (mm + nn), kAcaMaxRank);
                e += std::min(mm * nn, cap * (mm + nn));
            }
        }
        return e * esz * 5 / 4;   // padding of the stored layouts
    }

    static int snap(double mult, int per_decade) {
        // nearest level in log space, ties to the lower level
        return (int)std::ceil(per_decade * std::log10(mult) - 0.5);
    }

    SrvOp *find_op(int mesh, int level) {
        for (auto &o : ops)
            if (o->mesh == mesh && o->level == level) return o.get();
        return nullptr;
    }
    bool in_flight(int mesh, int level) {
        return std::find(inflight.begin(), inflight.end(), std::make_pair(mesh, level)) != inflight.end();
    }

    // ------------------------------------------------ the assembler thread
    // Operators of one (mesh, level) on the assembler's stream; touches no
    // server state but the mesh's cluster-order tables on its first operator
    // (no request of that mesh can be admitted before it is published).
    std::unique_ptr<SrvOp> build_op(SrvMesh &M, int mi, int level, hipStream_t as, hipStream_t as2) {
        const auto t0 = std::chrono::steady_clock::now();
        DevBuf kap(sizeof(double) * (size_t)M.mesh.N);
        const double mult = std::pow(10.0, (double)level / desc.levels_per_decade);
        k_scale<<<(unsigned)((M.mesh.N + 255) / 256), 256, 0, as>>>(M.kappa.as<double>(), mult, M.mesh.N,
                                                                    kap.as<double>());
        HIP_LAUNCH_CHECK();
        auto op = std::make_unique<SrvOp>();
        op->mesh = mi;
        op->level = level;
        // G and S are independent: S is assembled by a second thread on its own
        // stream (ordered after the scaling), G on this one
        hipEvent_t ready;
        HIP_CHECK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
        HIP_CHECK(hipEventRecord(ready, as));
        HIP_CHECK(hipStreamWaitEvent(as2, ready, 0));
        std::unique_ptr<rte_hmat> Sop;
        std::exception_ptr serr;
        std::thread ts([&] {
            try {
                HIP_CHECK(hipSetDevice(device));
                Sop = assemble_hmat(M.mesh, mesh_plan(M.mesh, opts(RTE_SURFACE)), opts(RTE_SURFACE), 1, kap.as<double>(),
                                     as2);
            } catch (...) {
                serr = std::current_exception();
            }
        });
        std::exception_ptr gerr;
        try {
            op->G = assemble_hmat(M.mesh, mesh_plan(M.mesh, opts(RTE_VOLUME)), opts(RTE_VOLUME), 1, kap.as<double>(), as);
        } catch (...) {
            gerr = std::current_exception();
        }
        ts.join();
        (void)hipEventDestroy(ready);
        if (gerr) std::rethrow_exception(gerr);
        if (serr) std::rethrow_exception(serr);
        op->S = std::move(Sop);
        op->bytes = op->G->h.stats.bytes + op->S->h.stats.bytes;
        std::lock_guard<std::mutex> order_lock(M.order_mu);   // another assembler may build this mesh too
        if (!M.have_order) {
            M.tgt_nat.alloc(sizeof(int64_t) * (size_t)M.mesh.N);
            HIP_CHECK(hipMemcpyAsync(M.tgt_nat.p, op->G->h.tgt_nat.p, M.tgt_nat.bytes, hipMemcpyDeviceToDevice, as));
            M.src_pos.alloc(sizeof(int64_t) * (size_t)M.mesh.L);
            HIP_CHECK(hipMemcpyAsync(M.src_pos.p, op->S->h.src_pos.p, M.src_pos.bytes, hipMemcpyDeviceToDevice, as));
            M.kap_c.alloc(sizeof(double) * (size_t)M.mesh.N);
            permute_gather(M.tgt_nat.as<int64_t>(), M.mesh.N, 1, M.mesh.N, M.mesh.N, M.kappa.as<double>(),
                           M.kap_c.as<double>(), as);
            HIP_CHECK(hipStreamSynchronize(as));   // the tables are complete before another op can be published
            M.have_order = true;
        }
        HIP_CHECK(hipStreamSynchronize(as));   // kap is released on return
        op->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return op;
    }

    void worker_loop(int w) {
        (void)hipSetDevice(device);
        for (;;) {
            Job j;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return stopping || !jobs.empty(); });
                if (stopping) return;
                j = jobs.front();
                jobs.pop_front();
            }
            std::unique_ptr<SrvOp> op;
            std::string err;
            try {
                op = build_op(*j.m, j.mesh, j.level, as[w], as2[w]);
                op->reserved = j.reserved;
            } catch (const std::exception &e) {
                err = e.what();
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                if (op) built.push_back(std::move(op));
                else {
                    worker_error = err.empty() ? "assembly failed" : err;
                    inflight.erase(std::remove(inflight.begin(), inflight.end(), std::make_pair(j.mesh, j.level)),
                                   inflight.end());
                    reserved -= j.reserved;
                }
            }
            done_cv.notify_all();
        }
    }

    // move finished operators into the resident set (main thread)
    void publish() {
        std::vector<std::unique_ptr<SrvOp>> got;
        std::string err;
        {
            std::lock_guard<std::mutex> lk(mu);
            got.swap(built);
            err.swap(worker_error);
            for (auto &o : got) {
                inflight.erase(std::remove(inflight.begin(), inflight.end(), std::make_pair(o->mesh, o->level)),
                               inflight.end());
                reserved -= o->reserved;
            }
        }
        for (auto &o : got) {
            resident += o->bytes;
            SrvMesh &M = *meshes[o->mesh];
            M.est_bytes = std::max(M.est_bytes, o->bytes);
            stats.assembled += 1;
            stats.assemble_ms += o->ms;
            o->used = ++clock;
            ops.push_back(std::move(o));
        }
        if (!err.empty()) throw Error(RTE_E_INTERNAL, "server: " + err);
    }

    void enqueue(int mi, int level, int64_t est) {
        {
            std::lock_guard<std::mutex> lk(mu);
            jobs.push_back({meshes[mi].get(), mi, level, est});
            inflight.push_back({mi, level});
            reserved += est;
        }
        cv.notify_one();
    }

    bool busy() {
        std::lock_guard<std::mutex> lk(mu);
        return !inflight.empty();
    }

    // ------------------------------------------------ budget
    // Evict unused operators (least recently used first, those the oldest
    // waiting requests need last) until `bytes` more fit; false if they do not.
    bool make_room(int64_t bytes, const std::vector<std::pair<int, int>> &wanted) {
        auto held = [&] {
            std::lock_guard<std::mutex> lk(mu);
            return resident + reserved;
        };
        while (held() + bytes > desc.hbm_budget) {
            SrvOp *v = nullptr;
            bool v_wanted = true;
            for (auto &o : ops) {
                if (o->users) continue;
                const bool wn = std::find(wanted.begin(), wanted.end(), std::make_pair(o->mesh, o->level)) !=
                                wanted.end();
                if (!v || (v_wanted && !wn) || (v_wanted == wn && o->used < v->used)) {
                    v = o.get();
                    v_wanted = wn;
                }
            }
            if (!v) return false;
            resident -= v->bytes;
            stats.evicted += 1;
            ops.erase(std::remove_if(ops.begin(), ops.end(), [&](const std::unique_ptr<SrvOp> &o) { return o.get() == v; }),
                      ops.end());
        }
        return true;
    }

    bool fits_now(int64_t bytes) {
        std::lock_guard<std::mutex> lk(mu);
        return resident + reserved + bytes <= desc.hbm_budget;
    }

    int64_t state_bytes(const SrvReq &r) const {
        const int64_t N = meshes[r.mesh]->mesh.N;
        return (int64_t)sizeof(double) * N * (2 + 4 * (int64_t)r.bands.size());
    }

    std::vector<int> distinct_levels(const SrvReq &r) const {
        std::vector<int> l = r.levels;
        std::sort(l.begin(), l.end());
        l.erase(std::unique(l.begin(), l.end()), l.end());
        return l;
    }

    // admit a request whose operators are all resident
    void admit(SrvReq &r) {
        SrvMesh &M = *meshes[r.mesh];
        for (int l : distinct_levels(r)) find_op(r.mesh, l)->users += 1;
        const int nb = (int)r.bands.size();
        const int64_t N = M.mesh.N, L = M.mesh.L;
        r.ops.clear();
        for (int b = 0; b < nb; ++b) {
            SrvOp *o = find_op(r.mesh, r.levels[b]);
            RTE_REQUIRE(o, "server: operator of an admitted request is missing");
            o->used = ++clock;
            r.ops.push_back(o);
        }
        r.state_bytes = state_bytes(r);
        r.st.alloc((size_t)r.state_bytes);
        HIP_CHECK(hipMemsetAsync(r.st.p, 0, r.st.bytes, s));   // T = 0, J = 0
        resident += r.state_bytes;
        // S^E_b = S_hat Q_b, Q_b = B_nu(T_wall), wall values in surface cluster order
        grow<double>(q, 2 * L, s);
        permute_gather(M.src_pos.as<int64_t>(), L, 1, L, L, r.Tw.as<double>(), q.as<double>() + L, s);
        for (int b = 0; b < nb; ++b) {
            k_srv_emission<<<(unsigned)((L + 255) / 256), 256, 0, s>>>(nu[r.bands[b]], q.as<double>() + L, L,
                                                                       q.as<double>());
            HIP_LAUNCH_CHECK();
            const HMat &S = r.ops[b]->S->h;
            grow<double>(ws, matvec_ws_all(S, 1), s);
            matvec_launch_all(S, 1, q.as<double>(), r.SE(N, b), nullptr, ws.as<double>(), s, kMatvecAccurate);
        }
        r.state = RTE_REQ_ACTIVE;
        r.phase = 0;
        active.push_back(&r);
    }

    // One admission pass.  (1) In arrival order, every waiting request whose
    // operators are resident is admitted while slots and the budget allow.
    // (2) The missing operators of the oldest waiting requests are queued for
    // the assembler, within the budget (unused operators are evicted, those
    // these requests need last).  With nothing running and nothing being
    // assembled, the oldest request is served even beyond the budget, so the
    // server always makes progress.
    void admission() {
        publish();
        std::vector<std::pair<int, int>> wanted;
        {
            int look = 0;
            for (SrvReq *r : pending) {
                if (look++ >= kLookahead) break;
                for (int l : r->levels) wanted.push_back({r->mesh, l});
            }
        }
        int scanned = 0;
        for (auto it = pending.begin(); it != pending.end() && (int)active.size() < desc.max_active &&
                                        scanned < kWindow;
             ++scanned) {
            SrvReq &r = **it;
            bool ready = true;
            for (int l : r.levels) ready = ready && find_op(r.mesh, l) != nullptr;
            if (!ready) {
                ++it;
                continue;
            }
            // pin this request's operators while room is made for its state
            std::vector<SrvOp *> mine;
            for (int l : distinct_levels(r)) {
                SrvOp *o = find_op(r.mesh, l);
                o->users += 1;
                mine.push_back(o);
            }
            const bool fits = make_room(state_bytes(r), wanted);
            for (SrvOp *o : mine) o->users -= 1;
            if (!fits && !(active.empty() && !busy())) break;
            if (!fits) stats.over_budget += 1;
            admit(r);
            it = pending.erase(it);
        }
        // assembly ahead of admission for the oldest waiting requests.  Only
        // the oldest may evict (its resident operators pinned meanwhile, so
        // making room for its missing levels never evicts the ones it already
        // has); the others are assembled only into free room.  Letting them
        // evict too can livelock: two requests that together exceed the budget
        // evict each other's operators without end.
        int look = 0;
        for (SrvReq *r : pending) {
            const bool head = look == 0;
            if (look++ >= kLookahead) break;
            const SrvMesh &M = *meshes[r->mesh];
            std::vector<SrvOp *> pin;
            if (head)
                for (int l : distinct_levels(*r))
                    if (SrvOp *o = find_op(r->mesh, l)) { o->users += 1; pin.push_back(o); }
            bool stop = false;
            for (int l : distinct_levels(*r)) {
                if (find_op(r->mesh, l) || in_flight(r->mesh, l)) continue;
                const bool room = head ? make_room(M.est_bytes, wanted) : fits_now(M.est_bytes);
                if (!room) {
                    if (!(head && active.empty() && !busy())) { stop = true; break; }
                    stats.over_budget += 1;
                }
                enqueue(r->mesh, l, M.est_bytes);
            }
            for (SrvOp *o : pin) o->users -= 1;
            if (stop) return;
        }
    }

    void retire(SrvReq &r) {
        const SrvMesh &M = *meshes[r.mesh];
        r.out.alloc(sizeof(double) * (size_t)M.mesh.N);
        permute_scatter(M.tgt_nat.as<int64_t>(), M.mesh.N, 1, M.mesh.N, M.mesh.N, r.T(), r.out.as<double>(), s);
        HIP_CHECK(hipStreamSynchronize(s));
        for (int l : distinct_levels(r)) {
            SrvOp *o = find_op(r.mesh, l);
            o->users -= 1;
            o->used = ++clock;
        }
        resident -= r.state_bytes;
        r.st.release();
        r.state = RTE_REQ_DONE;
        stats.completed += 1;
    }
    // one sweep of every active request
    void sweep() {
        // columns grouped by (operator, inner) in a fixed order
        struct Group { SrvOp *op; int inner; std::vector<SrvCol> cols; };
        std::vector<Group> groups;
        std::vector<std::pair<SrvReq *, std::vector<int>>> colidx;   // per request: its column numbers
        for (SrvReq *r : active) {
            const int64_t N = meshes[r->mesh]->mesh.N;
            const bool inner = mixed() && r->phase == 1;
            const bool save = mixed() && r->phase == 0;
            for (int b = 0; b < (int)r->bands.size(); ++b) {
                SrvCol c{nu[r->bands[b]], r->a[b], r->T(), mixed() ? r->Sm(N, b) : nullptr,
                         inner ? r->Jacc(N, b) : r->SE(N, b), r->J(N, b), mixed() ? r->Jacc(N, b) : nullptr,
                         inner ? 1 : 0, save ? 1 : 0};
                auto it = std::find_if(groups.begin(), groups.end(),
                                       [&](const Group &g) { return g.op == r->ops[b] && g.inner == (int)inner; });
                if (it == groups.end()) {
                    groups.push_back({r->ops[b], (int)inner, {}});
                    it = groups.end() - 1;
                }
                it->cols.push_back(c);
            }
        }
        std::vector<SrvCol> all;
        std::vector<int64_t> goff;
        for (auto &g : groups) {
            goff.push_back((int64_t)all.size());
            all.insert(all.end(), g.cols.begin(), g.cols.end());
        }
        const int ncol = (int)all.size();
        // the column of (request, band) in `all`
        std::map<std::pair<SrvReq *, int>, int> where;
        {
            std::vector<int> fill(groups.size(), 0);
            for (SrvReq *r : active) {
                const bool inner = mixed() && r->phase == 1;
                for (int b = 0; b < (int)r->bands.size(); ++b) {
                    size_t gi = 0;
                    while (!(groups[gi].op == r->ops[b] && groups[gi].inner == (int)inner)) ++gi;
                    where[{r, b}] = (int)(goff[gi] + fill[gi]++);
                }
            }
        }
        hcols.reserve(sizeof(SrvCol) * ncol);
        std::memcpy(hcols.p, all.data(), sizeof(SrvCol) * ncol);
        grow<SrvCol>(cols, ncol, s);
        HIP_CHECK(hipMemcpyAsync(cols.p, hcols.p, sizeof(SrvCol) * ncol, hipMemcpyHostToDevice, s));
        grow<double>(part, (int64_t)ncol * kSrvResidBlocks * 2, s);
        grow<double>(res, 2 * (int64_t)ncol, s);
        const auto t0 = std::chrono::steady_clock::now();
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            const Group &g = groups[gi];
            const HMat &G = g.op->G->h;
            const int64_t N = meshes[g.op->mesh]->mesh.N;
            const int nc = (int)g.cols.size();
            grow<double>(x, (int64_t)nc * N, s);
            grow<double>(y, (int64_t)nc * N, s);
            grow<double>(ws, matvec_ws_all(G, nc), s);
            const SrvCol *dc = cols.as<SrvCol>() + goff[gi];
            k_srv_x<<<dim3((unsigned)((N + 255) / 256), (unsigned)nc), 256, 0, s>>>(dc, N, x.as<double>());
            HIP_LAUNCH_CHECK();
            matvec_launch_all(G, nc, x.as<double>(), y.as<double>(), nullptr, ws.as<double>(), s,
                              g.inner ? kMatvecLow : kMatvecAccurate);
            k_srv_update<<<dim3(kSrvResidBlocks, (unsigned)nc), 256, 0, s>>>(
                dc, N, y.as<double>(), part.as<double>() + goff[gi] * kSrvResidBlocks * 2);
            HIP_LAUNCH_CHECK();
            g.op->used = ++clock;
        }
        k_srv_resid<<<(ncol + 63) / 64, 64, 0, s>>>(part.as<double>(), ncol, res.as<double>());
        HIP_LAUNCH_CHECK();
        // temperatures of every active request in one launch
        std::vector<SrvNewt> nt;
        std::vector<SrvBand> bt;
        int64_t maxN = 0;
        for (SrvReq *r : active) {
            const SrvMesh &M = *meshes[r->mesh];
            nt.push_back({r->T(), M.kap_c.as<double>(), M.mesh.N, (int32_t)r->bands.size(), (int32_t)bt.size()});
            for (int b = 0; b < (int)r->bands.size(); ++b)
                bt.push_back({nu[r->bands[b]], w[r->bands[b]], std::pow(10.0, (double)r->levels[b] / desc.levels_per_decade),
                              r->a[b], r->J(M.mesh.N, b)});
            maxN = std::max(maxN, M.mesh.N);
        }
        hnewt.reserve(sizeof(SrvNewt) * nt.size());
        hband.reserve(sizeof(SrvBand) * bt.size());
        std::memcpy(hnewt.p, nt.data(), sizeof(SrvNewt) * nt.size());
        std::memcpy(hband.p, bt.data(), sizeof(SrvBand) * bt.size());
        grow<SrvNewt>(newt, (int64_t)nt.size(), s);
        grow<SrvBand>(bandt, (int64_t)bt.size(), s);
        HIP_CHECK(hipMemcpyAsync(newt.p, hnewt.p, sizeof(SrvNewt) * nt.size(), hipMemcpyHostToDevice, s));
        HIP_CHECK(hipMemcpyAsync(bandt.p, hband.p, sizeof(SrvBand) * bt.size(), hipMemcpyHostToDevice, s));
        k_srv_newton<<<dim3((unsigned)((maxN + 255) / 256), (unsigned)nt.size()), 256, 0, s>>>(newt.as<SrvNewt>(),
                                                                                                bandt.as<SrvBand>());
        HIP_LAUNCH_CHECK();
        hres.reserve(sizeof(double) * 2 * ncol);
        HIP_CHECK(hipMemcpyAsync(hres.p, res.p, sizeof(double) * 2 * ncol, hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        stats.sweep_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        stats.steps += 1;
        stats.columns += ncol;
        const double *rv = static_cast<const double *>(hres.p);
        // per-request convergence, the state machine of the single solve
        std::vector<SrvReq *> still;
        for (SrvReq *r : active) {
            double q = 0.0;
            for (int b = 0; b < (int)r->bands.size(); ++b) {
                const int c = where[{r, b}];
                const double num = rv[2 * c], den = rv[2 * c + 1];
                q = std::max(q, den > 0.0 ? std::sqrt(num / den) : (num > 0.0 ? INFINITY : 0.0));
            }
            r->iterations += 1;
            bool finished = false;
            if (!std::isfinite(q)) {
                finished = true;
            } else if (!mixed() || r->phase == 0) {
                r->residual = q;
                if (mixed()) r->outer += 1;
                if (q <= r->tol) {
                    r->converged = true;
                    finished = true;
                } else if (mixed()) {
                    r->phase = 1;
                    r->inner = 0;
                    r->inner_tol = std::max(2e-3 * q, 0.25 * r->tol);
                }
            } else {
                r->inner += 1;
                if (q <= r->inner_tol || r->inner >= 200) r->phase = 0;
            }
            if (!finished && r->iterations >= r->max_iter) finished = true;
            if (finished) retire(*r);
            else still.push_back(r);
        }
        active.swap(still);
    }

    void step() {
        HIP_CHECK(hipSetDevice(device));
        admission();
        if (!active.empty()) {
            sweep();
        } else if (!pending.empty()) {
            // nothing to sweep: wait (briefly) for the assembler
            std::unique_lock<std::mutex> lk(mu);
            done_cv.wait_for(lk, std::chrono::milliseconds(5), [&] { return !built.empty() || !worker_error.empty(); });
        }
        stats.resident_bytes = resident;
        stats.operators = (int64_t)ops.size();
    }

    ~Server() {
        {
            std::lock_guard<std::mutex> lk(mu);
            stopping = true;
        }
        cv.notify_all();
        for (auto &t : workers)
            if (t.joinable()) t.join();
        if (s) (void)hipStreamSynchronize(s);
        for (int w = 0; w < kAssemblers; ++w) {
            if (as[w]) (void)hipStreamSynchronize(as[w]);
            if (as2[w]) (void)hipStreamSynchronize(as2[w]);
        }
        reqs.clear();
        ops.clear();
        built.clear();
        if (s) (void)hipStreamDestroy(s);
        for (int w = 0; w < kAssemblers; ++w) {
            if (as[w]) (void)hipStreamDestroy(as[w]);
            if (as2[w]) (void)hipStreamDestroy(as2[w]);
        }
    }
};

// ---------------------------------------------------------------- entry points (called by the C ABI)
Server *server_create(const rte_server_desc_t &d, hipStream_t s) {
    RTE_REQUIRE(d.n_catalogue >= 1 && d.n_catalogue <= 4096 && d.nu, "server: band catalogue required");
    RTE_REQUIRE(d.levels_per_decade >= 1 && d.levels_per_decade <= 1000, "server: levels_per_decade out of range");
    RTE_REQUIRE(d.precision == RTE_FP64 || d.precision == RTE_MIXED_BF16,
                "server: precision must be RTE_FP64 or RTE_MIXED_BF16");
    RTE_REQUIRE(d.max_active >= 1, "server: max_active must be >= 1");
    RTE_REQUIRE(d.recompress == 0 || d.recompress == 1, "server: recompress must be 0 or 1");
    RTE_REQUIRE(d.hbm_budget >= 0, "server: hbm_budget must be >= 0");
    auto S = std::make_unique<Server>();
    S->desc = d;
    S->user = s;
    HIP_CHECK(hipGetDevice(&S->device));
    HIP_CHECK(hipStreamCreateWithFlags(&S->s, hipStreamNonBlocking));
    for (int w = 0; w < Server::kAssemblers; ++w) {
        HIP_CHECK(hipStreamCreateWithFlags(&S->as[w], hipStreamNonBlocking));
        HIP_CHECK(hipStreamCreateWithFlags(&S->as2[w], hipStreamNonBlocking));
    }
    for (int b = 0; b < d.n_catalogue; ++b) {
        RTE_REQUIRE(std::isfinite(d.nu[b]) && d.nu[b] > 0 && (b == 0 || d.nu[b] > d.nu[b - 1]),
                    "server: catalogue frequencies must be positive and increasing");
        S->nu.push_back(d.nu[b]);
    }
    // trapezoid weights on the catalogue; a request with a subset keeps them
    const int nb = d.n_catalogue;
    S->w.assign(nb, 1.0);
    if (nb > 1) {
        S->w[0] = 0.5 * (S->nu[1] - S->nu[0]);
        S->w[nb - 1] = 0.5 * (S->nu[nb - 1] - S->nu[nb - 2]);
        for (int b = 1; b + 1 < nb; ++b) S->w[b] = 0.5 * (S->nu[b + 1] - S->nu[b - 1]);
    }
    if (S->desc.hbm_budget == 0) {
        size_t fr = 0, tot = 0;
        HIP_CHECK(hipMemGetInfo(&fr, &tot));
        S->desc.hbm_budget = (int64_t)(0.8 * (double)fr);
    }
    S->stats.budget = S->desc.hbm_budget;
    Server *raw = S.get();
    for (int w = 0; w < Server::kAssemblers; ++w) S->workers.emplace_back([raw, w] { raw->worker_loop(w); });
    return S.release();
}

void server_destroy(Server *S) { delete S; }

// order the server's sweep stream after the caller's (inputs written there)
static void after_user(Server &S) {
    hipEvent_t e;
    HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIP_CHECK(hipEventRecord(e, S.user));
    HIP_CHECK(hipStreamWaitEvent(S.s, e, 0));
    for (int w = 0; w < Server::kAssemblers; ++w) HIP_CHECK(hipStreamWaitEvent(S.as[w], e, 0));
    (void)hipEventDestroy(e);
}

int server_add_mesh(Server &S, const rte_mesh_desc_t &md, const double *kappa) {
    auto M = std::make_unique<SrvMesh>();
    mesh_init(M->mesh, md);
    RTE_REQUIRE(M->mesh.L > 0, "server: the mesh has no emitting face");
    M->kappa.alloc(sizeof(double) * (size_t)M->mesh.N);
    after_user(S);
    HIP_CHECK(hipMemcpyAsync(M->kappa.p, kappa, M->kappa.bytes, hipMemcpyDeviceToDevice, S.s));
    HIP_CHECK(hipStreamSynchronize(S.s));
    M->est_bytes = S.bound_bytes(M->mesh);
    S.meshes.push_back(std::move(M));
    return (int)S.meshes.size() - 1;
}

int64_t server_submit(Server &S, const rte_request_t &q) {
    RTE_REQUIRE(q.mesh_id >= 0 && q.mesh_id < (int)S.meshes.size(), "request: unknown mesh");
    RTE_REQUIRE(q.n_bands >= 1 && q.n_bands <= (int)S.nu.size() && q.bands && q.kappa_mult,
                "request: bands and kappa multipliers required");
    RTE_REQUIRE(q.tol > 0 && std::isfinite(q.tol), "request: tol must be > 0");
    RTE_REQUIRE(q.max_iter >= 1, "request: max_iter must be >= 1");
    const SrvMesh &M = *S.meshes[q.mesh_id];
    auto r = std::make_unique<SrvReq>();
    r->id = S.next_id++;
    r->mesh = q.mesh_id;
    for (int b = 0; b < q.n_bands; ++b) {
        RTE_REQUIRE(q.bands[b] >= 0 && q.bands[b] < (int)S.nu.size() && (b == 0 || q.bands[b] > q.bands[b - 1]),
                    "request: band indices must be increasing catalogue indices");
        RTE_REQUIRE(std::isfinite(q.kappa_mult[b]) && q.kappa_mult[b] > 0, "request: kappa multipliers must be > 0");
        const double ab = q.a ? q.a[b] : 0.0;
        RTE_REQUIRE(std::isfinite(ab) && ab >= 0.0 && ab < 1.0, "request: scattering coefficients must lie in [0, 1)");
        r->a.push_back(ab);
        r->bands.push_back(q.bands[b]);
        r->levels.push_back(Server::snap(q.kappa_mult[b], S.desc.levels_per_decade));
    }
    r->tol = q.tol;
    r->max_iter = q.max_iter;
    r->Tw.alloc(sizeof(double) * (size_t)M.mesh.L);
    after_user(S);
    HIP_CHECK(hipMemcpyAsync(r->Tw.p, q.T_wall, r->Tw.bytes, hipMemcpyDeviceToDevice, S.s));
    HIP_CHECK(hipStreamSynchronize(S.s));
    const int64_t id = r->id;
    S.pending.push_back(r.get());
    S.reqs[id] = std::move(r);
    S.stats.submitted += 1;
    return id;
}

void server_step(Server &S, int32_t *n_active, int32_t *n_pending) {
    S.step();
    if (n_active) *n_active = (int32_t)S.active.size();
    if (n_pending) *n_pending = (int32_t)S.pending.size();
}

void server_poll(Server &S, int64_t id, rte_request_info_t &info) {
    auto it = S.reqs.find(id);
    RTE_REQUIRE(it != S.reqs.end(), "server: unknown request id");
    const SrvReq &r = *it->second;
    info.state = r.state;
    info.converged = r.converged ? 1 : 0;
    info.iterations = r.iterations;
    info.outer_steps = r.outer;
    info.residual = r.residual;
    info.n_bands = (int32_t)r.bands.size();
}

void server_levels(Server &S, int64_t id, int32_t *levels) {
    auto it = S.reqs.find(id);
    RTE_REQUIRE(it != S.reqs.end(), "server: unknown request id");
    for (size_t b = 0; b < it->second->levels.size(); ++b) levels[b] = it->second->levels[b];
}

void server_fetch(Server &S, int64_t id, double *T_out) {
    auto it = S.reqs.find(id);
    RTE_REQUIRE(it != S.reqs.end(), "server: unknown request id");
    SrvReq &r = *it->second;
    RTE_REQUIRE(r.state == RTE_REQ_DONE, "server: the request has not finished");
    const SrvMesh &M = *S.meshes[r.mesh];
    HIP_CHECK(hipMemcpyAsync(T_out, r.out.p, sizeof(double) * (size_t)M.mesh.N, hipMemcpyDeviceToDevice, S.s));
    HIP_CHECK(hipStreamSynchronize(S.s));
    S.reqs.erase(it);
}

int64_t server_mesh_size(Server &S, int mesh, int64_t *L) {
    RTE_REQUIRE(mesh >= 0 && mesh < (int)S.meshes.size(), "server: unknown mesh");
    if (L) *L = S.meshes[mesh]->mesh.L;
    return S.meshes[mesh]->mesh.N;
}

rte_server_stats_t server_stats(Server &S) { return S.stats; }

}  // namespace rte
