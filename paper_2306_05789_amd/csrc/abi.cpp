// The C ABI (include/rte.h): argument validation, handle management and
// error translation.  Every entry point catches everything and returns a
// status; the message of the last error is kept per thread.
#include <exception>
#include <thread>
#include <atomic>
#include <chrono>
#include <algorithm>
#include <cmath>
#include <numeric>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_set>

#include "rte_internal.h"
#include "serve.h"

using namespace rte;

namespace {

thread_local std::string g_last_error;

// Workspace of rte_hmat_matvec_noalloc: a file-scope device array, so that the
// call allocates nothing.  Each device that runs the library holds its own copy
// until the process ends.  Host code never uses the array's name as an address:
// the device address of each copy is taken with hipGetSymbolAddress on the
// call's first use on that device and kept per device.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;   // device -> device address of its copy of `scratch`

void *scratch_address(int device) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) return it->second;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        throw Error(RTE_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = ptr;
    return ptr;
}


template <typename F>
rte_status_t guard(F &&f) {
    try {
        g_last_error.clear();
        return f();
    } catch (const Error &e) {
        g_last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return RTE_E_OUT_OF_MEMORY;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return RTE_E_INTERNAL;
    } catch (...) {
        g_last_error = "unknown error";
        return RTE_E_INTERNAL;
    }
}

template <typename T>
std::vector<T> to_host(const T *dev, int64_t n, hipStream_t s) {
    std::vector<T> h((size_t)n);
    if (n) {
        HIP_CHECK(hipMemcpyAsync(h.data(), dev, sizeof(T) * (size_t)n, hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
    }
    return h;
}

void check_device_pointer(const void *p, const char *what) {
    RTE_REQUIRE(p != nullptr, std::string(what) + " is NULL");
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error(RTE_E_INVALID_ARG, std::string(what) + " is not a device pointer");
    }
    RTE_REQUIRE(attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged,
                std::string(what) + " is not device memory");
}

void check_kappa(const double *kappa, int64_t n, hipStream_t s) {
    check_device_pointer(kappa, "kappa");
    auto h = to_host(kappa, n, s);
    for (double v : h) RTE_REQUIRE(std::isfinite(v) && v >= 0.0, "kappa must be finite and >= 0");
}

// Stored elements [0, count) of one array of band storage as FP64: FP64 as is,
// FP32 widened, BF16 hi (+ lo for the accurate operator) summed in FP64.
std::vector<double> read_stored(const HMat &H, const void *hi, const void *lo, int64_t count, int op) {
    std::vector<double> out((size_t)count);
    if (count == 0) return out;
    if (H.precision == RTE_FP64) {
        HIP_CHECK(hipMemcpy(out.data(), hi, sizeof(double) * count, hipMemcpyDeviceToHost));
    } else if (H.precision == RTE_FP32) {
        std::vector<float> f((size_t)count);
        HIP_CHECK(hipMemcpy(f.data(), hi, sizeof(float) * count, hipMemcpyDeviceToHost));
        for (int64_t e = 0; e < count; ++e) out[e] = f[e];
    } else {
        auto wid = [](uint16_t h) {
            const uint32_t u = (uint32_t)h << 16;
            float f;
            std::memcpy(&f, &u, 4);
            return (double)f;
        };
        std::vector<uint16_t> h((size_t)count), l(op == RTE_OP_LOW ? 0 : (size_t)count);
        HIP_CHECK(hipMemcpy(h.data(), hi, 2 * count, hipMemcpyDeviceToHost));
        if (op != RTE_OP_LOW) HIP_CHECK(hipMemcpy(l.data(), lo, 2 * count, hipMemcpyDeviceToHost));
        for (int64_t e = 0; e < count; ++e) out[e] = wid(h[e]) + (op == RTE_OP_LOW ? 0.0 : wid(l[e]));
    }
    return out;
}

// The row side of a block (rows [t0, t1) x K stored columns, split into
// target-leaf slices) as a row-major [m][ncol] matrix; column c of the result
// is stored column col(c).
template <typename ColOf>
void unpack_rows(const HMat &H, const void *hi, const void *lo, int64_t t0, int64_t t1, int64_t K, int64_t ncol,
                 ColOf col, int op, double *out) {
    const Plan &P = *H.plan;
    const int64_t g = H.kgroup, kgp = (K + g - 1) / g * g;
    const int li0 = P.leaf_of(t0);
    const int64_t total = kgp * (H.leaf_prp_h[P.leaf_of(t1 - 1) + 1] - H.leaf_prp_h[li0]);
    const std::vector<double> v = read_stored(H, hi, lo, total, op);
    for (int64_t i = 0; i < t1 - t0; ++i) {
        const int li = P.leaf_of(t0 + i);
        const int64_t rp = H.leaf_prp_h[li + 1] - H.leaf_prp_h[li];
        const int64_t base = kgp * (H.leaf_prp_h[li] - H.leaf_prp_h[li0]), r = t0 + i - P.leaf_start[li];
        // element (row r of the slice, column l) at ((l / g) * rp + r) * g + l % g
        for (int64_t c = 0; c < ncol; ++c) {
            const int64_t l = col(c);
            out[i * ncol + c] = v[(size_t)(base + ((l / g) * rp + r) * g + l % g)];
        }
    }
}

void block_factors(const HMat &H, int band, int64_t block, int op, int32_t *rank, int64_t *mo, int64_t *no,
                   double *U, double *V) {
    RTE_REQUIRE(band >= 0 && band < H.n_bands, "rte_hmat_block_factors: band out of range");
    RTE_REQUIRE(block >= 0 && block < (int64_t)H.plan->lowrank.size(), "rte_hmat_block_factors: block out of range");
    RTE_REQUIRE(op == RTE_OP_ACCURATE || op == RTE_OP_LOW, "rte_hmat_block_factors: unknown operator");
    const BandStore &B = H.bands[band];
    const Block &bl = H.plan->lowrank[block];
    const int64_t m = bl.t1 - bl.t0, n = bl.s1 - bl.s0, k = B.rank[block];
    *rank = B.rank[block];
    *mo = m;
    *no = n;
    if (!U || !V || k <= 0) return;
    unpack_rows(H, B.U[block], B.Ulo[block], bl.t0, bl.t1, k, k, [](int64_t c) { return c; }, op, U);
    // V: [n][pad4(k)], or [nP/8][k][8] over stored source coordinates
    const int64_t g = H.kgroup;
    const int64_t nv = g > 1 ? H.pwidth(bl.s0, bl.s1) * k : n * ((k + 3) & ~(int64_t)3);
    const std::vector<double> vt = read_stored(H, B.V[block], B.Vlo[block], nv, op);
    for (int64_t j = 0; j < n; ++j) {
        const int64_t jp = H.src_p_h[bl.s0 + j] - H.src_p_h[bl.s0];
        for (int64_t l = 0; l < k; ++l)
            V[j * k + l] = g > 1 ? vt[((jp / 8) * k + l) * 8 + jp % 8] : vt[j * ((k + 3) & ~(int64_t)3) + l];
    }
}

}  // namespace

namespace rte {

// Assembly of one H-matrix per band on a validated plan and kappa (device,
// [n_bands][N], natural order); see rte_hmat_assemble.
std::unique_ptr<rte_hmat> assemble_hmat(const Mesh &m, std::shared_ptr<const Plan> plan,
                                        const rte_hmat_opts_t &o, int n_bands, const double *kappa,
                                        hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const double alloc0 = alloc_ms_this_thread();
    double alloc_other = 0.0;   // allocation time of the second band thread
    size_t free_at_start = 0, total_mem = 0;
    HIP_CHECK(hipMemGetInfo(&free_at_start, &total_mem));
    free_at_start += pool_idle_bytes();
    auto hm = std::make_unique<rte_hmat>();
    HMat &H = hm->h;
    HIP_CHECK(hipGetDevice(&H.device));
    H.mesh = &m;
    H.n_bands = n_bands;
    const rte_hmat_opts_t *opts = &o;
    H.opts = o;
    // default launch shape (the autotuner may change it): 8 waves per phase-B
    // workgroup, 256 KiB phase-A chunks (fewer partials to add), 4 tiles per
    // matrix-core task; the fastest or within 2 % of it on the 29^3-49^3 cubes
    H.cfg = MatvecConfig{8, 256, 4};
    H.precision = opts->precision;
    H.kind = opts->kind;
    H.plan = std::move(plan);
    const Plan &P = *H.plan;
    H.tgt_nat = upload(P.tgt_nat, s);
    H.src_nat = upload(P.src_nat, s);
    H.src_pos = upload(opts->kind == RTE_VOLUME ? P.tgt_nat : P.src.perm, s);
    // FP64 / FP32 slices are column-major with rows padded to 4 (vector
    // loads along the rows); BF16 slices are K-grouped (8 columns of a row
    // contiguous) with unpadded rows and sources counted in stored
    // coordinates in which every source leaf is rounded up to 8
    const bool kgrouped = H.precision == RTE_MIXED_BF16;
    H.kgroup = kgrouped ? 8 : 1;
    const int64_t unit = kgrouped ? 1 : 4;
    H.leaf_prp_h.assign(1, 0);
    for (auto &lf : P.tgt_leaves)
        H.leaf_prp_h.push_back(H.leaf_prp_h.back() + (lf.second - lf.first + unit - 1) / unit * unit);
    H.leaf_start = upload(P.leaf_start, s);
    H.leaf_prp = upload(H.leaf_prp_h, s);
    {
        const int64_t ns = (int64_t)P.src_nat.size();
        H.src_p_h.assign(ns + 1, 0);
        std::vector<int64_t> pmap;
        int64_t pos = 0;
        for (int id : P.src.leaves) {
            const ClusterNode &nd = P.src.nodes[id];
            for (int64_t j = nd.start; j < nd.stop; ++j) {
                H.src_p_h[j] = pos + (j - nd.start);
                pmap.push_back(j);
            }
            const int64_t w = kgrouped ? ((nd.stop - nd.start + 7) & ~(int64_t)7) : nd.stop - nd.start;
            for (int64_t e = nd.stop - nd.start; e < w; ++e) pmap.push_back(-1);
            pos += w;
        }
        H.src_p_h[ns] = pos;
        H.n_src_p = pos;
        H.src_p = upload(H.src_p_h, s);
        H.src_pmap = upload(pmap, s);
    }
    H.kappa_c.alloc(sizeof(double) * (size_t)m.N * n_bands);
    permute_gather(H.tgt_nat.as<int64_t>(), m.N, n_bands, m.N, m.N, kappa, H.kappa_c.as<double>(), s);
    H.bands.resize(n_bands);
    int64_t evaluated = 0, bytes = 0, dense_e = 0, lr_e = 0, nfb = 0, aca_e = 0, retried = 0;
    int64_t lr_aca = 0, rc_blocks = 0;
    double rc_ms = 0.0;
    double aca_ms = 0, fill_ms = 0, aca_entry_ms = 0;
    int aca_l = 0, fill_l = 0, aca_entry_l = 0;
    double wsum = 0, wr = 0;
    int maxr = 0;
    matvec_reserve(H, n_bands);   // the bands' plans are then built from two threads
    // Bands are independent: with more than one, a second host thread on its
    // own stream takes every other band as it comes free, so one band's ACA
    // tail and host work overlap the other's kernels.
    {
        std::atomic<int> next{0};
        auto run = [&](hipStream_t st) {
            for (int b; (b = next.fetch_add(1)) < n_bands;) {
                assemble_band(H, b, kappa + (int64_t)b * m.N, st);
                matvec_build(H, b, st);   // host work while the band's last kernels run
                band_settle(H.bands[b], st);
            }
        };
        if (n_bands == 1) {
            run(s);
        } else {
            hipStream_t s2 = nullptr;
            hipEvent_t ready = nullptr;
            HIP_CHECK(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
            HIP_CHECK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
            HIP_CHECK(hipEventRecord(ready, s));   // the uploads above come first
            HIP_CHECK(hipStreamWaitEvent(s2, ready, 0));
            const int dev = H.device;
            std::exception_ptr e1, e2;
            std::thread t2([&] {
                try {
                    HIP_CHECK(hipSetDevice(dev));
                    run(s2);
                    HIP_CHECK(hipStreamSynchronize(s2));
                    alloc_other = alloc_ms_this_thread();
                } catch (...) {
                    e2 = std::current_exception();
                    next.store(n_bands);   // the other thread stops taking bands
                }
            });
            try {
                run(s);
            } catch (...) {
                e1 = std::current_exception();
                next.store(n_bands);
            }
            t2.join();
            (void)hipStreamSynchronize(s2);
            (void)hipEventDestroy(ready);
            (void)hipStreamDestroy(s2);
            if (e1) std::rethrow_exception(e1);
            if (e2) std::rethrow_exception(e2);
        }
    }
    for (int b = 0; b < n_bands; ++b) {
        const BandStore &B = H.bands[b];
        evaluated += B.evaluated;
        aca_e += B.aca_entries;
        retried += B.aca_retried;
        aca_ms += B.aca_ms;
        aca_entry_ms += B.aca_entry_ms;
        aca_entry_l += B.aca_entry_launches;
        fill_ms += B.fill_ms;
        aca_l += B.aca_launches;
        fill_l += B.fill_launches;
        bytes += B.bytes;
        dense_e += B.dense_entries;
        lr_e += B.lr_entries;
        lr_aca += B.lr_entries + B.rc_before - B.rc_after;
        rc_blocks += B.rc_blocks;
        rc_ms += B.rc_ms;
        for (size_t k = 0; k < P.lowrank.size(); ++k) {
            const Block &bl = P.lowrank[k];
            const double mn = (double)((bl.t1 - bl.t0) + (bl.s1 - bl.s0));
            if (B.rank[k] < 0) { ++nfb; continue; }
            wsum += mn;
            wr += mn * B.rank[k];
            maxr = std::max(maxr, B.rank[k]);
        }
    }
    matvec_build_all(H, s);
    HIP_CHECK(hipStreamSynchronize(s));
    rte_hmat_stats_t &st = H.stats;
    st.n_tgt = (int64_t)P.tgt_nat.size();
    st.n_src = (int64_t)P.src_nat.size();
    st.n_bands = n_bands;
    st.precision = H.precision;
    st.n_dense = (int64_t)P.dense.size();
    st.n_lowrank = (int64_t)P.lowrank.size();
    st.n_fallback_dense = nfb;
    st.dense_entries = dense_e;
    st.lowrank_entries = lr_e;
    st.max_rank = maxr;
    st.mean_rank = wsum > 0 ? wr / wsum : 0.0;
    st.compression = 1.0 - (double)(dense_e + lr_e) / ((double)st.n_tgt * st.n_src * n_bands);
    st.bytes = bytes;
    st.entries_evaluated = evaluated;
    st.aca_entries = aca_e;
    st.aca_retried = retried;
    st.aca_kernel_ms = aca_ms;
    st.aca_launches = aca_l;
    st.aca_entry_ms = aca_entry_ms;
    st.aca_entry_launches = aca_entry_l;
    st.fill_kernel_ms = fill_ms;
    st.fill_launches = fill_l;
    st.assemble_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    st.alloc_ms = alloc_ms_this_thread() - alloc0 + alloc_other;
    st.free_bytes = (int64_t)free_at_start;
    st.lowrank_entries_aca = lr_aca;
    st.recompressed_blocks = rc_blocks;
    st.recompress_ms = rc_ms;
    return hm;
}

}  // namespace rte

extern "C" {

rte_status_t rte_server_create(const rte_server_desc_t *desc, void *stream, rte_server_t *out) {
    return guard([&] {
        RTE_REQUIRE(desc && out, "rte_server_create: NULL argument");
        *out = nullptr;
        auto h = std::make_unique<rte_server>();
        h->srv = server_create(*desc, (hipStream_t)stream);
        *out = h.release();
        return RTE_OK;
    });
}

rte_status_t rte_server_add_mesh(rte_server_t s, const rte_mesh_desc_t *mesh, const double *kappa, int32_t *mesh_id) {
    return guard([&] {
        RTE_REQUIRE(s && mesh && mesh_id, "rte_server_add_mesh: NULL argument");
        Mesh probe;
        mesh_init(probe, *mesh);
        check_kappa(kappa, probe.N, nullptr);
        *mesh_id = server_add_mesh(*s->srv, *mesh, kappa);
        return RTE_OK;
    });
}

rte_status_t rte_server_submit(rte_server_t s, const rte_request_t *req, int64_t *id) {
    return guard([&] {
        RTE_REQUIRE(s && req && id, "rte_server_submit: NULL argument");
        int64_t L = 0;
        server_mesh_size(*s->srv, req->mesh_id, &L);
        check_device_pointer(req->T_wall, "T_wall");
        auto tw = to_host(req->T_wall, L, nullptr);
        for (double v : tw) RTE_REQUIRE(std::isfinite(v) && v > 0.0, "request: T_wall must be finite and > 0");
        *id = server_submit(*s->srv, *req);
        return RTE_OK;
    });
}

rte_status_t rte_server_step(rte_server_t s, int32_t *n_active, int32_t *n_pending) {
    return guard([&] {
        RTE_REQUIRE(s, "rte_server_step: NULL server");
        server_step(*s->srv, n_active, n_pending);
        return RTE_OK;
    });
}

rte_status_t rte_server_poll(rte_server_t s, int64_t id, rte_request_info_t *info) {
    return guard([&] {
        RTE_REQUIRE(s && info, "rte_server_poll: NULL argument");
        server_poll(*s->srv, id, *info);
        return RTE_OK;
    });
}

rte_status_t rte_server_levels(rte_server_t s, int64_t id, int32_t *levels) {
    return guard([&] {
        RTE_REQUIRE(s && levels, "rte_server_levels: NULL argument");
        server_levels(*s->srv, id, levels);
        return RTE_OK;
    });
}

rte_status_t rte_server_fetch(rte_server_t s, int64_t id, double *T_out) {
    return guard([&] {
        RTE_REQUIRE(s && T_out, "rte_server_fetch: NULL argument");
        check_device_pointer(T_out, "T_out");
        server_fetch(*s->srv, id, T_out);
        return RTE_OK;
    });
}

rte_status_t rte_server_stats(rte_server_t s, rte_server_stats_t *stats) {
    return guard([&] {
        RTE_REQUIRE(s && stats, "rte_server_stats: NULL argument");
        *stats = server_stats(*s->srv);
        return RTE_OK;
    });
}

void rte_server_destroy(rte_server_t s) {
    if (!s) return;
    server_destroy(s->srv);
    delete s;
}

const char *rte_status_string(rte_status_t s) {
    switch (s) {
        case RTE_OK: return "ok";
        case RTE_E_INVALID_ARG: return "invalid argument";
        case RTE_E_OUT_OF_MEMORY: return "out of memory";
        case RTE_E_BUDGET: return "memory budget exceeded";
        case RTE_E_DEVICE: return "device error";
        case RTE_E_NOT_CONVERGED: return "not converged";
        case RTE_E_INTERNAL: return "internal error";
    }
    return "unknown status";
}

const char *rte_last_error(void) { return g_last_error.c_str(); }

const char *rte_version(void) { return "rte-mi355x 0.1 (gfx950)"; }

rte_status_t rte_mesh_create(const rte_mesh_desc_t *desc, rte_mesh_t *out) {
    return guard([&] {
        RTE_REQUIRE(desc && out, "rte_mesh_create: NULL argument");
        *out = nullptr;
        auto m = std::make_unique<rte_mesh>();
        mesh_init(m->m, *desc);
        *out = m.release();
        return RTE_OK;
    });
}

rte_status_t rte_mesh_sizes(rte_mesh_t mesh, int64_t *N, int64_t *L) {
    return guard([&] {
        RTE_REQUIRE(mesh, "rte_mesh_sizes: NULL mesh");
        if (N) *N = mesh->m.N;
        if (L) *L = mesh->m.L;
        return RTE_OK;
    });
}

rte_status_t rte_mesh_emitting_ids(rte_mesh_t mesh, int64_t *ids) {
    return guard([&] {
        RTE_REQUIRE(mesh && ids, "rte_mesh_emitting_ids: NULL argument");
        std::memcpy(ids, mesh->m.emitting.data(), sizeof(int64_t) * mesh->m.emitting.size());
        return RTE_OK;
    });
}

void rte_mesh_destroy(rte_mesh_t mesh) { delete mesh; }

rte_status_t rte_plan_create(rte_mesh_t mesh, const rte_hmat_opts_t *opts, rte_plan_t *out) {
    return guard([&] {
        RTE_REQUIRE(mesh && opts && out, "rte_plan_create: NULL argument");
        *out = nullptr;
        auto p = std::make_unique<rte_plan>();
        p->p = build_plan(mesh->m, *opts);
        *out = p.release();
        return RTE_OK;
    });
}

rte_status_t rte_plan_info(rte_plan_t plan, rte_plan_info_t *info) {
    return guard([&] {
        RTE_REQUIRE(plan && info, "rte_plan_info: NULL argument");
        const Plan &P = *plan->p;
        info->n_tgt = (int64_t)P.tgt_nat.size();
        info->n_src = (int64_t)P.src_nat.size();
        info->n_dense = (int64_t)P.dense.size();
        info->n_lowrank = (int64_t)P.lowrank.size();
        info->dense_entries = 0;
        for (auto &b : P.dense) info->dense_entries += (b.t1 - b.t0) * (b.s1 - b.s0);
        info->lowrank_sum_mn = 0;
        for (auto &b : P.lowrank) info->lowrank_sum_mn += (b.t1 - b.t0) + (b.s1 - b.s0);
        info->n_tgt_leaves = (int64_t)P.tgt_leaves.size();
        return RTE_OK;
    });
}

rte_status_t rte_plan_export(rte_plan_t plan, int64_t *tgt_perm, int64_t *src_perm, int64_t *blocks) {
    return guard([&] {
        RTE_REQUIRE(plan, "rte_plan_export: NULL plan");
        const Plan &P = *plan->p;
        if (tgt_perm) std::memcpy(tgt_perm, P.tgt_nat.data(), sizeof(int64_t) * P.tgt_nat.size());
        if (src_perm) std::memcpy(src_perm, P.src_nat.data(), sizeof(int64_t) * P.src_nat.size());
        if (blocks) {
            int64_t k = 0;
            for (auto &b : P.dense) {
                blocks[k++] = b.t0; blocks[k++] = b.t1; blocks[k++] = b.s0; blocks[k++] = b.s1; blocks[k++] = 0;
            }
            for (auto &b : P.lowrank) {
                blocks[k++] = b.t0; blocks[k++] = b.t1; blocks[k++] = b.s0; blocks[k++] = b.s1; blocks[k++] = 1;
            }
        }
        return RTE_OK;
    });
}

void rte_plan_destroy(rte_plan_t plan) { delete plan; }

rte_status_t rte_entries(rte_mesh_t mesh, int32_t kind, const double *kappa, int64_t n, const int64_t *rows,
                         const int64_t *cols, double *out, int32_t precision, void *stream) {
    return guard([&] {
        RTE_REQUIRE(mesh, "rte_entries: NULL mesh");
        RTE_REQUIRE(kind == RTE_VOLUME || kind == RTE_SURFACE, "rte_entries: bad kind");
        RTE_REQUIRE(precision == RTE_FP64 || precision == RTE_FP32 || precision == RTE_MIXED_BF16,
                    "rte_entries: bad precision");
        RTE_REQUIRE(n >= 0, "rte_entries: n < 0");
        if (n == 0) return RTE_OK;
        hipStream_t s = (hipStream_t)stream;
        const Mesh &m = mesh->m;
        check_kappa(kappa, m.N, s);
        check_device_pointer(rows, "rows");
        check_device_pointer(cols, "cols");
        check_device_pointer(out, "out");
        auto hr = to_host(rows, n, s), hc = to_host(cols, n, s);
        for (int64_t v : hr) RTE_REQUIRE(v >= 0 && v < m.N, "rte_entries: row id out of range");
        if (kind == RTE_VOLUME) {
            for (int64_t v : hc) RTE_REQUIRE(v >= 0 && v < m.N, "rte_entries: column id out of range");
        } else {
            std::unordered_set<int64_t> em(m.emitting.begin(), m.emitting.end());
            for (int64_t v : hc) RTE_REQUIRE(em.count(v), "rte_entries: column is not an emitting vertex");
        }
        entries_launch(m, kind, kappa, n, rows, cols, out, precision, s);
        HIP_CHECK(hipStreamSynchronize(s));
        return RTE_OK;
    });
}

rte_status_t rte_hmat_assemble(rte_mesh_t mesh, int32_t n_bands, const double *kappa, const rte_hmat_opts_t *opts,
                               void *stream, rte_hmat_t *out) {
    return guard([&] {
        RTE_REQUIRE(mesh && opts && out, "rte_hmat_assemble: NULL argument");
        *out = nullptr;
        RTE_REQUIRE(n_bands >= 1 && n_bands <= 4096, "rte_hmat_assemble: n_bands out of range");
        hipStream_t s = (hipStream_t)stream;
        const Mesh &m = mesh->m;
        auto plan = mesh_plan(m, *opts);
        check_kappa(kappa, m.N * n_bands, s);
        *out = assemble_hmat(m, std::move(plan), *opts, n_bands, kappa, s).release();
        return RTE_OK;
    });
}

rte_status_t rte_hmat_matvec(rte_hmat_t h, int32_t band, int32_t nrhs, const double *x, double *y, void *stream) {
    return guard([&] {
        RTE_REQUIRE(h, "rte_hmat_matvec: NULL matrix");
        const HMat &H = h->h;
        RTE_REQUIRE(band >= 0 && band < H.n_bands, "rte_hmat_matvec: band out of range");
        RTE_REQUIRE(nrhs >= 1 && nrhs <= 4096, "rte_hmat_matvec: nrhs out of range");
        check_device_pointer(x, "x");
        check_device_pointer(y, "y");
        hipStream_t s = (hipStream_t)stream;
        const int64_t ns = H.stats.n_src, nt = H.stats.n_tgt;
        DevBuf xc(sizeof(double) * ns * nrhs), yc(sizeof(double) * nt * nrhs);
        permute_gather(H.src_pos.as<int64_t>(), ns, nrhs, ns, ns, x, xc.as<double>(), s);
        matvec_launch(H, band, nrhs, xc.as<double>(), yc.as<double>(), nullptr, s);
        permute_scatter(H.tgt_nat.as<int64_t>(), nt, nrhs, nt, nt, yc.as<double>(), y, s);
        HIP_CHECK(hipStreamSynchronize(s));
        return RTE_OK;
    });
}

rte_status_t rte_hmat_matvec_noalloc(rte_hmat_t h, int32_t band, int32_t nrhs, const double *x, double *y,
                                     void *stream) {
    return guard([&] {
        RTE_REQUIRE(h, "rte_hmat_matvec_noalloc: NULL matrix");
        const HMat &H = h->h;
        RTE_REQUIRE(band >= 0 && band < H.n_bands, "rte_hmat_matvec_noalloc: band out of range");
        RTE_REQUIRE(nrhs >= 1 && nrhs <= 4096, "rte_hmat_matvec_noalloc: nrhs out of range");
        check_device_pointer(x, "x");
        check_device_pointer(y, "y");
        int dev = 0;
        HIP_CHECK(hipGetDevice(&dev));
        RTE_REQUIRE(dev == H.device, "rte_hmat_matvec_noalloc: the matrix lives on another device");
        // layout of the workspace: x and y in cluster order, then the matvec's own
        // workspace, each 256-byte aligned
        auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
        const int64_t ns = H.stats.n_src, nt = H.stats.n_tgt;
        const size_t bx = al(sizeof(double) * (size_t)(ns * nrhs)), by = al(sizeof(double) * (size_t)(nt * nrhs));
        const size_t bw = al(sizeof(double) * (size_t)matvec_ws(H, band, nrhs));
        if (bx + by + bw > kNoAllocBytes)
            throw Error(RTE_E_BUDGET, "rte_hmat_matvec_noalloc: needs " + std::to_string(bx + by + bw) +
                                          " bytes of workspace, more than its fixed " +
                                          std::to_string(kNoAllocBytes) + "; use rte_hmat_matvec");
        char *base = static_cast<char *>(scratch_address(dev));
        double *xc = reinterpret_cast<double *>(base), *yc = reinterpret_cast<double *>(base + bx);
        double *ws = reinterpret_cast<double *>(base + bx + by);
        hipStream_t s = (hipStream_t)stream;
        permute_gather(H.src_pos.as<int64_t>(), ns, nrhs, ns, ns, x, xc, s);
        matvec_launch_ws(H, band, nrhs, xc, yc, nullptr, ws, s);
        permute_scatter(H.tgt_nat.as<int64_t>(), nt, nrhs, nt, nt, yc, y, s);
        HIP_CHECK(hipStreamSynchronize(s));
        return RTE_OK;
    });
}

rte_status_t rte_hmat_matvec_batched(rte_hmat_t h, int32_t nrhs, const double *x, double *y, int32_t op,
                                     void *stream) {
    return guard([&] {
        RTE_REQUIRE(h, "rte_hmat_matvec_batched: NULL matrix");
        const HMat &H = h->h;
        RTE_REQUIRE(nrhs >= 1 && nrhs <= 4096, "rte_hmat_matvec_batched: nrhs out of range");
        RTE_REQUIRE(op == RTE_OP_ACCURATE || op == RTE_OP_LOW, "rte_hmat_matvec_batched: unknown operator");
        check_device_pointer(x, "x");
        check_device_pointer(y, "y");
        hipStream_t s = (hipStream_t)stream;
        const int64_t ns = H.stats.n_src, nt = H.stats.n_tgt, nv = (int64_t)nrhs * H.n_bands;
        DevBuf xc(sizeof(double) * ns * nv), yc(sizeof(double) * nt * nv),
            ws(sizeof(double) * (size_t)matvec_ws_all(H, nrhs));
        poison(ws, s);
        permute_gather(H.src_pos.as<int64_t>(), ns, (int)nv, ns, ns, x, xc.as<double>(), s);
        matvec_launch_all(H, nrhs, xc.as<double>(), yc.as<double>(), nullptr, ws.as<double>(), s,
                          op == RTE_OP_LOW ? kMatvecLow : kMatvecAccurate);
        permute_scatter(H.tgt_nat.as<int64_t>(), nt, (int)nv, nt, nt, yc.as<double>(), y, s);
        HIP_CHECK(hipStreamSynchronize(s));
        return RTE_OK;
    });
}

rte_status_t rte_hmat_get_config(rte_hmat_t h, rte_matvec_config_t *cfg) {
    return guard([&] {
        RTE_REQUIRE(h && cfg, "rte_hmat_get_config: NULL argument");
        cfg->phase_b_waves = h->h.cfg.waves_b;
        cfg->phase_a_kib = h->h.cfg.task_kib;
        cfg->phase_a_tiles = h->h.cfg.tiles;
        return RTE_OK;
    });
}

rte_status_t rte_hmat_set_config(rte_hmat_t h, const rte_matvec_config_t *cfg, void *stream) {
    return guard([&] {
        RTE_REQUIRE(h && cfg, "rte_hmat_set_config: NULL argument");
        matvec_configure(h->h, MatvecConfig{cfg->phase_b_waves, cfg->phase_a_kib, cfg->phase_a_tiles},
                         (hipStream_t)stream);
        HIP_CHECK(hipStreamSynchronize((hipStream_t)stream));
        return RTE_OK;
    });
}

rte_status_t rte_hmat_autotune(rte_hmat_t h, int32_t nrhs, int32_t op, int32_t reps, void *stream,
                               rte_matvec_config_t *best, double *best_ms, int32_t *trials) {
    return guard([&] {
        RTE_REQUIRE(h, "rte_hmat_autotune: NULL matrix");
        RTE_REQUIRE(nrhs >= 1 && nrhs <= 4096, "rte_hmat_autotune: nrhs out of range");
        RTE_REQUIRE(op == RTE_OP_ACCURATE || op == RTE_OP_LOW, "rte_hmat_autotune: unknown operator");
        RTE_REQUIRE(reps >= 1 && reps <= 1000, "rte_hmat_autotune: reps out of range");
        int n = 0;
        double ms = 0;
        const MatvecConfig c = matvec_autotune(h->h, nrhs, op == RTE_OP_LOW ? kMatvecLow : kMatvecAccurate, reps,
                                               (hipStream_t)stream, &ms, &n);
        if (best) *best = rte_matvec_config_t{c.waves_b, c.task_kib, c.tiles};
        if (best_ms) *best_ms = ms;
        if (trials) *trials = n;
        return RTE_OK;
    });
}

rte_status_t rte_hmat_time_matvec(rte_hmat_t h, int32_t nrhs, int32_t op, int32_t reps, void *stream, double *ms) {
    return guard([&] {
        RTE_REQUIRE(h && ms, "rte_hmat_time_matvec: NULL argument");
        RTE_REQUIRE(nrhs >= 1 && nrhs <= 4096, "rte_hmat_time_matvec: nrhs out of range");
        RTE_REQUIRE(op == RTE_OP_ACCURATE || op == RTE_OP_LOW, "rte_hmat_time_matvec: unknown operator");
        RTE_REQUIRE(reps >= 1 && reps <= 1000, "rte_hmat_time_matvec: reps out of range");
        *ms = matvec_time(h->h, nrhs, op == RTE_OP_LOW ? kMatvecLow : kMatvecAccurate, reps, (hipStream_t)stream);
        return RTE_OK;
    });
}

rte_status_t rte_hmat_stats(rte_hmat_t h, rte_hmat_stats_t *stats) {
    return guard([&] {
        RTE_REQUIRE(h && stats, "rte_hmat_stats: NULL argument");
        *stats = h->h.stats;
        return RTE_OK;
    });
}

rte_status_t rte_kappa_levels(const double *values, int32_t n, double tol, int32_t max_levels, double *levels,
                              int32_t *map, int32_t *n_levels) {
    return guard([&] {
        RTE_REQUIRE(values && levels && map && n_levels, "rte_kappa_levels: NULL argument");
        RTE_REQUIRE(n >= 1 && max_levels >= 1, "rte_kappa_levels: need n >= 1 and max_levels >= 1");
        RTE_REQUIRE(std::isfinite(tol) && tol > 0.0, "rte_kappa_levels: tol must be > 0");
        for (int32_t b = 0; b < n; ++b)
            RTE_REQUIRE(std::isfinite(values[b]) && values[b] > 0.0, "rte_kappa_levels: values must be finite and > 0");
        // sorted order (ties by index), then the greedy cover of the logarithms by
        // intervals [ln v, ln v + 2 ln(1 + tol)], each level at its middle
        std::vector<int32_t> idx(n);
        std::iota(idx.begin(), idx.end(), 0);
        std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return values[a] < values[b]; });
        const double w = std::log1p(tol);
        int32_t nl = 0;
        double level = 0.0, lo = 0.0;
        for (int32_t q = 0; q < n; ++q) {
            const int32_t b = idx[q];
            const double lv = std::log(values[b]);
            if (nl == 0 || lv > lo + 2.0 * w) {
                RTE_REQUIRE(nl < max_levels, "rte_kappa_levels: more than max_levels levels needed (raise tol)");
                lo = lv;
                level = values[b] * (1.0 + tol);
                levels[nl++] = level;
            }
            map[b] = nl - 1;
        }
        *n_levels = nl;
        return RTE_OK;
    });
}

rte_status_t rte_hmat_select_bands(rte_hmat_t h, int32_t n_bands, const int32_t *band_op, void *stream,
                                   rte_hmat_t *out) {
    return guard([&] {
        RTE_REQUIRE(h && band_op && out, "rte_hmat_select_bands: NULL argument");
        const HMat &H = h->h;
        RTE_REQUIRE(n_bands >= 1 && n_bands <= 4096, "rte_hmat_select_bands: n_bands out of range");
        for (int32_t b = 0; b < n_bands; ++b)
            RTE_REQUIRE(band_op[b] >= 0 && band_op[b] < H.n_bands, "rte_hmat_select_bands: band index out of range");
        hipStream_t s = (hipStream_t)stream;
        int dev = 0;
        HIP_CHECK(hipGetDevice(&dev));
        RTE_REQUIRE(dev == H.device, "rte_hmat_select_bands: the matrix lives on another device");
        auto hv = std::make_unique<rte_hmat>();
        HMat &V = hv->h;
        V.mesh = H.mesh;
        V.plan = H.plan;
        V.opts = H.opts;
        V.n_bands = n_bands;
        V.precision = H.precision;
        V.kind = H.kind;
        V.device = H.device;
        V.cfg = H.cfg;
        V.kgroup = H.kgroup;
        V.leaf_prp_h = H.leaf_prp_h;
        V.src_p_h = H.src_p_h;
        V.n_src_p = H.n_src_p;
        auto dup = [&](const DevBuf &a) {
            DevBuf b(a.bytes);
            if (a.bytes) HIP_CHECK(hipMemcpyAsync(b.p, a.p, a.bytes, hipMemcpyDeviceToDevice, s));
            return b;
        };
        V.tgt_nat = dup(H.tgt_nat);
        V.src_nat = dup(H.src_nat);
        V.src_pos = dup(H.src_pos);
        V.leaf_start = dup(H.leaf_start);
        V.leaf_prp = dup(H.leaf_prp);
        V.src_p = dup(H.src_p);
        V.src_pmap = dup(H.src_pmap);
        // kappa at the targets: the rows of the selected bands
        const int64_t nt = (int64_t)H.plan->tgt_nat.size();
        V.kappa_c.alloc(sizeof(double) * (size_t)nt * n_bands);
        for (int32_t b = 0; b < n_bands; ++b)
            HIP_CHECK(hipMemcpyAsync(V.kappa_c.as<double>() + (int64_t)b * nt, H.kappa_c.as<double>() + band_op[b] * nt,
                                     sizeof(double) * nt, hipMemcpyDeviceToDevice, s));
        // the stored blocks of the selected bands, not owned: h keeps the storage
        V.bands.resize(n_bands);
        for (int32_t b = 0; b < n_bands; ++b) {
            const BandStore &B = H.bands[band_op[b]];
            BandStore &C = V.bands[b];
            C.dense_blocks = B.dense_blocks;
            C.dense_ptr = B.dense_ptr;
            C.dense_lo = B.dense_lo;
            C.rank = B.rank;
            C.U = B.U;
            C.V = B.V;
            C.Ulo = B.Ulo;
            C.Vlo = B.Vlo;
            C.bytes = B.bytes;
            C.dense_entries = B.dense_entries;
            C.lr_entries = B.lr_entries;
        }
        matvec_reserve(V, n_bands);
        for (int32_t b = 0; b < n_bands; ++b) matvec_build(V, b, s);
        matvec_build_all(V, s);
        HIP_CHECK(hipStreamSynchronize(s));
        V.stats = H.stats;
        V.stats.n_bands = n_bands;
        *out = hv.release();
        return RTE_OK;
    });
}

rte_status_t rte_hmat_block_factors(rte_hmat_t h, int32_t band, int64_t block, int32_t *rank, int64_t *mo,
                                    int64_t *no, double *U, double *V) {
    return guard([&] {
        RTE_REQUIRE(h && rank && mo && no, "rte_hmat_block_factors: NULL argument");
        block_factors(h->h, band, block, RTE_OP_ACCURATE, rank, mo, no, U, V);
        return RTE_OK;
    });
}

rte_status_t rte_hmat_block_factors_op(rte_hmat_t h, int32_t band, int64_t block, int32_t op, int32_t *rank,
                                       int64_t *mo, int64_t *no, double *U, double *V) {
    return guard([&] {
        RTE_REQUIRE(h && rank && mo && no, "rte_hmat_block_factors_op: NULL argument");
        block_factors(h->h, band, block, op, rank, mo, no, U, V);
        return RTE_OK;
    });
}

rte_status_t rte_hmat_dense_block(rte_hmat_t h, int32_t band, int64_t index, int32_t op, int64_t *count,
                                  int64_t *range, double *A) {
    return guard([&] {
        RTE_REQUIRE(h && count, "rte_hmat_dense_block: NULL argument");
        const HMat &H = h->h;
        RTE_REQUIRE(band >= 0 && band < H.n_bands, "rte_hmat_dense_block: band out of range");
        RTE_REQUIRE(op == RTE_OP_ACCURATE || op == RTE_OP_LOW, "rte_hmat_dense_block: unknown operator");
        const BandStore &B = H.bands[band];
        *count = (int64_t)B.dense_blocks.size();
        if (!range && !A) return RTE_OK;
        RTE_REQUIRE(index >= 0 && index < *count, "rte_hmat_dense_block: index out of range");
        const Block &bl = B.dense_blocks[(size_t)index];
        if (range) {
            range[0] = bl.t0;
            range[1] = bl.t1;
            range[2] = bl.s0;
            range[3] = bl.s1;
        }
        if (!A) return RTE_OK;
        // columns in stored source coordinates (padded per source leaf on BF16 storage)
        const int64_t s0p = H.src_p_h[bl.s0];
        unpack_rows(H, B.dense_ptr[(size_t)index], B.dense_lo[(size_t)index], bl.t0, bl.t1, H.pwidth(bl.s0, bl.s1),
                    bl.s1 - bl.s0, [&](int64_t c) { return H.src_p_h[bl.s0 + c] - s0p; }, op, A);
        return RTE_OK;
    });
}

void rte_hmat_destroy(rte_hmat_t h) { delete h; }

rte_status_t rte_fixed_point_solve(rte_mesh_t mesh, rte_hmat_t vol, rte_hmat_t surf, const rte_solve_desc_t *desc,
                                   double *T_out, double *J_out, rte_solve_stats_t *stats, void *stream) {
    return guard([&] {
        RTE_REQUIRE(mesh && vol && surf && desc, "rte_fixed_point_solve: NULL argument");
        hipStream_t s = (hipStream_t)stream;
        const Mesh &m = mesh->m;
        RTE_REQUIRE(desc->nrhs >= 1 && desc->nrhs <= 4096, "solve: nrhs out of range");
        check_device_pointer(desc->T_wall, "T_wall");
        auto tw = to_host(desc->T_wall, m.L * desc->nrhs, s);
        for (double v : tw) RTE_REQUIRE(std::isfinite(v) && v > 0.0, "solve: T_wall must be finite and > 0");
        if (desc->T0) {
            check_device_pointer(desc->T0, "T0");
            auto t0 = to_host(desc->T0, m.N * desc->nrhs, s);
            for (double v : t0) RTE_REQUIRE(std::isfinite(v) && v >= 0.0, "solve: T0 must be finite and >= 0");
        }
        if (T_out) check_device_pointer(T_out, "T_out");
        if (J_out) check_device_pointer(J_out, "J_out");
        return fixed_point_solve(m, vol->h, surf->h, *desc, T_out, J_out, stats, s);
    });
}

}  // extern "C"
