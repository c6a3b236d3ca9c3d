// Device scratch reused across assemblies.
//
// An assembly's ACA batches need several GB of scratch (the factor columns
// of every block up to its rank cap, and the per-step partial sums) for a
// few hundred milliseconds.  Allocating and freeing that on every assembly
// costs host time, and hipFree waits for the whole device, so an assembly
// freeing its scratch on one thread stalls until the concurrent assembly on
// another stream has drained too.  Scratch that has been given back after its
// stream drained (DevBuf::settled) is kept here per device and handed out
// again; a buffer released without that guarantee (an exception unwinding
// past queued work) is freed with hipFree instead.
#include <algorithm>
#include <chrono>

#include "rte_internal.h"

namespace rte {

namespace {

struct Idle {
    int device;
    void *p;
    size_t cap;
    uint64_t stamp;
};

struct Pool {
    std::mutex mu;
    std::vector<Idle> idle;
    uint64_t clock = 0;
};

Pool &pool() {
    static Pool *p = new Pool();   // lives until the process ends (buffers stay with the device)
    return *p;
}

thread_local double t_alloc_ms = 0.0;

struct Clock {
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    ~Clock() {
        t_alloc_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

constexpr size_t kGranule = (size_t)2 << 20;

size_t idle_bytes_locked(Pool &P, int dev) {
    size_t b = 0;
    for (const Idle &i : P.idle)
        if (i.device == dev) b += i.cap;
    return b;
}

// keep at most an eighth of the device memory idle, dropping the least recently given back first
void cap_idle_locked(Pool &P, int dev) {
    size_t fb = 0, tb = 0;
    if (hipMemGetInfo(&fb, &tb) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    while (idle_bytes_locked(P, dev) > tb / 8) {
        auto it = std::min_element(P.idle.begin(), P.idle.end(), [&](const Idle &a, const Idle &b) {
            return (a.device == dev ? a.stamp : UINT64_MAX) < (b.device == dev ? b.stamp : UINT64_MAX);
        });
        (void)hipFree(it->p);
        P.idle.erase(it);
    }
}

}  // namespace

double &alloc_ms_this_thread() { return t_alloc_ms; }

void *pool_take(size_t bytes, size_t *cap) {
    Clock c;
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    const size_t want = (bytes + kGranule - 1) / kGranule * kGranule;
    Pool &P = pool();
    {
        std::lock_guard<std::mutex> g(P.mu);
        // best fit among the idle buffers of this device that are at most twice as large
        auto best = P.idle.end();
        for (auto it = P.idle.begin(); it != P.idle.end(); ++it)
            if (it->device == dev && it->cap >= want && it->cap <= 2 * want &&
                (best == P.idle.end() || it->cap < best->cap))
                best = it;
        if (best != P.idle.end()) {
            void *p = best->p;
            *cap = best->cap;
            P.idle.erase(best);
            return p;
        }
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        pool_trim();
        e = hipMalloc(&p, want);
    }
    if (e != hipSuccess)
        throw Error(e == hipErrorOutOfMemory ? RTE_E_OUT_OF_MEMORY : RTE_E_DEVICE,
                    std::string("hipMalloc (scratch): ") + hipGetErrorString(e));
    *cap = want;
    return p;
}

void pool_give(void *p, size_t cap) {
    Clock c;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(p);
        return;
    }
    Pool &P = pool();
    std::lock_guard<std::mutex> g(P.mu);
    P.idle.push_back({dev, p, cap, ++P.clock});
    cap_idle_locked(P, dev);
}

size_t pool_idle_bytes() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    Pool &P = pool();
    std::lock_guard<std::mutex> g(P.mu);
    return idle_bytes_locked(P, dev);
}

void pool_trim() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    Pool &P = pool();
    std::lock_guard<std::mutex> g(P.mu);
    for (auto it = P.idle.begin(); it != P.idle.end();) {
        if (it->device == dev) {
            (void)hipFree(it->p);
            it = P.idle.erase(it);
        } else {
            ++it;
        }
    }
}

void DevBuf::alloc(size_t b) {
    release();
    if (b) {
        Clock c;
        hipError_t e = hipMalloc(&p, b);
        if (e == hipErrorOutOfMemory) {   // idle scratch may be what is missing
            (void)hipGetLastError();
            pool_trim();
            e = hipMalloc(&p, b);
        }
        if (e != hipSuccess) {
            p = nullptr;
            throw Error(e == hipErrorOutOfMemory ? RTE_E_OUT_OF_MEMORY : RTE_E_DEVICE,
                        std::string("hipMalloc: ") + hipGetErrorString(e));
        }
    }
    bytes = b;
}

void DevBuf::release() noexcept {
    if (p) {
        bool kept = false;
        if (pooled && settled) {
            try {
                pool_give(p, cap);
                kept = true;
            } catch (...) {
            }
        }
        if (!kept) {
            Clock c;
            (void)hipFree(p);
        }
    }
    p = nullptr;
    bytes = cap = 0;
    pooled = settled = false;
}

DevBuf DevBuf::scratch(size_t b) {
    DevBuf d;
    if (b) {
        d.p = pool_take(b, &d.cap);
        d.pooled = true;
    }
    d.bytes = b;
    return d;
}

}  // namespace rte
