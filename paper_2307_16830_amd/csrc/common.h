// Shared internals of libopf: error reporting, device buffers, launch helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "opf.h"

namespace opf {

void set_error(const char* fmt, ...);

// Returned through the C ABI as an opf_status.
struct Error {
    int code;
};

#define OPF_HIP(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) {                                                              \
            ::opf::set_error("%s:%d: %s: %s", __FILE__, __LINE__, #expr, hipGetErrorString(e_)); \
            throw ::opf::Error{OPF_E_DEVICE};                                                \
        }                                                                                    \
    } while (0)

#define OPF_CHECK(cond, code, ...)           \
    do {                                     \
        if (!(cond)) {                       \
            ::opf::set_error(__VA_ARGS__);   \
            throw ::opf::Error{code};        \
        }                                    \
    } while (0)

#define OPF_LAUNCH_CHECK() OPF_HIP(hipGetLastError())

// Run a body that may throw opf::Error / std::bad_alloc and map to a status.
template <class F>
int guarded(F&& f) {
    try {
        f();
        return OPF_OK;
    } catch (const Error& e) {
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return OPF_E_NOMEM;
    } catch (...) {
        set_error("unexpected C++ exception");
        return OPF_E_INVALID;
    }
}

// A slice of device memory that buffers of the calling host thread are carved from instead of hipMalloc
// (bump allocation, 256-byte aligned, nothing freed individually).  The solve server installs one per request
// while it creates that request's model and IPM state, so that admission can count the request's exact
// footprint and the request's memory comes from the server's pool without device-synchronizing frees.
struct DeviceRegion {
    char* base = nullptr;
    size_t cap = 0;
    size_t used = 0;
};
DeviceRegion*& thread_region();  // the calling thread's region, or nullptr (plain hipMalloc)

// Owning HBM buffer.
template <class T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    bool pooled = false;  // carved from a DeviceRegion: not freed individually
    DBuf() = default;
    explicit DBuf(size_t count) { alloc(count); }
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    DBuf(DBuf&& o) noexcept : p(o.p), n(o.n), pooled(o.pooled) {
        o.p = nullptr;
        o.n = 0;
        o.pooled = false;
    }
    DBuf& operator=(DBuf&& o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            n = o.n;
            pooled = o.pooled;
            o.p = nullptr;
            o.n = 0;
            o.pooled = false;
        }
        return *this;
    }
    ~DBuf() { release(); }
    void alloc(size_t count) {
        release();
        n = count;
        if (count == 0) return;
        if (DeviceRegion* r = thread_region()) {
            const size_t off = (r->used + 255) & ~size_t(255), bytes = count * sizeof(T);
            if (off > r->cap || bytes > r->cap - off) {
                n = 0;
                set_error("device region of %zu bytes exhausted (%zu used, %zu more requested)", r->cap, off, bytes);
                throw Error{OPF_E_NOMEM};
            }
            p = reinterpret_cast<T*>(r->base + off);
            r->used = off + bytes;
            pooled = true;
            return;
        }
        hipError_t e = hipMalloc(reinterpret_cast<void**>(&p), count * sizeof(T));
        if (e != hipSuccess) {
            p = nullptr;
            n = 0;
            set_error("hipMalloc of %zu bytes failed: %s", count * sizeof(T), hipGetErrorString(e));
            throw Error{OPF_E_NOMEM};
        }
    }
    void release() {
        if (p && !pooled) (void)hipFree(p);
        p = nullptr;
        n = 0;
        pooled = false;
    }
    void upload(const std::vector<T>& h, hipStream_t s = nullptr) {
        alloc(h.size());
        if (!h.empty()) {
            OPF_HIP(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
            OPF_HIP(hipStreamSynchronize(s));
        }
    }
};

// Device uploads recorded on the host and performed at the first device use,
// so that host-only queries (structure, patterns, symbolic analysis) work
// without touching the GPU.
struct Deferred {
    std::vector<std::function<void(hipStream_t)>> jobs;
    bool done = false;
    hipStream_t stream = nullptr;  // the uploads run on this stream (synchronised before run() returns)
    template <class T>
    void upload(DBuf<T>& d, std::vector<T> h) {
        jobs.push_back([&d, h = std::move(h)](hipStream_t s) { d.upload(h, s); });
    }
    template <class T>
    void alloc(DBuf<T>& d, size_t n) {
        jobs.push_back([&d, n](hipStream_t) { d.alloc(n); });
    }
    void run() {
        if (done) return;
        for (auto& j : jobs) j(stream);
        jobs.clear();
        done = true;
    }
};

inline unsigned ceil_div(size_t a, size_t b) { return static_cast<unsigned>((a + b - 1) / b); }

}  // namespace opf
