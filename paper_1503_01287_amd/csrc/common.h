// Internal helpers of the gfx950 AMG library: error state, device buffers,
// launch checks. Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "amg_p2.h"

namespace amgp2 {

// An error raised inside the library; carries an AMG_* status code. The C ABI
// catches it, stores the message for amg_last_error() and returns the code.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string &msg);

#define AMG_HIP(call)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            throw ::amgp2::Error(e_ == hipErrorOutOfMemory ? AMG_ENOMEM : AMG_EHIP,        \
                                 std::string(#call) + ": " + hipGetErrorString(e_) + " (" + \
                                     __FILE__ + ":" + std::to_string(__LINE__) + ")");      \
    } while (0)

#define AMG_CHECK_LAUNCH() AMG_HIP(hipGetLastError())

#define AMG_REQUIRE(cond, code, msg)                  \
    do {                                              \
        if (!(cond)) throw ::amgp2::Error(code, msg); \
    } while (0)

// Host to device copy, complete on return. Large copies go through two
// pinned staging halves, the host copy of one chunk overlapping the DMA of
// the previous one; small ones copy from the source directly.
void copy_h2d(void *dst, const void *src, size_t bytes, hipStream_t s);

// When set (on a thread that builds one system of a batch), device buffers
// released on this thread are not freed but collected here, and freed once
// every system is built: a free waits for the whole device, so frees on
// many threads would serialise their builds.
inline thread_local std::vector<void *> *deferred_frees = nullptr;

// Owning device allocation.
template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t count) {
        release();
        n = count;
        if (count) AMG_HIP(hipMalloc(reinterpret_cast<void **>(&p), count * sizeof(T)));
    }
    void release() {
        if (p) {
            if (deferred_frees)
                deferred_frees->push_back(p);
            else
                (void)hipFree(p);
        }
        p = nullptr;
        n = 0;
    }
    // Host to device, complete on return: the source is often a temporary
    // the caller frees right away, and an asynchronous copy from pageable
    // memory may read its source after the call has returned.
    void upload(const T *h, size_t count, hipStream_t s) {
        if (count != n) alloc(count);
        if (count) copy_h2d(p, h, count * sizeof(T), s);
    }
    void upload(const std::vector<T> &v, hipStream_t s) { upload(v.data(), v.size(), s); }
    std::vector<T> download(hipStream_t s) const {
        std::vector<T> h(n);
        if (n) {
            AMG_HIP(hipMemcpyAsync(h.data(), p, n * sizeof(T), hipMemcpyDeviceToHost, s));
            AMG_HIP(hipStreamSynchronize(s));
        }
        return h;
    }
    void zero(hipStream_t s) {
        if (n) AMG_HIP(hipMemsetAsync(p, 0, n * sizeof(T), s));
    }
};

inline int ceil_div(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

}  // namespace amgp2
