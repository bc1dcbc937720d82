// Shared host/device definitions for the SYK HIP library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

#include "../../include/syk.h"

namespace syk {

// Interleaved complex numbers, matching the caller's complex128 / complex64 buffers.
template <typename R>
struct alignas(2 * sizeof(R)) cplx {
    R re, im;
};
using c128 = cplx<double>;
using c64 = cplx<float>;

// Error carrying a status code across the internal layers; the C-ABI turns it
// into a return value and the thread-local message of syk_last_error().
struct Error : std::runtime_error {
    syk_status code;
    Error(syk_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

inline void hip_check(hipError_t e, const char* what, const char* file, int line)
{
    if (e != hipSuccess) {
        char buf[512];
        std::snprintf(buf, sizeof buf, "%s failed at %s:%d: %s", what, file, line, hipGetErrorString(e));
        throw Error(SYK_EHIP, buf);
    }
}
#define SYK_HIP(call) ::syk::hip_check((call), #call, __FILE__, __LINE__)

inline void require(bool ok, const std::string& msg)
{
    if (!ok) throw Error(SYK_EINVAL, msg);
}

inline size_t elem_bytes(syk_dtype d) { return d == SYK_C128 ? 16 : 8; }

// Device buffer owned by the library (workspaces, tables).
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) {
            (void)hipDeviceSynchronize();   // work enqueued earlier may still read it
            (void)hipFree(p);
        }
        p = nullptr;
        bytes = 0;
    }
    void ensure(size_t n)
    {
        if (n <= bytes) return;
        release();
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            throw Error(e == hipErrorOutOfMemory ? SYK_ENOMEM : SYK_EHIP,
                        std::string("hipMalloc of ") + std::to_string(n) + " bytes: " + hipGetErrorString(e));
        }
        bytes = n;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

}  // namespace syk
