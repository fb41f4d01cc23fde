// Host-side plumbing shared by the library's translation units: error
// reporting (thread-local text, integer codes of tsknn.h) and a growable
// device buffer.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <string>

#include "tsknn.h"

namespace tsk {

// thread-local text of the last error (defined in tsknn.hip)
extern thread_local std::string g_err;

int set_err(int code, const char *fmt, ...);

} // namespace tsk

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) {                                                                    \
            (void)hipGetLastError();                                                               \
            return tsk::set_err(e_ == hipErrorOutOfMemory ? TSK_ERR_OOM : TSK_ERR_DEVICE,          \
                                "%s: %s", #expr, hipGetErrorString(e_));                           \
        }                                                                                          \
    } while (0)

#define TSK_TRY(expr)                                                                              \
    do {                                                                                           \
        int rc_ = (expr);                                                                          \
        if (rc_ != TSK_OK)                                                                         \
            return rc_;                                                                            \
    } while (0)

namespace tsk {
// A "_dev" argument must be device memory (or managed memory) visible to
// `device` (< 0: any device): a kernel that reads or writes through a host
// address faults the GPU, so such a pointer is an argument error.  NULL is
// left to the caller's own checks.
inline int check_dev_ptr(const void *p, int device, const char *what)
{
    if (!p)
        return TSK_OK;
    hipPointerAttribute_t a;
    a.type = hipMemoryTypeUnregistered;
    a.device = -1;
    const hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return tsk::set_err(TSK_ERR_INVALID_ARG, "%s is not device memory (%s)", what,
                            hipGetErrorString(e));
    }
    if (a.type == hipMemoryTypeManaged)
        return TSK_OK;
    if (a.type != hipMemoryTypeDevice)
        return tsk::set_err(TSK_ERR_INVALID_ARG, "%s is not device memory", what);
    if (device >= 0 && a.device != device)
        return tsk::set_err(TSK_ERR_INVALID_ARG, "%s is on device %d, not on device %d", what,
                            a.device, device);
    return TSK_OK;
}

// ------------------------------------------------------------------ device buffers
template <typename T> struct DevBuf {
    T *p = nullptr;
    size_t cap = 0; // elements
    // borrowed: p points into memory the buffer does not own (a carved
    // region of a fixed array); it is never freed, and a request beyond cap
    // is an error instead of a reallocation
    bool borrowed = false;
    void borrow(T *q, size_t n)
    {
        p = q;
        cap = n;
        borrowed = true;
    }
    int ensure(size_t n)
    {
        if (n <= cap && p)
            return TSK_OK;
        if (borrowed)
            return tsk::set_err(TSK_ERR_INVALID_ARG,
                                "workspace of %zu elements exceeds its fixed region of %zu", n,
                                cap);
        if (p) {
            (void)hipFree(p);
            p = nullptr;
            cap = 0;
        }
        size_t want = std::max<size_t>(n, 1);
        hipError_t e = hipMalloc((void **)&p, want * sizeof(T));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            return tsk::set_err(e == hipErrorOutOfMemory ? TSK_ERR_OOM : TSK_ERR_DEVICE,
                           "hipMalloc of %zu bytes: %s", want * sizeof(T), hipGetErrorString(e));
        }
        cap = want;
        return TSK_OK;
    }
    void release()
    {
        if (p && !borrowed)
            (void)hipFree(p);
        p = nullptr;
        cap = 0;
        borrowed = false;
    }
};

} // namespace tsk
