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
// ------------------------------------------------------------------ device buffers
template <typename T> struct DevBuf {
    T *p = nullptr;
    size_t cap = 0; // elements
    int ensure(size_t n)
    {
        if (n <= cap && p)
            return TSK_OK;
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
        if (p)
            (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

} // namespace tsk
