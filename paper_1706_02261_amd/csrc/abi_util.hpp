// Error reporting and argument checks shared by the C-ABI host files.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/bpm.h"
#include "internal.hpp"

namespace bpm {
namespace abi {

// message of the calling thread's last failed call
inline thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
inline int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

inline bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

inline int check_workspace(void* ws, size_t have, size_t need) {
    if (!ws || have < need)
        return fail(BPM_ERR_WORKSPACE, "workspace %p of %zu bytes; %zu bytes needed", ws, have,
                    need);
    if (!aligned(ws, kAlign))
        return fail(BPM_ERR_WORKSPACE, "workspace must be %zu-byte aligned", kAlign);
    return BPM_OK;
}

inline int device_status(hipError_t e, const char* what) {
    if (e == hipSuccess) return BPM_OK;
    return fail(BPM_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace abi
}  // namespace bpm
