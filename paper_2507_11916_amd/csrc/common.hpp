// Shared host helpers: thread-local error text and HIP error checks.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>

#include "hb.h"

namespace hb {

hb_status fail(hb_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

#define HB_HIP(call)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess) return ::hb::fail(HB_E_DEVICE, "%s: %s (%s:%d)", #call, hipGetErrorString(e_), \
                                                __FILE__, __LINE__);                                   \
    } while (0)

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

}  // namespace hb
