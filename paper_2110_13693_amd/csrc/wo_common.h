// Error handling shared by the host files of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/wo.h"

// Record a thread-local message for wo_last_error() and return s.
wo_status wo_fail(wo_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

// True when WO_FAULT_INJECT=alloc asks allocations to fail (tests).
bool wo_fault_injected();

#define WO_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return wo_fail(WO_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)
