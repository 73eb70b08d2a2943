// Device-side bounds checks of the checked build (compiled with
// -DMK_DEVICE_CHECKS; build.py --device-checks).
//
// Before a launch the host finds, for each buffer a kernel addresses, the
// number of bytes from the pointer it passes to the end of the allocation
// behind it.  Each kernel compares the end of every range it is about to
// read or write (per trace, per tile or per row run) with that extent; a
// failed comparison sets a word of the kernel's translation unit, which
// mk_device_checks() reads and clears.  The access itself is not
// suppressed: the checked build is for runs whose accesses are believed to
// be in bounds, to confirm it.  In the normal build the checks and extents
// compile to nothing.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#ifdef MK_DEVICE_CHECKS
static __device__ unsigned int mk_check_word;
#define MK_DCHECK(cond)                                         \
    do {                                                        \
        if (!(cond)) atomicOr(&mk_check_word, 1u);              \
    } while (0)
// hipError_t NAME(unsigned* out): this translation unit's word, then zero
#define MK_CHECK_TAKE(NAME)                                                              \
    hipError_t NAME(unsigned* out) {                                                     \
        hipError_t e = hipMemcpyFromSymbol(out, HIP_SYMBOL(mk_check_word), sizeof(unsigned)); \
        const unsigned zero = 0;                                                         \
        if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(mk_check_word), &zero, sizeof(unsigned)); \
        return e;                                                                        \
    }
#else
#define MK_DCHECK(cond) ((void)0)
#define MK_CHECK_TAKE(NAME)           \
    hipError_t NAME(unsigned* out) {  \
        *out = 0;                     \
        return hipSuccess;            \
    }
#endif

// extents in bytes; "unknown" (a null pointer, or the normal build) passes every check
constexpr int64_t kExtentUnknown = INT64_MAX;
