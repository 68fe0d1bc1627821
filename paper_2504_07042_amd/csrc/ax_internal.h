// Internal helpers shared by the library's translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/axhosfem.h"

namespace ax {

// Largest supported N1 = N + 1 of the element kernels.
constexpr int kMaxN1 = 16;

// Thread-local message behind ax_last_error().
void set_error(const char* fmt, ...);
void clear_error();

inline int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    set_error("%s", buf);
    return code;
}

inline int hip_check(hipError_t e, const char* what)
{
    if (e != hipSuccess) return fail(AX_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return AX_OK;
}

#define AX_TRY(expr)              \
    do {                          \
        int _s = (expr);          \
        if (_s != AX_OK) return _s; \
    } while (0)

// Basis tables passed by value as kernel arguments (they land in the kernel-argument segment
// and are read with scalar loads: every lane of a wave reads the same entry).
template <typename T>
struct Basis {
    T D[kMaxN1 * kMaxN1];  // D[a * N1 + n]
    double xi[kMaxN1];
    double w[kMaxN1];
};

template <typename T>
inline void fill_basis(Basis<T>& b, int N1, const double* D, const double* xi, const double* w)
{
    for (int q = 0; q < kMaxN1 * kMaxN1; ++q) b.D[q] = T(0);
    for (int q = 0; q < kMaxN1; ++q) {
        b.xi[q] = 0.0;
        b.w[q] = 0.0;
    }
    for (int q = 0; q < N1 * N1; ++q) b.D[q] = T(D[q]);
    for (int q = 0; q < N1; ++q) {
        if (xi) b.xi[q] = xi[q];
        if (w) b.w[q] = w[q];
    }
}

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace ax
