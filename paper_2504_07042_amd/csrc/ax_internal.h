// Internal helpers shared by the library's translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cmath>
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

// Debug builds compiled with -DAX_LDS_POISON=1 fill a kernel's LDS with all-ones bytes before
// its first use.  All-ones is a NaN in FP64, FP32 and FP16, so a read of an LDS word that no
// thread wrote in this launch reaches the output as NaN and fails any parity check.  Every thread
// of the block calls it, before anything else touches that LDS array.
#ifndef AX_LDS_POISON
#define AX_LDS_POISON 0
#endif
__device__ __forceinline__ void lds_poison(void* p, int bytes)
{
#if AX_LDS_POISON
    unsigned* w = (unsigned*)p;
    for (int q = (int)threadIdx.x; q < bytes / 4; q += (int)blockDim.x) w[q] = 0xffffffffu;
    __syncthreads();
#else
    (void)p;
    (void)bytes;
#endif
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
    // Even-odd split of a centro-antisymmetric D (D[N-a][N-n] = -D[a][n]), H = N1 / 2:
    //   P[a][n] = (D[a][n] + D[a][N-n]) / 2,  M[a][n] = (D[a][n] - D[a][N-n]) / 2  (a, n < H)
    //   Cm[a] = D[a][H], Rm[n] = D[H][n]  (middle column / row, odd N1 only)
    T P[(kMaxN1 / 2) * (kMaxN1 / 2)];
    T M[(kMaxN1 / 2) * (kMaxN1 / 2)];
    T Cm[kMaxN1 / 2];
    T Rm[kMaxN1 / 2];
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
    const int H = N1 / 2, N = N1 - 1;
    for (int q = 0; q < (kMaxN1 / 2) * (kMaxN1 / 2); ++q) b.P[q] = b.M[q] = T(0);
    for (int q = 0; q < kMaxN1 / 2; ++q) b.Cm[q] = b.Rm[q] = T(0);
    for (int a = 0; a < H; ++a)
        for (int n = 0; n < H; ++n) {
            b.P[a * H + n] = T(0.5 * (D[a * N1 + n] + D[a * N1 + (N - n)]));
            b.M[a * H + n] = T(0.5 * (D[a * N1 + n] - D[a * N1 + (N - n)]));
        }
    if (N1 % 2)
        for (int a = 0; a < H; ++a) {
            b.Cm[a] = T(D[a * N1 + H]);
            b.Rm[a] = T(D[H * N1 + a]);
        }
}

// True if D is centro-antisymmetric (D[N-a][N-n] = -D[a][n]) to within rounding, which every
// GLL differentiation matrix is; the kernels then use the even-odd split above.
inline bool centro_antisymmetric(int N1, const double* D)
{
    double mx = 0.0, dev = 0.0;
    for (int q = 0; q < N1 * N1; ++q) mx = mx > fabs(D[q]) ? mx : fabs(D[q]);
    for (int a = 0; a < N1; ++a)
        for (int n = 0; n < N1; ++n) {
            const double d = fabs(D[a * N1 + n] + D[(N1 - 1 - a) * N1 + (N1 - 1 - n)]);
            dev = dev > d ? dev : d;
        }
    return dev <= 1e-13 * mx;
}

// True if the nodes and weights are mirror-symmetric (xi[N-k] = -xi[k], w[N-k] = w[k], and a
// zero middle node for odd N1) exactly, as the GLL nodes built here are; the even-odd kernels
// then keep only half of them.  A null xi (not needed by the caller) only checks w.
inline bool symmetric_nodes(int N1, const double* xi, const double* w)
{
    if (!w) return false;
    for (int k = 0; k < N1; ++k)
        if ((xi && xi[N1 - 1 - k] != -xi[k]) || w[N1 - 1 - k] != w[k]) return false;
    return true;
}

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Launch variants of the AxLocal kernels per (N1, tuning kind TUNE_*, precision FP64/FP32); the
// fields are those of the public ax_tune.
struct TuneEntry {
    int kernel;     // AX_KERNEL_AUTO, AX_KERNEL_TILE or AX_KERNEL_ITEM
    int tile_alt;   // tile kernel: 0 default elements per work-group, 1 the alternative
    int item_alt;   // per-item kernels: 0 the 256-lane shape, 1 the order's alternative
    int waves_alt;  // single-mesh per-item kernel: 0 default register budget, 1 the alternative
    int grid_mult;  // persistent grid = grid_mult x resident capacity
};
TuneEntry tune_get(int N1, int kind, int prec);

// XCD-aware tile order.  Work-groups are dispatched round-robin over the 8 XCDs of the chip,
// each with its own L2, so tile b and tile b + 1 (which gather from the same cache lines of the
// source vector) would land on different L2s.  Tile index of work-group b: within each window of
// 8 S tiles, the work-groups of one XCD (b = x, x + 8, ...) take S consecutive tiles, so
// neighbouring tiles share an L2 while the 8 XCDs still stream from one region of memory at a
// time.  Work-groups past the last whole window keep the plain order.
#ifndef AX_XCD_CHUNK
#define AX_XCD_CHUNK 64
#endif
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t G)
{
    constexpr int64_t kXcd = 8, S = AX_XCD_CHUNK, W = kXcd * S;
    if (b >= (G / W) * W) return b;
    return (b / W) * W + (b % kXcd) * S + (b / kXcd) % S;
}


// Energy partials of the CG's fused operator (gathering AxLocal, one column): each work-group
// writes the energy sum of its elements to epart (epart_cap entries available); nparts receives
// the number of work-groups launched.
struct FusedOut {
    double* epart;
    int64_t epart_cap;
    int64_t nparts;
};

}  // namespace ax
