// Gather-scatter building blocks shared by the assembly and solver kernels (internal header).
#pragma once

#include "ax_internal.h"

namespace ax {

// Sums of the local copies of U global nodes g[u] (ascending local id each, the order of the plain
// loop).  The first copies of all U nodes are fetched with independent loads (offsets, then
// indices, then values), so the common single-copy node costs three overlapped round trips; the
// further copies of a shared node (up to 7 more: a vertex of a hexahedral mesh has 8) are fetched
// together too, any beyond those in a loop.  valid[u] false yields 0 without loads.
template <int U, typename T, typename IP>
__device__ __forceinline__ void gather_sums(const IP* __restrict__ gptr, const int32_t* __restrict__ gidx,
                                            const T* __restrict__ x, const int64_t* g, const bool* valid, T* s)
{
    int64_t q0[U], q1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        q0[u] = valid[u] ? (int64_t)gptr[g[u]] : 0;
        q1[u] = valid[u] ? (int64_t)gptr[g[u] + 1] : 0;
    }
    int32_t id[U];
#pragma unroll
    for (int u = 0; u < U; ++u) id[u] = q1[u] > q0[u] ? gidx[q0[u]] : 0;
#pragma unroll
    for (int u = 0; u < U; ++u) s[u] = q1[u] > q0[u] ? T(0) + x[id[u]] : T(0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (q1[u] - q0[u] < 2) continue;
        constexpr int kMore = 7;
        int32_t idm[kMore];
#pragma unroll
        for (int m = 0; m < kMore; ++m) idm[m] = q0[u] + 1 + m < q1[u] ? gidx[q0[u] + 1 + m] : -1;
        T v[kMore];
#pragma unroll
        for (int m = 0; m < kMore; ++m) v[m] = idm[m] >= 0 ? x[idm[m]] : T(0);
#pragma unroll
        for (int m = 0; m < kMore; ++m)
            if (idm[m] >= 0) s[u] += v[m];
        for (int64_t q = q0[u] + 1 + kMore; q < q1[u]; ++q) s[u] += x[gidx[q]];
    }
}

// nodes (or local entries) per thread and tile in the gather-scatter kernels
constexpr int kUnroll = 4;

}  // namespace ax
