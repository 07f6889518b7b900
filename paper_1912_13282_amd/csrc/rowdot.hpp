// Row dot products over the stencil layout: operators applied to a field
// (Sec. 2.3.1) and sparse matrix-vector products of the implicit system
// (Sec. 2.3.2) share them.
//
// One group of G lanes serves one row; a lane takes the positions gl, gl + G,
// ..., and issues the E index and value loads of a row segment, then the E
// gathers, before any arithmetic, so that they are in flight together.  The G
// partial sums are combined by a fixed butterfly: results do not depend on
// timing.
#pragma once

#include "common.hpp"

namespace rbf {

constexpr double kNaN = __builtin_nan("");

template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o);
    return v;
}

template <int G>
__device__ __forceinline__ bool group_any(bool b) {
    int v = b ? 1 : 0;
#pragma unroll
    for (int o = 1; o < G; o <<= 1) v |= __shfl_xor(v, o);
    return v != 0;
}

// acc[r] += sum over this lane's positions of w[r * stride + off + e] * x[idx[off + e]],
// e < n; bad is set when an index lies outside [0, n_x).
template <int G, int E, int R>
__device__ __forceinline__ void row_dot_partial(const int32_t* __restrict__ idx, const double* __restrict__ w,
                                                int64_t stride, int64_t off, int64_t n,
                                                const double* __restrict__ x, int64_t n_x, int gl, double (&acc)[R],
                                                bool& bad) {
    for (int64_t base = 0; base < n; base += G * E) {
        int j[E];
        double wv[R][E], xv[E];
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const int64_t e = base + gl + G * s;
            j[s] = (e < n) ? idx[off + e] : 0;
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int s = 0; s < E; ++s) {
                const int64_t e = base + gl + G * s;
                wv[r][s] = (e < n) ? w[r * stride + off + e] : 0.0;
            }
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const int64_t e = base + gl + G * s;
            const bool ok = j[s] >= 0 && (int64_t)j[s] < n_x;
            bad |= (e < n) && !ok;
            xv[s] = (e < n && ok) ? x[j[s]] : 0.0;
        }
#pragma unroll
        for (int s = 0; s < E; ++s)
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = fma(wv[r][s], xv[s], acc[r]);
    }
}

// Lanes per row and positions per lane for rows of at most n_max entries:
// G = 8 up to 64 positions (E = ceil(n_max / 8)), then 16 x 8, then 64 lanes
// looping by 4.  L<G, E>::launch(grid, stream, args...) is called with the grid
// of one G-lane group per row.
template <template <int, int> class L, typename... A>
hipError_t dispatch_row_shape(int n_max, int64_t N, hipStream_t s, A... args) {
    auto go = [&](auto gt, auto et) {
        constexpr int G = decltype(gt)::value, E = decltype(et)::value;
        const int64_t threads = N * G;
        return L<G, E>::launch(dim3((unsigned)((threads + 255) / 256)), s, args...);
    };
    using std::integral_constant;
    switch (n_max <= 64 ? (n_max + 7) / 8 : 0) {
        case 1: return go(integral_constant<int, 8>(), integral_constant<int, 1>());
        case 2: return go(integral_constant<int, 8>(), integral_constant<int, 2>());
        case 3: return go(integral_constant<int, 8>(), integral_constant<int, 3>());
        case 4: return go(integral_constant<int, 8>(), integral_constant<int, 4>());
        case 5: return go(integral_constant<int, 8>(), integral_constant<int, 5>());
        case 6: return go(integral_constant<int, 8>(), integral_constant<int, 6>());
        case 7: return go(integral_constant<int, 8>(), integral_constant<int, 7>());
        case 8: return go(integral_constant<int, 8>(), integral_constant<int, 8>());
        default: break;
    }
    if (n_max <= 128) return go(integral_constant<int, 16>(), integral_constant<int, 8>());
    return go(integral_constant<int, 64>(), integral_constant<int, 4>());
}

// true if the byte ranges [a, a + na) and [b, b + nb) overlap
inline bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

}  // namespace rbf
