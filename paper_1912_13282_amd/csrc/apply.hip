// Explicit evaluation of stencil operators on a field (Sec. 2.3.1): the dot
// product of each node's weights with the field values at its stencil nodes,
// and the explicit Euler step of eqs. (exp-start)-(exp-end) built from it.
//
// Both passes are bandwidth-bound: every stencil index and weight is read once
// and the field is gathered (it stays in the caches when the node numbering is
// spatially coherent).  Rows are served by groups of lanes (rowdot.hpp).
#include "rowdot.hpp"

using namespace rbf;

namespace {

// out[r][row] = sum_p w[r][p] u[idx[p]] over the row's range
template <int G, int E, int R>
__global__ __launch_bounds__(256) void k_apply(int64_t N, const int64_t* __restrict__ offsets,
                                               const int32_t* __restrict__ idx, const double* __restrict__ w,
                                               int64_t nnz, const double* __restrict__ u, int64_t n_u,
                                               double* __restrict__ out) {
    const int gl = threadIdx.x & (G - 1);
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    if (row >= N) return;  // whole groups leave together (G divides 64)
    const int64_t off = offsets[row], end = offsets[row + 1];
    bool bad = off < 0 || end < off || end > nnz;
    const int64_t n = bad ? 0 : end - off;
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
    row_dot_partial<G, E, R>(idx, w, nnz, off, n, u, n_u, gl, acc, bad);
    bad = group_any<G>(bad);
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = group_sum<G>(acc[r]);
    if (gl < R) {
        double v = acc[0];
#pragma unroll
        for (int r = 1; r < R; ++r)
            if (gl == r) v = acc[r];
        out[(int64_t)gl * N + row] = bad ? kNaN : v;
    }
}

// One explicit Euler step: interior rows use the Laplacian weights, Neumann
// rows the normal-derivative weights c_j = sum_l n_l w_grad[l][p] (Sec. 2.3.1).
template <int G, int E>
__global__ __launch_bounds__(256) void k_explicit(int64_t N, int d, const int64_t* __restrict__ offsets,
                                                  const int32_t* __restrict__ idx, int64_t nnz,
                                                  const double* __restrict__ w_lap, const double* __restrict__ w_grad,
                                                  const uint8_t* __restrict__ kind, const double* __restrict__ normals,
                                                  const double* __restrict__ g, const double* __restrict__ src,
                                                  const double* __restrict__ u, double dt,
                                                  double* __restrict__ u_new) {
    const int gl = threadIdx.x & (G - 1);
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    if (row >= N) return;
    const int k = kind[row];  // uniform over the group: every branch below is too
    if (k == RBF_NODE_DIRICHLET) {
        if (gl == 0) u_new[row] = g ? g[row] : u[row];
        return;
    }
    if (k != RBF_NODE_INTERIOR && k != RBF_NODE_NEUMANN) {
        if (gl == 0) u_new[row] = kNaN;
        return;
    }
    const bool neu = k == RBF_NODE_NEUMANN;
    if (neu && (!w_grad || !normals)) {
        if (gl == 0) u_new[row] = kNaN;
        return;
    }
    const int64_t off = offsets[row], end = offsets[row + 1];
    bool bad = off < 0 || end < off || end > nnz || (neu && end == off);
    const int64_t n = bad ? 0 : end - off;
    double nrm[3] = {0.0, 0.0, 0.0};
    if (neu)
        for (int l = 0; l < d; ++l) nrm[l] = normals[row * d + l];
    double acc = 0.0, c0 = 0.0;
    for (int64_t base = 0; base < n; base += G * E) {
        int j[E];
        double wv[E], uv[E];
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const int64_t e = base + gl + G * s;
            j[s] = (e < n) ? idx[off + e] : 0;
        }
        if (!neu) {
#pragma unroll
            for (int s = 0; s < E; ++s) {
                const int64_t e = base + gl + G * s;
                wv[s] = (e < n) ? w_lap[off + e] : 0.0;
            }
        } else {
#pragma unroll
            for (int s = 0; s < E; ++s) {
                const int64_t e = base + gl + G * s;
                double c = 0.0;
                if (e < n)
                    for (int l = 0; l < d; ++l) c = fma(nrm[l], w_grad[l * nnz + off + e], c);
                wv[s] = c;
            }
        }
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const int64_t e = base + gl + G * s;
            const bool ok = j[s] >= 0 && (int64_t)j[s] < N;
            bad |= (e < n) && !ok;
            uv[s] = (e < n && ok) ? u[j[s]] : 0.0;
        }
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const int64_t e = base + gl + G * s;
            if (neu && e == 0) {
                c0 = wv[s];                   // the node's own coefficient
                bad |= j[s] != (int32_t)row;  // position 0 must be the node itself
            } else {
                acc = fma(wv[s], uv[s], acc);
            }
        }
    }
    bad = group_any<G>(bad);
    acc = group_sum<G>(acc);
    if (neu) c0 = group_sum<G>(c0);
    if (gl == 0) {
        double v;
        if (neu)
            v = ((g ? g[row] : 0.0) - acc) / c0;
        else
            v = u[row] + dt * (acc + (src ? src[row] : 0.0));
        u_new[row] = bad ? kNaN : v;
    }
}

// out[p] = sum_k coef[row][k] w[k][p] over the row's range (eq. gen-op)
template <int G, int E>
__global__ __launch_bounds__(256) void k_combine(int64_t N, const int64_t* __restrict__ offsets, int64_t nnz,
                                                 const double* __restrict__ w, int K,
                                                 const double* __restrict__ coef, double* __restrict__ out) {
    const int gl = threadIdx.x & (G - 1);
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    if (row >= N) return;
    const int64_t off = offsets[row], end = offsets[row + 1];
    if (off < 0 || end < off || end > nnz) return;
    double c[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) c[k] = (k < K) ? coef[row * K + k] : 0.0;
    for (int64_t e = gl; e < end - off; e += G) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < 10; ++k)
            if (k < K) v = fma(c[k], w[(int64_t)k * nnz + off + e], v);
        out[off + e] = v;
    }
}

template <int G, int E>
struct CombineL {
    static hipError_t launch(dim3 grid, hipStream_t s, int64_t N, const int64_t* offsets, int64_t nnz,
                             const double* w, int K, const double* coef, double* out) {
        hipLaunchKernelGGL((k_combine<G, E>), grid, dim3(256), 0, s, N, offsets, nnz, w, K, coef, out);
        return hipGetLastError();
    }
};

template <int R>
struct ApplyL {
    template <int G, int E>
    struct L {
        static hipError_t launch(dim3 grid, hipStream_t s, int64_t N, const int64_t* offsets, const int32_t* idx,
                                 const double* w, int64_t nnz, const double* u, int64_t n_u, double* out) {
            hipLaunchKernelGGL((k_apply<G, E, R>), grid, dim3(256), 0, s, N, offsets, idx, w, nnz, u, n_u, out);
            return hipGetLastError();
        }
    };
};

template <int G, int E>
struct ExplicitL {
    static hipError_t launch(dim3 grid, hipStream_t s, int64_t N, int d, const int64_t* offsets, const int32_t* idx,
                             int64_t nnz, const double* w_lap, const double* w_grad, const uint8_t* kind,
                             const double* normals, const double* g, const double* src, const double* u, double dt,
                             double* u_new) {
        hipLaunchKernelGGL((k_explicit<G, E>), grid, dim3(256), 0, s, N, d, offsets, idx, nnz, w_lap, w_grad, kind,
                           normals, g, src, u, dt, u_new);
        return hipGetLastError();
    }
};

}  // namespace

extern "C" rbf_status rbf_apply_operators(rbf_ctx* ctx, int64_t N, const int64_t* offsets, const int32_t* idx,
                                          const double* w, int n_ops, int64_t nnz, int n_max, const double* u,
                                          int64_t n_u, double* out) {
    if (!ctx || !offsets || !w || !u || !out || N < 1 || nnz < 0 || n_max < 1 || n_u < 1) return RBF_EINVAL;
    if (nnz > 0 && !idx) return RBF_EINVAL;
    if (n_ops < 1 || n_ops > 4) return RBF_EINVAL;
    if (n_u > INT32_MAX + (int64_t)1) return RBF_EINVAL;  // indices are int32
    const size_t out_b = (size_t)n_ops * (size_t)N * sizeof(double);
    if (ranges_overlap(out, out_b, u, (size_t)n_u * sizeof(double)) ||
        ranges_overlap(out, out_b, w, (size_t)n_ops * (size_t)nnz * sizeof(double)))
        return RBF_EINVAL;
    RBF_HIP_CHECK(hipSetDevice(ctx->device));
    hipError_t e;
    switch (n_ops) {
        case 1: e = dispatch_row_shape<ApplyL<1>::L>(n_max, N, ctx->stream, N, offsets, idx, w, nnz, u, n_u, out); break;
        case 2: e = dispatch_row_shape<ApplyL<2>::L>(n_max, N, ctx->stream, N, offsets, idx, w, nnz, u, n_u, out); break;
        case 3: e = dispatch_row_shape<ApplyL<3>::L>(n_max, N, ctx->stream, N, offsets, idx, w, nnz, u, n_u, out); break;
        default: e = dispatch_row_shape<ApplyL<4>::L>(n_max, N, ctx->stream, N, offsets, idx, w, nnz, u, n_u, out); break;
    }
    return e == hipSuccess ? RBF_OK : RBF_EHIP;
}

extern "C" rbf_status rbf_explicit_step(rbf_ctx* ctx, int64_t N, int d, const int64_t* offsets, const int32_t* idx,
                                        int64_t nnz, int n_max, const double* w_lap, const double* w_grad,
                                        const uint8_t* kind, const double* normals, const double* g, const double* s,
                                        const double* u, double dt, double* u_new) {
    if (!ctx || !offsets || !w_lap || !kind || !u || !u_new || N < 1 || nnz < 0 || n_max < 1) return RBF_EINVAL;
    if (nnz > 0 && !idx) return RBF_EINVAL;
    if (d != 2 && d != 3) return RBF_EDIM;
    if (N > INT32_MAX + (int64_t)1) return RBF_EINVAL;
    // Neumann rows need w_grad and normals; given neither, every Neumann row gets NaN
    if ((w_grad == nullptr) != (normals == nullptr)) return RBF_EINVAL;
    const size_t nb = (size_t)N * sizeof(double);
    if (ranges_overlap(u_new, nb, u, nb) || ranges_overlap(u_new, nb, w_lap, (size_t)nnz * sizeof(double))) return RBF_EINVAL;
    RBF_HIP_CHECK(hipSetDevice(ctx->device));
    const hipError_t e = dispatch_row_shape<ExplicitL>(n_max, N, ctx->stream, N, d, offsets, idx, nnz, w_lap, w_grad,
                                                   kind, normals, g, s, u, dt, u_new);
    return e == hipSuccess ? RBF_OK : RBF_EHIP;
}

extern "C" rbf_status rbf_combine_operators(rbf_ctx* ctx, int64_t N, const int64_t* offsets, int64_t nnz, int n_max,
                                            const double* w, int n_ops, const double* coef, double* out) {
    if (!ctx || !offsets || !w || !coef || !out || N < 1 || nnz < 0 || n_max < 1) return RBF_EINVAL;
    if (n_ops < 1 || n_ops > 10) return RBF_EINVAL;
    if (ranges_overlap(out, (size_t)nnz * sizeof(double), w, (size_t)n_ops * (size_t)nnz * sizeof(double)))
        return RBF_EINVAL;
    RBF_HIP_CHECK(hipSetDevice(ctx->device));
    const hipError_t e = dispatch_row_shape<CombineL>(n_max, N, ctx->stream, N, offsets, nnz, w, n_ops, coef, out);
    return e == hipSuccess ? RBF_OK : RBF_EHIP;
}
