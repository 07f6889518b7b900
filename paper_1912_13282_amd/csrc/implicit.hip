// Implicit solution (Sec. 2.3.2): the system M u = r of eqs. (implicit-start)
// -(implicit-end) in the stencil layout, and its solution by BiCGStab with
// Jacobi row scaling, every step on the device.
//
// One BiCGStab iteration (van der Vorst 1992) on the scaled system
// A = D^-1 M, b = D^-1 r:
//     p = r + beta (p - omega v)          k_vec<P>      beta = (rho / rho_prev)(alpha / omega)
//     v = A p,  alpha = rho / (rh . v)    k_spmv<V>
//     s = r - alpha v,  |s|^2             k_vec<S>      |s| small: x += alpha p, done
//     t = A s,  omega = (t . s)/(t . t)   k_spmv<T>
//     x += alpha p + omega s,  r = s - omega t,  rho = rh . r,  |r|^2      k_vec<X>
// The scalars live in device memory.  Each dot product is summed per block in
// a fixed order; a one-block kernel then adds the block sums, again in a fixed
// order, and updates the scalars (k_reduce), so no kernel waits for the host
// and the result does not depend on timing.  (Letting the last block of the
// producing kernel do it would need a device-scope release per block, which
// writes back the L2 of every XCD: far slower than the extra launch.)  Every
// kernel returns at once when the solve has ended; the host checks the state
// every CHECK_EVERY iterations.
#include "rowdot.hpp"

using namespace rbf;

namespace {

// ------------------------------------------------------------------ assembly
constexpr int AG = 8;  // lanes per row of the assembly

__global__ __launch_bounds__(256) void k_assemble(int64_t N, int d, const int64_t* __restrict__ offsets,
                                                  const int32_t* __restrict__ idx, int64_t nnz,
                                                  const double* __restrict__ w_lap, const double* __restrict__ w_grad,
                                                  const uint8_t* __restrict__ kind, const double* __restrict__ normals,
                                                  const double* __restrict__ f, const double* __restrict__ g,
                                                  double* __restrict__ vals, double* __restrict__ rhs) {
    const int gl = threadIdx.x & (AG - 1);
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / AG;
    if (row >= N) return;
    const int k = kind[row];
    const int64_t off = offsets[row], end = offsets[row + 1];
    const bool range_ok = off >= 0 && end >= off && end <= nnz;
    const int64_t n = range_ok ? end - off : 0;
    bool bad = !range_ok || (k != RBF_NODE_INTERIOR && k != RBF_NODE_DIRICHLET && k != RBF_NODE_NEUMANN);
    if (k == RBF_NODE_NEUMANN && (!w_grad || !normals)) bad = true;
    // boundary rows are built around position 0, which must be the node itself
    if (!bad && k != RBF_NODE_INTERIOR) bad = n == 0 || idx[off] != (int32_t)row;
    double nrm[3] = {0.0, 0.0, 0.0};
    if (!bad && k == RBF_NODE_NEUMANN)
        for (int l = 0; l < d; ++l) nrm[l] = normals[row * d + l];
    for (int64_t e = gl; e < n; e += AG) {
        double v;
        if (bad) {
            v = kNaN;
        } else if (k == RBF_NODE_INTERIOR) {
            v = w_lap[off + e];
        } else if (k == RBF_NODE_DIRICHLET) {
            v = (e == 0) ? 1.0 : 0.0;
        } else {
            double c = 0.0;
            for (int l = 0; l < d; ++l) c = fma(nrm[l], w_grad[l * nnz + off + e], c);
            v = c;
        }
        vals[off + e] = v;
    }
    if (gl == 0) {
        const double* src = (k == RBF_NODE_INTERIOR) ? f : g;
        rhs[row] = bad ? kNaN : (src ? src[row] : 0.0);
    }
}

// ------------------------------------------------------------------ solver
constexpr int RUNNING = -1;
constexpr int NBMAX = 2048;      // blocks of the row-product kernels (bounds the block sums)
constexpr int NBVEC = 2048;      // blocks of the vector kernels
constexpr int CHECK_EVERY = 16;  // iterations between host checks

struct SolveState {
    double rho, rho_prev, alpha, omega;
    double rr, bb, tol2;
    double true_rr, true_bb;
    int status, half, iter, max_iter;
    int baddiag;
};

struct SolveArgs {
    int64_t N;
    const int64_t* offsets;
    const int32_t* idx;
    const double* vals;
    int64_t nnz;
    const double* b;
    double* x;
    double *dinv, *r, *rh, *p, *v, *s, *t;
    double* part;
    SolveState* st;
};

// Block sums of K values per thread, written to part[blockIdx.x][K] by thread 0
// (fixed order: wave butterflies, then the four waves in order).  blockDim = 256.
template <int K>
__device__ __forceinline__ void block_partials(double (&v)[K], double* part) {
    __shared__ double red[K][4];
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < K; ++q) v[q] = wave_sum_d(v[q]);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int q = 0; q < K; ++q) red[q][wv] = v[q];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < K; ++q) part[(size_t)blockIdx.x * K + q] = (red[q][0] + red[q][1]) + (red[q][2] + red[q][3]);
}

__global__ void k_state_init(SolveState* st, int max_iter, double tol) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    st->rho = st->rho_prev = st->alpha = st->omega = 1.0;
    st->rr = st->bb = st->true_rr = st->true_bb = 0.0;
    st->tol2 = tol * tol;  // scaled by |b|^2 once that is known
    st->status = RUNNING;
    st->half = 0;
    st->iter = 0;
    st->max_iter = max_iter;
    st->baddiag = 0;
}

// dinv[i] = 1 / M[i][i] (Jacobi) or 1; a missing, zero or non-finite diagonal
// marks the state.
template <int G, int E>
__global__ __launch_bounds__(256) void k_diag(SolveArgs a, int jacobi) {
    const int gl = threadIdx.x & (G - 1);
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    if (row >= a.N) return;
    if (!jacobi) {
        if (gl == 0) a.dinv[row] = 1.0;
        return;
    }
    const int64_t off = a.offsets[row], end = a.offsets[row + 1];
    const bool range_ok = off >= 0 && end >= off && end <= a.nnz;
    const int64_t n = range_ok ? end - off : 0;
    int first = 0x7FFFFFFF;  // first position of the row in column `row`
    for (int64_t e = gl; e < n; e += G)
        if (a.idx[off + e] == (int32_t)row && e < first) first = (int)e;
#pragma unroll
    for (int o = 1; o < G; o <<= 1) first = min(first, __shfl_xor(first, o));
    if (gl == 0) {
        const double dval = (first < n) ? a.vals[off + first] : 0.0;
        const bool ok = dval != 0.0 && isfinite(dval);
        a.dinv[row] = ok ? 1.0 / dval : kNaN;
        if (!ok) a.st->baddiag = 1;  // every writer stores the same value
    }
}

enum { SP_R0, SP_V, SP_T, SP_TRUE };

// Row products of the matrix with a vector, grid-stride over rows, with the
// dot products each use needs:
//   SP_R0:   r = rh = D^-1 (b - M x), p = v = s = t = 0;  |r|^2, |D^-1 b|^2
//   SP_V:    v = D^-1 M p;  rh . v
//   SP_T:    t = D^-1 M s;  t . s, t . t
//   SP_TRUE: |b - M x|^2, |b|^2 (the unscaled residual of the result)
template <int G, int E, int U, int MODE>
__global__ __launch_bounds__(256) void k_spmv(SolveArgs a) {
    SolveState* st = a.st;
    if (MODE == SP_V || MODE == SP_T) {
        if (st->status != RUNNING) return;
    }
    if (MODE == SP_T && st->half) return;  // converged at the half step: omega = 0 (k_reduce)
    const double* xin = MODE == SP_V ? a.p : (MODE == SP_T ? a.s : a.x);
    const int gl = threadIdx.x & (G - 1);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x / G;
    double c0 = 0.0, c1 = 0.0;
    // U rows (row0, row0 + stride, ...) per pass: their loads are in flight together
    for (int64_t row0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G; row0 < a.N; row0 += U * stride) {
        int64_t off[U], n[U];
        bool bad[U];
        double acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = row0 + u * stride;
            const bool in = row < a.N;
            const int64_t o = in ? a.offsets[row] : 0, e = in ? a.offsets[row + 1] : 0;
            bad[u] = o < 0 || e < o || e > a.nnz;
            off[u] = o;
            n[u] = bad[u] ? 0 : e - o;
            acc[u] = 0.0;
        }
        const int64_t nmax = U == 1 ? n[0] : (n[0] > n[U - 1] ? n[0] : n[U - 1]);
        for (int64_t base = 0; base < nmax; base += G * E) {
            int j[U][E];
            double wv[U][E], xv[U][E];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int q = 0; q < E; ++q) {
                    const int64_t e = base + gl + G * q;
                    j[u][q] = (e < n[u]) ? a.idx[off[u] + e] : 0;
                    wv[u][q] = (e < n[u]) ? a.vals[off[u] + e] : 0.0;
                }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int q = 0; q < E; ++q) {
                    const int64_t e = base + gl + G * q;
                    const bool ok = j[u][q] >= 0 && (int64_t)j[u][q] < a.N;
                    bad[u] |= (e < n[u]) && !ok;
                    xv[u][q] = (e < n[u] && ok) ? xin[j[u][q]] : 0.0;
                }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int q = 0; q < E; ++q) acc[u] = fma(wv[u][q], xv[u][q], acc[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = row0 + u * stride;
            const bool rbad = group_any<G>(bad[u]);
            double ax = group_sum<G>(acc[u]);
            if (rbad) ax = kNaN;
            if (gl != 0 || row >= a.N) continue;
            if (MODE == SP_R0) {
                const double di = a.dinv[row], bi = a.b[row];
                const double ri = di * (bi - ax);
                a.r[row] = ri;
                a.rh[row] = ri;
                a.p[row] = 0.0;
                a.v[row] = 0.0;
                a.s[row] = 0.0;
                a.t[row] = 0.0;
                c0 += ri * ri;
                c1 += (di * bi) * (di * bi);
            } else if (MODE == SP_V) {
                const double vi = a.dinv[row] * ax;
                a.v[row] = vi;
                c0 += a.rh[row] * vi;
            } else if (MODE == SP_T) {
                const double ti = a.dinv[row] * ax;
                a.t[row] = ti;
                c0 += ti * a.s[row];
                c1 += ti * ti;
            } else {
                const double ei = a.b[row] - ax;
                c0 += ei * ei;
                c1 += a.b[row] * a.b[row];
            }
        }
    }
    double tot[2] = {c0, c1};
    block_partials<2>(tot, a.part);
}

enum { VP, VS, VX };

//   VP: p = r + beta (p - omega v)
//   VS: s = r - alpha v;  |s|^2 (half-step convergence)
//   VX: x += alpha p + omega s;  r = s - omega t;  rho = rh . r, |r|^2
template <int MODE>
__global__ __launch_bounds__(256) void k_vec(SolveArgs a) {
    SolveState* st = a.st;
    if (st->status != RUNNING) return;
    const double alpha = st->alpha, omega = st->omega;
    const double beta = (st->rho / st->rho_prev) * (alpha / omega);
    const int64_t N = a.N, stride = (int64_t)gridDim.x * blockDim.x;
    double c0 = 0.0, c1 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        if (MODE == VP) {
            a.p[i] = a.r[i] + beta * (a.p[i] - omega * a.v[i]);
        } else if (MODE == VS) {
            const double si = a.r[i] - alpha * a.v[i];
            a.s[i] = si;
            c0 += si * si;
        } else {
            const double si = a.s[i];
            a.x[i] += alpha * a.p[i] + omega * si;
            const double ri = si - omega * a.t[i];
            a.r[i] = ri;
            c0 += a.rh[i] * ri;
            c1 += ri * ri;
        }
    }
    if (MODE == VP) return;
    double tot[2] = {c0, c1};
    block_partials<2>(tot, a.part);
}

enum { RD_R0, RD_V, RD_S, RD_T, RD_X, RD_TRUE };

// Sum of the nb block sums (fixed order) and the scalar update of each step.
template <int MODE>
__global__ __launch_bounds__(256) void k_reduce(SolveArgs a, int nb) {
    SolveState* st = a.st;
    if (MODE != RD_R0 && MODE != RD_TRUE && st->status != RUNNING) return;
    if (MODE == RD_T && st->half) {
        if (threadIdx.x == 0) st->omega = 0.0;
        return;
    }
    __shared__ double red[2][4];
    // eight independent accumulators per thread keep eight loads in flight;
    // they are combined in a fixed order
    double q0[8], q1[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) q0[k] = q1[k] = 0.0;
    for (int b0 = threadIdx.x; b0 < nb; b0 += 8 * 256) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int b = b0 + k * 256;
            if (b < nb) {
                q0[k] += a.part[2 * b];
                q1[k] += a.part[2 * b + 1];
            }
        }
    }
    double s0 = ((q0[0] + q0[1]) + (q0[2] + q0[3])) + ((q0[4] + q0[5]) + (q0[6] + q0[7]));
    double s1 = ((q1[0] + q1[1]) + (q1[2] + q1[3])) + ((q1[4] + q1[5]) + (q1[6] + q1[7]));
    s0 = wave_sum_d(s0);
    s1 = wave_sum_d(s1);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wv] = s0;
        red[1][wv] = s1;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double tot[2] = {(red[0][0] + red[0][1]) + (red[0][2] + red[0][3]),
                           (red[1][0] + red[1][1]) + (red[1][2] + red[1][3])};
    if (MODE == RD_R0) {
        st->rr = tot[0];
        st->bb = tot[1];
        st->rho = tot[0];
        // relative to |b|; a zero right-hand side is measured against the start
        st->tol2 = st->tol2 * (tot[1] > 0.0 ? tot[1] : tot[0]);
        if (st->baddiag)
            st->status = RBF_SOLVE_BADDIAG;
        else if (!isfinite(tot[0]) || !isfinite(tot[1]))
            st->status = RBF_SOLVE_BREAKDOWN;
        else if (tot[0] <= st->tol2)
            st->status = RBF_SOLVE_CONVERGED;
        else if (st->max_iter <= 0)
            st->status = RBF_SOLVE_MAXITER;
    } else if (MODE == RD_V) {
        if (!(tot[0] != 0.0) || !isfinite(tot[0]))
            st->status = RBF_SOLVE_BREAKDOWN;
        else
            st->alpha = st->rho / tot[0];
    } else if (MODE == RD_S) {
        if (tot[0] <= st->tol2) st->half = 1;
    } else if (MODE == RD_T) {
        if (!(tot[1] > 0.0) || !isfinite(tot[0]) || !isfinite(tot[1]))
            st->status = RBF_SOLVE_BREAKDOWN;
        else
            st->omega = tot[0] / tot[1];
    } else if (MODE == RD_X) {
        const double omega = st->omega;
        st->rho_prev = st->rho;
        st->rho = tot[0];
        st->rr = tot[1];
        st->iter += 1;
        if (st->half || tot[1] <= st->tol2)
            st->status = RBF_SOLVE_CONVERGED;
        else if (!isfinite(tot[1]) || !isfinite(tot[0]))
            st->status = RBF_SOLVE_BREAKDOWN;
        else if (st->iter >= st->max_iter)
            st->status = RBF_SOLVE_MAXITER;
        else if (tot[0] == 0.0 || omega == 0.0)
            st->status = RBF_SOLVE_BREAKDOWN;
    } else {
        st->true_rr = tot[0];
        st->true_bb = tot[1];
    }
}

unsigned blocks_for(int64_t threads, int64_t cap) {
    const int64_t b = (threads + 255) / 256;
    return (unsigned)(b < cap ? (b > 0 ? b : 1) : cap);
}

template <int G, int E>
struct DiagL {
    static hipError_t launch(dim3 grid, hipStream_t s, SolveArgs a, int jacobi) {
        hipLaunchKernelGGL((k_diag<G, E>), grid, dim3(256), 0, s, a, jacobi);
        return hipGetLastError();
    }
};

// the solver kernels with rows of at most n_max entries
template <int G, int E, int U>
struct SolverL {
    static hipError_t launch(hipStream_t s, SolveArgs a, int what) {
        const dim3 gr(blocks_for(a.N * G, NBMAX)), gv(blocks_for(a.N, NBVEC)), b(256), one(1);
        const int nr = (int)gr.x, nv = (int)gv.x;
        switch (what) {
            case 0:
                hipLaunchKernelGGL((k_spmv<G, E, U, SP_R0>), gr, b, 0, s, a);
                hipLaunchKernelGGL((k_reduce<RD_R0>), one, b, 0, s, a, nr);
                break;
            case 1:
                hipLaunchKernelGGL((k_vec<VP>), gv, b, 0, s, a);
                hipLaunchKernelGGL((k_spmv<G, E, U, SP_V>), gr, b, 0, s, a);
                hipLaunchKernelGGL((k_reduce<RD_V>), one, b, 0, s, a, nr);
                hipLaunchKernelGGL((k_vec<VS>), gv, b, 0, s, a);
                hipLaunchKernelGGL((k_reduce<RD_S>), one, b, 0, s, a, nv);
                hipLaunchKernelGGL((k_spmv<G, E, U, SP_T>), gr, b, 0, s, a);
                hipLaunchKernelGGL((k_reduce<RD_T>), one, b, 0, s, a, nr);
                hipLaunchKernelGGL((k_vec<VX>), gv, b, 0, s, a);
                hipLaunchKernelGGL((k_reduce<RD_X>), one, b, 0, s, a, nv);
                break;
            default:
                hipLaunchKernelGGL((k_spmv<G, E, U, SP_TRUE>), gr, b, 0, s, a);
                hipLaunchKernelGGL((k_reduce<RD_TRUE>), one, b, 0, s, a, nr);
                break;
        }
        return hipGetLastError();
    }
};

// Row-product shape of the solver (measured on 1M-row systems): two lanes per
// row for rows of at most 10 entries, eight lanes with two rows in flight up
// to 64, then 16 and 64 lanes.  Longer rows than n_max are still summed whole.
hipError_t solver_launch(int n_max, hipStream_t s, SolveArgs a, int what) {
    switch (n_max <= 10 ? (n_max + 1) / 2 : 0) {
        case 1: return SolverL<2, 1, 1>::launch(s, a, what);
        case 2: return SolverL<2, 2, 1>::launch(s, a, what);
        case 3: return SolverL<2, 3, 1>::launch(s, a, what);
        case 4: return SolverL<2, 4, 1>::launch(s, a, what);
        case 5: return SolverL<2, 5, 1>::launch(s, a, what);
        default: break;
    }
    switch (n_max <= 64 ? (n_max + 7) / 8 : 0) {
        case 2: return SolverL<8, 2, 2>::launch(s, a, what);
        case 3: return SolverL<8, 3, 2>::launch(s, a, what);
        case 4: return SolverL<8, 4, 2>::launch(s, a, what);
        case 5: return SolverL<8, 5, 2>::launch(s, a, what);
        case 6: return SolverL<8, 6, 2>::launch(s, a, what);
        case 7: return SolverL<8, 7, 2>::launch(s, a, what);
        case 8: return SolverL<8, 8, 2>::launch(s, a, what);
        default: break;
    }
    if (n_max <= 128) return SolverL<16, 8, 1>::launch(s, a, what);
    return SolverL<64, 4, 1>::launch(s, a, what);
}

size_t solve_ws_bytes(int64_t N) {
    return rbf_align(sizeof(SolveState)) + rbf_align((size_t)NBMAX * 2 * sizeof(double)) +
           7 * rbf_align((size_t)N * sizeof(double));
}

}  // namespace

extern "C" rbf_status rbf_assemble_implicit(rbf_ctx* ctx, int64_t N, int d, const int64_t* offsets,
                                            const int32_t* idx, int64_t nnz, const double* w_lap,
                                            const double* w_grad, const uint8_t* kind, const double* normals,
                                            const double* f, const double* g, double* vals, double* rhs) {
    if (!ctx || !offsets || !w_lap || !kind || !vals || !rhs || N < 1 || nnz < 0) return RBF_EINVAL;
    if (nnz > 0 && !idx) return RBF_EINVAL;
    if (d != 2 && d != 3) return RBF_EDIM;
    if (N > INT32_MAX + (int64_t)1) return RBF_EINVAL;
    if ((w_grad == nullptr) != (normals == nullptr)) return RBF_EINVAL;
    const size_t vb = (size_t)nnz * sizeof(double);
    if (ranges_overlap(vals, vb, w_lap, vb) || (w_grad && ranges_overlap(vals, vb, w_grad, (size_t)d * vb)))
        return RBF_EINVAL;
    RBF_HIP_CHECK(hipSetDevice(ctx->device));
    const int64_t threads = N * AG;
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, ctx->stream, N, d, offsets,
                       idx, nnz, w_lap, w_grad, kind, normals, f, g, vals, rhs);
    RBF_LAUNCH_CHECK();
    return RBF_OK;
}

extern "C" rbf_status rbf_bicgstab_workspace(int64_t N, size_t* bytes) {
    if (!bytes || N < 1) return RBF_EINVAL;
    *bytes = solve_ws_bytes(N);
    return RBF_OK;
}

extern "C" rbf_status rbf_bicgstab(rbf_ctx* ctx, int64_t N, const int64_t* offsets, const int32_t* idx,
                                   const double* vals, int64_t nnz, int n_max, const double* rhs, double* x,
                                   double tol, int max_iter, int precond, void* workspace, size_t ws_bytes,
                                   rbf_solve_info* info) {
    if (!ctx || !offsets || !vals || !rhs || !x || !workspace || N < 1 || nnz < 0 || n_max < 1) return RBF_EINVAL;
    if (nnz > 0 && !idx) return RBF_EINVAL;
    if (N > INT32_MAX + (int64_t)1) return RBF_EINVAL;
    if (!(tol >= 0.0) || max_iter < 0) return RBF_EINVAL;
    if (precond != RBF_PRECOND_NONE && precond != RBF_PRECOND_JACOBI) return RBF_EINVAL;
    if (ws_bytes < solve_ws_bytes(N)) return RBF_EWORKSPACE;
    if (ranges_overlap(x, (size_t)N * sizeof(double), rhs, (size_t)N * sizeof(double))) return RBF_EINVAL;
    RBF_HIP_CHECK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;

    char* w = (char*)workspace;
    SolveArgs a;
    a.N = N;
    a.offsets = offsets;
    a.idx = idx;
    a.vals = vals;
    a.nnz = nnz;
    a.b = rhs;
    a.x = x;
    a.st = (SolveState*)w;
    w += rbf_align(sizeof(SolveState));
    a.part = (double*)w;
    w += rbf_align((size_t)NBMAX * 2 * sizeof(double));
    double** vecs[7] = {&a.dinv, &a.r, &a.rh, &a.p, &a.v, &a.s, &a.t};
    for (double** q : vecs) {
        *q = (double*)w;
        w += rbf_align((size_t)N * sizeof(double));
    }

    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, a.st, max_iter, tol);
    RBF_LAUNCH_CHECK();
    if (dispatch_row_shape<DiagL>(n_max, N, s, a, precond == RBF_PRECOND_JACOBI ? 1 : 0) != hipSuccess)
        return RBF_EHIP;
    if (solver_launch(n_max, s, a, 0) != hipSuccess) return RBF_EHIP;

    SolveState hs;
    int enqueued = 0;
    for (;;) {
        RBF_HIP_CHECK(hipMemcpyAsync(&hs, a.st, sizeof(hs), hipMemcpyDeviceToHost, s));
        RBF_HIP_CHECK(hipStreamSynchronize(s));
        if (hs.status != RUNNING || enqueued >= max_iter) break;
        const int chunk = max_iter - enqueued < CHECK_EVERY ? max_iter - enqueued : CHECK_EVERY;
        for (int k = 0; k < chunk; ++k)
            if (solver_launch(n_max, s, a, 1) != hipSuccess) return RBF_EHIP;
        enqueued += chunk;
    }
    if (solver_launch(n_max, s, a, 2) != hipSuccess) return RBF_EHIP;
    RBF_HIP_CHECK(hipMemcpyAsync(&hs, a.st, sizeof(hs), hipMemcpyDeviceToHost, s));
    RBF_HIP_CHECK(hipStreamSynchronize(s));
    if (info) {
        info->status = hs.status == RUNNING ? RBF_SOLVE_MAXITER : hs.status;
        info->iterations = hs.iter;
        info->residual = hs.bb > 0.0 ? sqrt(hs.rr / hs.bb) : sqrt(hs.rr);
        info->true_residual = hs.true_bb > 0.0 ? sqrt(hs.true_rr / hs.true_bb) : sqrt(hs.true_rr);
    }
    return RBF_OK;
}
