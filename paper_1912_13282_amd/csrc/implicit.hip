// Implicit solution (Sec. 2.3.2): the system M u = r of eqs. (implicit-start)
// -(implicit-end) in the stencil layout, and its solution by BiCGStab with
// Jacobi row scaling or a block-Jacobi preconditioner, every step on the device.
//
// Block-Jacobi: the nodes are put in the order of a grid of cells (about 8
// nodes per cell in 2D, 16 in 3D) and cut into blocks of 64 consecutive nodes;
// the 64 x 64 diagonal block of M of every node block is inverted once (float32
// Gauss-Jordan with partial pivoting, one wavefront per block) and applied as a
// right preconditioner, M P^-1 y = r with x = P^-1 y, so the monitored residual
// is the true one.  Each iteration then adds two block products (one wavefront
// per block: a 16 KB inverse read coalesced, the vector entries broadcast by
// lane reads).
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
#include "cellorder.hpp"
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
    double rr, bb, tol2, rr0;
    double true_rr, true_bb;
    int status, half, iter, max_iter;
    int baddiag;
};

// A residual grown 10^6 times past the initial one ends the solve as DIVERGED.
constexpr double DIVERGE2 = 1e12;

struct SolveArgs {
    int64_t N;
    const int64_t* offsets;
    const int32_t* idx;
    const double* vals;
    int64_t nnz;
    const double* b;
    double* x;
    double *dinv, *r, *rh, *p, *v, *s, *t;
    double *ph, *sh;         // P^-1 p, P^-1 s (block-Jacobi)
    const double *xp, *xs;   // what the products take and x adds: p and s, or ph and sh
    const int32_t* perm;     // block-Jacobi: node ids in block order, or NULL
    const float* binv;       // block-Jacobi: inverses of the diagonal blocks
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
    st->rr = st->bb = st->rr0 = st->true_rr = st->true_bb = 0.0;
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
    const double* xin = MODE == SP_V ? a.xp : (MODE == SP_T ? a.xs : a.x);
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
                if (a.perm) {
                    a.ph[row] = 0.0;
                    a.sh[row] = 0.0;
                }
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
            a.x[i] += alpha * a.xp[i] + omega * a.xs[i];
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
        st->rr0 = tot[0];
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
        else if (tot[1] > DIVERGE2 * st->rr0)
            st->status = RBF_SOLVE_DIVERGED;
        else if (st->iter >= st->max_iter)
            st->status = RBF_SOLVE_MAXITER;
        else if (tot[0] == 0.0 || omega == 0.0)
            st->status = RBF_SOLVE_BREAKDOWN;
    } else {
        st->true_rr = tot[0];
        st->true_bb = tot[1];
    }
}

// ------------------------------------------------------------------ block-Jacobi
constexpr int BJ = 64;   // nodes per block (one per lane)
constexpr int BJ_PER_CELL_2D = 8, BJ_PER_CELL_3D = 16;

struct BjLayout {
    size_t perm, inv, binv, scratch, total;
    int64_t nblocks;
};

BjLayout bj_layout(int64_t N, int d) {
    BjLayout L;
    L.nblocks = (N + BJ - 1) / BJ;
    size_t o = 0;
    L.perm = o;
    o += rbf_align(sizeof(int32_t) * N);
    L.inv = o;
    o += rbf_align(sizeof(int32_t) * N);
    L.binv = o;
    o += rbf_align(sizeof(float) * BJ * BJ * L.nblocks);
    L.scratch = o;
    o += rbf_align(rbf::cell_order_ws(N, d));
    L.total = o;
    return L;
}

__global__ __launch_bounds__(256) void k_bj_inverse_perm(const int32_t* __restrict__ perm, int64_t N,
                                                         int32_t* __restrict__ inv) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N) inv[perm[p]] = (int32_t)p;
}

// Inverse of the diagonal block of node block b (one wavefront): lane l owns
// row l of [A | I] (A gathered from the row of node perm[64 b + l] through LDS,
// entries outside the block dropped, duplicates added), float32 Gauss-Jordan
// with partial pivoting (the pivot row by lane reads), then row k of the
// inverse, (I part) / U_kk of the row pivoted at step k, is stored in the
// layout of the product: element (k, j) at [j / 4][k][j % 4] of the block.  A
// block with a zero or non-finite pivot stores the inverse of its diagonal
// (Jacobi; identity where that is zero).  Padding rows past N are identity.
__global__ __launch_bounds__(256) void k_bj_setup(int64_t N, const int64_t* __restrict__ offsets,
                                                  const int32_t* __restrict__ idx, const double* __restrict__ vals,
                                                  int64_t nnz, const int32_t* __restrict__ perm,
                                                  const int32_t* __restrict__ inv, float* __restrict__ binv) {
    __shared__ float As[4][BJ][BJ + 1];
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    const int64_t b = (int64_t)blockIdx.x * 4 + wv;
    if (b * BJ >= N) return;
    const int64_t p = b * BJ + lane;
    const int node = p < N ? perm[p] : -1;
    float(&Ar)[BJ + 1] = As[wv][lane];
    for (int j = 0; j < BJ; ++j) Ar[j] = 0.0f;
    if (node < 0) {
        Ar[lane] = 1.0f;
    } else {
        const int64_t off = offsets[node], end = offsets[node + 1];
        if (off >= 0 && end >= off && end <= nnz)
            for (int64_t e = off; e < end; ++e) {
                const int c = idx[e];
                if (c < 0 || (int64_t)c >= N) continue;
                const int64_t q = inv[c];
                if (q / BJ == b) Ar[q % BJ] += (float)vals[e];
            }
    }
    float row[BJ], ii[BJ];
#pragma unroll
    for (int j = 0; j < BJ; ++j) {
        row[j] = Ar[j];
        ii[j] = (j == lane) ? 1.0f : 0.0f;
    }
    const float dg = Ar[lane];
    bool piv = false;
    int mystep = -1;
    float invd = 0.0f;
    int pmin = 0x7F7FFFFF, pmax = 0;
#pragma unroll
    for (int k = 0; k < BJ; ++k) {
        const int cand = piv ? -1 : __float_as_int(fabsf(row[k]));
        const int mi = wave_max_dpp_i(cand);
        pmin = min(pmin, mi);
        pmax = max(pmax, mi);
        const int pl = first_lane(ballot64(!piv && cand == mi));
        const bool me = lane == pl;
        const float inv_p = 1.0f / readlane_f(row[k], pl);
        if (me) {
            piv = true;
            mystep = k;
            invd = inv_p;
        }
        const float l = me ? 0.0f : row[k] * inv_p;
#pragma unroll
        for (int j = k + 1; j < BJ; ++j) row[j] = fmaf(-l, readlane_f(row[j], pl), row[j]);
#pragma unroll
        for (int j = 0; j < BJ; ++j) ii[j] = fmaf(-l, readlane_f(ii[j], pl), ii[j]);
    }
    const bool ok = pmin > 0 && pmax < 0x7F800000;  // wave-uniform
    float* B = binv + (size_t)b * BJ * BJ;
    if (ok) {
#pragma unroll
        for (int j4 = 0; j4 < BJ / 4; ++j4)
            *reinterpret_cast<float4*>(B + ((size_t)j4 * BJ + mystep) * 4) =
                make_float4(ii[4 * j4] * invd, ii[4 * j4 + 1] * invd, ii[4 * j4 + 2] * invd, ii[4 * j4 + 3] * invd);
    } else {
        const float di = (dg != 0.0f && isfinite(dg)) ? 1.0f / dg : 1.0f;
#pragma unroll
        for (int j4 = 0; j4 < BJ / 4; ++j4)
            *reinterpret_cast<float4*>(B + ((size_t)j4 * BJ + lane) * 4) =
                make_float4(4 * j4 == lane ? di : 0.0f, 4 * j4 + 1 == lane ? di : 0.0f, 4 * j4 + 2 == lane ? di : 0.0f,
                            4 * j4 + 3 == lane ? di : 0.0f);
    }
}

// out = P^-1 in, one wavefront per block (IN_S: the s vector, skipped once the
// half step has converged).
template <bool IN_S>
__global__ __launch_bounds__(256) void k_bj_apply(SolveArgs a) {
    SolveState* st = a.st;
    if (st->status != RUNNING) return;
    if (IN_S && st->half) return;
    const double* in = IN_S ? a.s : a.p;
    double* out = IN_S ? a.sh : a.ph;
    const int lane = lane_id();
    const int64_t nb = (a.N + BJ - 1) / BJ;
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); b < nb; b += nw) {
        const int64_t p = b * BJ + lane;
        const int node = p < a.N ? a.perm[p] : -1;
        const double y = node >= 0 ? in[node] : 0.0;
        const float* B = a.binv + (size_t)b * BJ * BJ;
        double acc = 0.0;
#pragma unroll
        for (int j4 = 0; j4 < BJ / 4; ++j4) {
            const float4 m = *reinterpret_cast<const float4*>(B + ((size_t)j4 * BJ + lane) * 4);
            acc = fma((double)m.x, readlane_d(y, 4 * j4), acc);
            acc = fma((double)m.y, readlane_d(y, 4 * j4 + 1), acc);
            acc = fma((double)m.z, readlane_d(y, 4 * j4 + 2), acc);
            acc = fma((double)m.w, readlane_d(y, 4 * j4 + 3), acc);
        }
        if (node >= 0) out[node] = acc;
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
        const dim3 gb(blocks_for(((a.N + BJ - 1) / BJ) * 64, 4096));   // one wavefront per node block
        const int nr = (int)gr.x, nv = (int)gv.x;
        switch (what) {
            case 0:
                hipLaunchKernelGGL((k_spmv<G, E, U, SP_R0>), gr, b, 0, s, a);
                hipLaunchKernelGGL((k_reduce<RD_R0>), one, b, 0, s, a, nr);
                break;
            case 1:
                hipLaunchKernelGGL((k_vec<VP>), gv, b, 0, s, a);
                if (a.perm) hipLaunchKernelGGL((k_bj_apply<false>), gb, b, 0, s, a);
                hipLaunchKernelGGL((k_spmv<G, E, U, SP_V>), gr, b, 0, s, a);
                hipLaunchKernelGGL((k_reduce<RD_V>), one, b, 0, s, a, nr);
                hipLaunchKernelGGL((k_vec<VS>), gv, b, 0, s, a);
                hipLaunchKernelGGL((k_reduce<RD_S>), one, b, 0, s, a, nv);
                if (a.perm) hipLaunchKernelGGL((k_bj_apply<true>), gb, b, 0, s, a);
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
           9 * rbf_align((size_t)N * sizeof(double));
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

extern "C" rbf_status rbf_block_jacobi_size(int64_t N, int d, size_t* bytes) {
    if (!bytes || N < 1) return RBF_EINVAL;
    if (d != 2 && d != 3) return RBF_EDIM;
    *bytes = bj_layout(N, d).total;
    return RBF_OK;
}

extern "C" rbf_status rbf_block_jacobi_setup(rbf_ctx* ctx, const double* X, int64_t N, int d, const int64_t* offsets,
                                             const int32_t* idx, const double* vals, int64_t nnz, void* pc,
                                             size_t pc_bytes) {
    if (!ctx || !X || !offsets || !vals || !pc || N < 1 || nnz < 0) return RBF_EINVAL;
    if (nnz > 0 && !idx) return RBF_EINVAL;
    if (d != 2 && d != 3) return RBF_EDIM;
    if (N > (int64_t)0x7FFFFFFF - 8192) return RBF_EINVAL;
    const BjLayout L = bj_layout(N, d);
    if (pc_bytes < L.total) return RBF_EWORKSPACE;
    RBF_HIP_CHECK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    char* w = (char*)pc;
    int32_t* perm = (int32_t*)(w + L.perm);
    int32_t* inv = (int32_t*)(w + L.inv);
    float* binv = (float*)(w + L.binv);
    RBF_HIP_CHECK(rbf::cell_order_enqueue(s, X, N, d, d == 3 ? BJ_PER_CELL_3D : BJ_PER_CELL_2D, w + L.scratch, perm));
    hipLaunchKernelGGL(k_bj_inverse_perm, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, perm, N, inv);
    hipLaunchKernelGGL(k_bj_setup, dim3((unsigned)((L.nblocks + 3) / 4)), dim3(256), 0, s, N, offsets, idx, vals, nnz,
                       perm, inv, binv);
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
                                   double tol, int max_iter, int precond, const void* pc, size_t pc_bytes,
                                   void* workspace, size_t ws_bytes, rbf_solve_info* info) {
    if (!ctx || !offsets || !vals || !rhs || !x || !workspace || N < 1 || nnz < 0 || n_max < 1) return RBF_EINVAL;
    if (nnz > 0 && !idx) return RBF_EINVAL;
    if (N > INT32_MAX + (int64_t)1) return RBF_EINVAL;
    if (!(tol >= 0.0) || max_iter < 0) return RBF_EINVAL;
    if (precond != RBF_PRECOND_NONE && precond != RBF_PRECOND_JACOBI && precond != RBF_PRECOND_BLOCK_JACOBI)
        return RBF_EINVAL;
    if (precond == RBF_PRECOND_BLOCK_JACOBI && !pc) return RBF_EINVAL;
    // the block-Jacobi data's size depends on d only through its scratch; the 3D
    // layout is the larger one, the 2D one is the minimum accepted
    if (precond == RBF_PRECOND_BLOCK_JACOBI && pc_bytes < bj_layout(N, 2).total) return RBF_EWORKSPACE;
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
    double** vecs[9] = {&a.dinv, &a.r, &a.rh, &a.p, &a.v, &a.s, &a.t, &a.ph, &a.sh};
    for (double** q : vecs) {
        *q = (double*)w;
        w += rbf_align((size_t)N * sizeof(double));
    }
    const bool bj = precond == RBF_PRECOND_BLOCK_JACOBI;
    if (bj) {
        const BjLayout L = bj_layout(N, 2);  // perm and inverses sit at the same offsets for d = 2 and 3
        a.perm = (const int32_t*)((const char*)pc + L.perm);
        a.binv = (const float*)((const char*)pc + L.binv);
    } else {
        a.perm = nullptr;
        a.binv = nullptr;
    }
    a.xp = bj ? a.ph : a.p;
    a.xs = bj ? a.sh : a.s;

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
