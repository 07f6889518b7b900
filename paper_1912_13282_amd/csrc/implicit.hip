// Implicit solution (Sec. 2.3.2): the system M u = r of eqs. (implicit-start)
// -(implicit-end) in the stencil layout, and its solution by BiCGStab with
// Jacobi row scaling or a block-Jacobi preconditioner, every step on the device.
//
// Block-Jacobi: the nodes are put in the order of a grid of cells (about 8
// nodes per cell in 2D, 16 in 3D) and cut into blocks of 64 consecutive nodes;
// the 64 x 64 diagonal block of M of every node block is inverted once (float32
// Gauss-Jordan with partial pivoting, one wavefront per block), stored as
// float16 rows scaled by their largest entry, and applied as a right
// preconditioner, M P^-1 y = r with x = P^-1 y, so the monitored residual is the
// true one.  The solve runs in block order: M (rows renumbered, columns mapped),
// r and x are copied into that order in the workspace at the start and x is
// copied back at the end, so every vector pass is contiguous and the row
// products gather from spatially compact rows.  The block products are fused
// into the p and s updates (one wavefront per block: an 8 KB inverse read
// coalesced, the vector entries broadcast by lane reads).
//
// One BiCGStab iteration i (van der Vorst 1992) on the scaled system
// A = D^-1 M, b = D^-1 r (D = I for the block form, whose products take
// ph = P^-1 p and sh = P^-1 s, and whose x adds them), five launches:
//     rho_i = rh . r, status; p = r + beta (p - omega v)     k_vec<P> | k_bj_vec<P>
//         beta = (rho_i / rho_{i-1})(alpha / omega)
//     v = A p,  rh . v                                       k_spmv<V>
//     alpha = rho_i / (rh . v);  s = r - alpha v,  |s|^2     k_vec<S> | k_bj_vec<S>
//     t = A s,  t . s,  t . t                                k_spmv<T>
//     omega = (t . s)/(t . t) (0 if |s| is small: converged at the half step);
//     x += alpha p + omega s,  r = s - omega t,  rh . r, |r|^2          k_vec<X>
// Each dot product is summed per block in a fixed order; every block of the
// kernel that needs the scalar adds the producing kernel's block sums itself,
// in the same fixed order (so all blocks agree bit for bit), and block 0
// records it in the device-side state for later kernels and the host.  No
// kernel waits for the host and the result does not depend on timing.  A kernel
// never reads a state field that its own block 0 writes (rho alternates between
// two slots by iteration parity).  (Letting the last block of the
// producing kernel do it would need a device-scope release per block, which
// writes back the L2 of every XCD: far slower than the extra launch.)  Every
// kernel returns at once when the solve has ended.  The host enqueues
// CHECK_EVERY iterations at a time, each chunk followed by one single-block
// kernel that makes the next iteration's checks, and then reads the state.
// When the recursively updated residual has converged, the residual of x is
// computed afresh (the two drift apart by rounding over many iterations) and
// the iteration restarts from x if that one is above twice the tolerance.
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
constexpr int NBMAX = 1024;      // blocks of the row-product kernels (bounds the block sums)
constexpr int NBVEC = 1024;      // blocks of the vector kernels
static_assert(NBVEC <= NBMAX, "the vector kernels share the block sums of the row products");
constexpr int CHECK_EVERY = 16;  // iterations between host checks

struct SolveState {
    double rho[2];        // rho_i at [i & 1] (rho_0 = 1)
    double alpha, omega;  // of the latest iteration
    double rr, bb, tol2, rr0;
    double true_rr, true_bb;
    int status, half, iter, max_iter;
    int baddiag;
    int iter_base;  // iterations done before the latest restart
    int verified;   // convergence confirmed by a recomputed residual
};

// A residual grown 10^6 times past the initial one ends the solve as DIVERGED.
constexpr double DIVERGE2 = 1e12;
// On convergence the residual is recomputed from x; above RESTART_SLACK times
// the tolerance the iteration restarts from x, at most MAX_RESTARTS times (the
// recursively updated residual drifts from b - M x by rounding).
constexpr double RESTART_SLACK2 = 4.0;  // squared
constexpr int MAX_RESTARTS = 3;

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
    const _Float16* binv;    // block-Jacobi (the system in block order): inverses, rows scaled, or NULL
    const float* bscale;     // block-Jacobi: the row scales
    double* part;            // block sums of the row products (two per block)
    double* part_s;          // block sums of |s|^2 (one per block)
    double* part_x;          // block sums of rh . r and |r|^2 of the x update (two per block)
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

// Grid-stride work split by XCD.  The hardware hands workgroups to the eight
// XCDs in turn (workgroup b to XCD b mod 8), each with its own L2.  When the
// grid is a multiple of eight, the workgroups of XCD x take part x of the items
// (contiguous, a multiple of `align` long), so the vector entries a row
// product gathers, and the rows that the next pass reads, stay within the L2
// of one XCD instead of being fetched by all eight.  per_block items per
// workgroup and pass; this thread's (or lane group's) items are first,
// first + stride, ... below hi.
struct XcdSplit {
    int64_t first, hi, stride;
};
__device__ __forceinline__ XcdSplit xcd_split(int64_t n, int64_t align, int per_block, int sub) {
    const int nx = (gridDim.x % 8 == 0) ? 8 : 1;
    const int x = (int)(blockIdx.x % nx), lb = (int)(blockIdx.x / nx), lg = (int)(gridDim.x / nx);
    int64_t part = (n + nx - 1) / nx;
    part = (part + align - 1) / align * align;
    const int64_t lo = min(n, (int64_t)x * part);
    XcdSplit r;
    r.hi = min(n, lo + part);
    r.first = lo + (int64_t)lb * per_block + sub;
    r.stride = (int64_t)lg * per_block;
    return r;
}

__global__ void k_state_init(SolveState* st, int max_iter, double tol) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    st->rho[0] = st->rho[1] = st->alpha = st->omega = 1.0;
    st->rr = st->bb = st->rr0 = st->true_rr = st->true_bb = 0.0;
    st->tol2 = tol * tol;  // scaled by |b|^2 once that is known
    st->status = RUNNING;
    st->half = 0;
    st->iter = 0;
    st->max_iter = max_iter;
    st->baddiag = 0;
    st->iter_base = 0;
    st->verified = 0;
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
    const double* xin = MODE == SP_V ? a.xp : (MODE == SP_T ? a.xs : a.x);
    const int gl = threadIdx.x & (G - 1);
    const XcdSplit xs = xcd_split(a.N, 64, 256 / G, threadIdx.x / G);
    const int64_t stride = xs.stride;
    double c0 = 0.0, c1 = 0.0;
    // U rows (row0, row0 + stride, ...) per pass: their loads are in flight together
    for (int64_t row0 = xs.first; row0 < xs.hi; row0 += U * stride) {
        int64_t off[U], n[U];
        bool bad[U];
        double acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = row0 + u * stride;
            const bool in = row < xs.hi;
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
            if (gl != 0 || row >= xs.hi) continue;
            if (MODE == SP_R0) {
                const double di = a.dinv[row], bi = a.b[row];
                const double ri = di * (bi - ax);
                a.r[row] = ri;
                a.rh[row] = ri;
                a.p[row] = 0.0;
                a.v[row] = 0.0;
                a.s[row] = 0.0;
                a.t[row] = 0.0;
                if (a.binv) {
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

enum { RD_R0, RD_CHECK, RD_TRUE, RD_RESTART };

// Whether the solve is running, as one value for the whole block: block 0 of
// the same kernel may record an outcome while other blocks start, and all
// wavefronts of a block must take the same branch (the block sums use
// barriers, and a wavefront that went on alone would act on partial sums).
__device__ __forceinline__ bool block_running(const SolveState* st) {
    __shared__ int s;
    if (threadIdx.x == 0) s = st->status;
    __syncthreads();
    return s == RUNNING;
}

// Sums of the nb block sums part[b][0..1] and (S) the ns block sums ps[b], each
// in a fixed order, by the whole block; the totals are valid in every thread
// (all compute them from the same partial sums) and the function may be
// called again in the same kernel.
template <bool S>
__device__ __forceinline__ void sum_parts(const double* part, int nb, const double* ps, int ns, double (&tot)[3]) {
    __shared__ double red[3][4];
    // eight independent accumulators per thread and sum keep the loads of both
    // arrays in flight together; they are combined in a fixed order
    double q[3][8];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int k = 0; k < 8; ++k) q[c][k] = 0.0;
    const int nm = S && ns > nb ? ns : nb;
    for (int b0 = threadIdx.x; b0 < nm; b0 += 8 * 256) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int b = b0 + k * 256;
            if (b < nb) {
                q[0][k] += part[2 * b];
                q[1][k] += part[2 * b + 1];
            }
            if (S && b < ns) q[2][k] += ps[b];
        }
    }
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < (S ? 3 : 2); ++c) {
        double sc = ((q[c][0] + q[c][1]) + (q[c][2] + q[c][3])) + ((q[c][4] + q[c][5]) + (q[c][6] + q[c][7]));
        sc = wave_sum_d(sc);
        if ((threadIdx.x & 63) == 0) red[c][wv] = sc;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) tot[c] = (S || c < 2) ? (red[c][0] + red[c][1]) + (red[c][2] + red[c][3]) : 0.0;
    __syncthreads();  // red may be written again
}

// Start of iteration it (> 1, counted from the latest start or restart):
// rho_it = rh . r and |r|^2 of iteration it - 1
// from the nbx block sums of its x update, and the end-of-iteration checks;
// block 0 records rho_it, |r|^2, the iterations done and the outcome.  Every
// thread of the calling block gets rho_it; false: the solve has ended.  Called
// by every thread of a block that found the solve running.
__device__ bool iteration_head(const SolveArgs& a, int it, int nbx, double& rho_it) {
    SolveState* st = a.st;
    if (it <= 1) {  // from the initial residual
        rho_it = st->rho[1];
        return true;
    }
    double t[3];
    sum_parts<false>(a.part_x, nbx, nullptr, 0, t);
    const int done = st->iter_base + it - 1;
    int status = RUNNING;
    if (st->half || t[1] <= st->tol2)
        status = RBF_SOLVE_CONVERGED;
    else if (!isfinite(t[0]) || !isfinite(t[1]))
        status = RBF_SOLVE_BREAKDOWN;
    else if (t[1] > DIVERGE2 * st->rr0)
        status = RBF_SOLVE_DIVERGED;
    else if (done >= st->max_iter)
        status = RBF_SOLVE_MAXITER;
    else if (t[0] == 0.0 || st->omega == 0.0)
        status = RBF_SOLVE_BREAKDOWN;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rho[it & 1] = t[0];
        st->rr = t[1];
        st->iter = done;
        if (status != RUNNING) st->status = status;
    }
    rho_it = t[0];
    return status == RUNNING;
}

// alpha = rho_it / (rh . v) from the nbv block sums of the row product v = A p;
// block 0 records it or the breakdown.  Uniform; false: breakdown.
__device__ bool half_step_alpha(const SolveArgs& a, int it, int nbv, double& alpha) {
    double t[3];
    sum_parts<false>(a.part, nbv, nullptr, 0, t);
    const bool ok = t[0] != 0.0 && isfinite(t[0]);
    alpha = ok ? a.st->rho[it & 1] / t[0] : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (ok)
            a.st->alpha = alpha;
        else
            a.st->status = RBF_SOLVE_BREAKDOWN;
    }
    return ok;
}

// omega = (t . s) / (t . t) from the nbt block sums of t = A s, or 0 when |s|^2
// (ns block sums) is within the tolerance (converged at the half step); block 0
// records omega and the half flag or the breakdown.  Uniform; false: breakdown.
__device__ bool full_step_omega(const SolveArgs& a, int nbt, int ns, double& omega) {
    SolveState* st = a.st;
    double t[3];
    sum_parts<true>(a.part, nbt, a.part_s, ns, t);
    const bool half = t[2] <= st->tol2;
    const bool ok = half || (t[1] > 0.0 && isfinite(t[0]) && isfinite(t[1]));
    omega = half ? 0.0 : (ok ? t[0] / t[1] : 0.0);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (!ok) {
            st->status = RBF_SOLVE_BREAKDOWN;
        } else {
            st->omega = omega;
            if (half) st->half = 1;
        }
    }
    return ok;
}

enum { VP, VS, VX };

// Vector passes of iteration it; nb (and ns) count the block sums of the
// kernel(s) before, whose scalars they finish (see the header comment):
//   VP: head of the iteration, p = r + beta (p - omega v)
//   VS: alpha;  s = r - alpha v;  |s|^2
//   VX: omega;  x += alpha p + omega s;  r = s - omega t;  rh . r, |r|^2
template <int MODE>
__global__ __launch_bounds__(256) void k_vec(SolveArgs a, int it, int nb, int ns) {
    SolveState* st = a.st;
    if (!block_running(st)) return;
    double alpha = 0.0, omega = 0.0, beta = 0.0;
    if (MODE == VP) {
        double rho_it;
        if (!iteration_head(a, it, nb, rho_it)) return;
        omega = st->omega;
        beta = (rho_it / st->rho[(it - 1) & 1]) * (st->alpha / omega);
    } else if (MODE == VS) {
        if (!half_step_alpha(a, it, nb, alpha)) return;
    } else {
        alpha = st->alpha;
        if (!full_step_omega(a, nb, ns, omega)) return;
    }
    const XcdSplit xs = xcd_split(a.N, 64, 256, threadIdx.x);
    double c0 = 0.0, c1 = 0.0;
    for (int64_t i = xs.first; i < xs.hi; i += xs.stride) {
        if (MODE == VP) {
            a.p[i] = a.r[i] + beta * (a.p[i] - omega * a.v[i]);
        } else if (MODE == VS) {
            const double si = a.r[i] - alpha * a.v[i];
            a.s[i] = si;
            c0 += si * si;
        } else {
            const double si = a.s[i];
            a.x[i] += alpha * a.xp[i] + omega * a.xs[i];
            const double ri = omega != 0.0 ? si - omega * a.t[i] : si;  // omega = 0: converged at s
            a.r[i] = ri;
            c0 += a.rh[i] * ri;
            c1 += ri * ri;
        }
    }
    if (MODE == VP) return;
    if (MODE == VS) {
        double tot[1] = {c0};
        block_partials<1>(tot, a.part_s);
    } else {
        double tot[2] = {c0, c1};
        block_partials<2>(tot, a.part_x);
    }
}

// Sum of the nb block sums (fixed order) and the scalar update of the steps
// outside the iteration: the start (RD_R0), the end-of-chunk check of iteration
// it (RD_CHECK, what the next iteration's head would record), the check of a
// converged x and the restart from it (RD_RESTART), and the residual of the
// result (RD_TRUE).
template <int MODE>
__global__ __launch_bounds__(256) void k_reduce(SolveArgs a, int nb, int it) {
    SolveState* st = a.st;
    if (MODE == RD_CHECK) {
        double rho_it;
        if (block_running(st)) iteration_head(a, it, nb, rho_it);
        return;
    }
    double tot[3];
    sum_parts<false>(a.part, nb, nullptr, 0, tot);
    if (threadIdx.x != 0) return;
    if (MODE == RD_R0) {
        st->rr = tot[0];
        st->rr0 = tot[0];
        st->bb = tot[1];
        st->rho[1] = tot[0];
        // relative to |b|; a zero right-hand side is measured against the start
        st->tol2 = st->tol2 * (tot[1] > 0.0 ? tot[1] : tot[0]);
        if (st->baddiag)
            st->status = RBF_SOLVE_BADDIAG;
        else if (!isfinite(tot[0]) || !isfinite(tot[1]))
            st->status = RBF_SOLVE_BREAKDOWN;
        else if (tot[0] <= st->tol2) {
            st->status = RBF_SOLVE_CONVERGED;
            st->verified = 1;
        } else if (st->max_iter <= 0) {
            st->status = RBF_SOLVE_MAXITER;
        }
    } else if (MODE == RD_RESTART) {
        // the residual recomputed from x after the recursion reported convergence
        // (r, rh, p, v, s, t already reset by the row product)
        if (!isfinite(tot[0])) {
            st->status = RBF_SOLVE_BREAKDOWN;
        } else if (tot[0] <= RESTART_SLACK2 * st->tol2) {
            st->verified = 1;  // stays converged, with the monitored residual
        } else {
            st->rr = tot[0];
            st->rho[1] = tot[0];
            st->rho[0] = st->alpha = st->omega = 1.0;
            st->half = 0;
            st->iter_base = st->iter;
            st->status = RUNNING;
        }
    } else {
        st->true_rr = tot[0];
        st->true_bb = tot[1];
    }
}

// ------------------------------------------------------------------ block-Jacobi
constexpr int BJ = 64;   // nodes per block (one per lane)
constexpr int BJ_PER_CELL_2D = 8, BJ_PER_CELL_3D = 16;

struct BjLayout {
    size_t perm, inv, binv, bscale, scratch, total;
    int64_t nblocks;
};

// float16 entries of an inverse row scaled by its largest magnitude; element
// (k, j) of block b at binv[b][j / 8][k][j % 8], the scale of row k at
// bscale[b][k]
typedef _Float16 half8 __attribute__((ext_vector_type(8)));

BjLayout bj_layout(int64_t N, int d) {
    BjLayout L;
    L.nblocks = (N + BJ - 1) / BJ;
    size_t o = 0;
    L.perm = o;
    o += rbf_align(sizeof(int32_t) * N);
    L.inv = o;
    o += rbf_align(sizeof(int32_t) * N);
    L.binv = o;
    o += rbf_align(sizeof(_Float16) * BJ * BJ * L.nblocks);
    L.bscale = o;
    o += rbf_align(sizeof(float) * BJ * L.nblocks);
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
// inverse, (I part) / U_kk of the row pivoted at step k, is divided by its
// largest magnitude and stored as float16 in the layout of the product, the
// scale beside it.  A block with a zero or non-finite pivot stores the inverse
// of its diagonal (Jacobi; identity where that is zero).  Padding rows past N
// are identity.
__global__ __launch_bounds__(256) void k_bj_setup(int64_t N, const int64_t* __restrict__ offsets,
                                                  const int32_t* __restrict__ idx, const double* __restrict__ vals,
                                                  int64_t nnz, const int32_t* __restrict__ perm,
                                                  const int32_t* __restrict__ inv, _Float16* __restrict__ binv,
                                                  float* __restrict__ bscale) {
    __shared__ float As[4][BJ][BJ + 1];
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    const int64_t b = (int64_t)blockIdx.x * 4 + wv;
    if (b * BJ >= N) return;
    const int64_t p = b * BJ + lane;
    const int32_t pn = p < N ? perm[p] : -1;
    const int node = (pn >= 0 && (int64_t)pn < N) ? pn : -1;
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
    _Float16* B = binv + (size_t)b * BJ * BJ;
    if (ok) {
        float m = 0.0f;
#pragma unroll
        for (int j = 0; j < BJ; ++j) m = fmaxf(m, fabsf(ii[j]));
        const float sc = (m > 0.0f && isfinite(m)) ? m : 1.0f;
        const float is = 1.0f / sc;
#pragma unroll
        for (int j8 = 0; j8 < BJ / 8; ++j8) {
            half8 h;
#pragma unroll
            for (int q = 0; q < 8; ++q) h[q] = (_Float16)(ii[8 * j8 + q] * is);
            *reinterpret_cast<half8*>(B + ((size_t)j8 * BJ + mystep) * 8) = h;
        }
        bscale[b * BJ + mystep] = sc * invd;
    } else {
        const float di = (dg != 0.0f && isfinite(dg)) ? 1.0f / dg : 1.0f;
#pragma unroll
        for (int j8 = 0; j8 < BJ / 8; ++j8) {
            half8 h;
#pragma unroll
            for (int q = 0; q < 8; ++q) h[q] = (_Float16)(8 * j8 + q == lane ? 1.0f : 0.0f);
            *reinterpret_cast<half8*>(B + ((size_t)j8 * BJ + lane) * 8) = h;
        }
        bscale[b * BJ + lane] = di;
    }
}

// The p and s updates of the block form (the system in block order, one
// wavefront per node block), each followed by its block product (the scalars
// as in k_vec: iteration head before p, alpha before s):
//   S = false:  p = r + beta (p - omega v),  ph = P^-1 p
//   S = true:   s = r - alpha v,  sh = P^-1 s,  |s|^2
// Row k of a block product is scale_k * sum_j h_kj y_j in float64 over the
// float16 entries h_kj; y_j comes from lane j by lane reads.
template <bool S>
__global__ __launch_bounds__(256) void k_bj_vec(SolveArgs a, int it, int nb) {
    SolveState* st = a.st;
    if (!block_running(st)) return;
    double alpha = 0.0, omega = 0.0, beta = 0.0;
    if (S) {
        if (!half_step_alpha(a, it, nb, alpha)) return;
    } else {
        double rho_it;
        if (!iteration_head(a, it, nb, rho_it)) return;
        omega = st->omega;
        beta = (rho_it / st->rho[(it - 1) & 1]) * (st->alpha / omega);
    }
    const int lane = lane_id();
    // node blocks split by XCD as the rows of the other passes (parts of
    // ceil(N / 512) blocks = ceil(N / 8) rows rounded up to 64)
    const XcdSplit xs = xcd_split((a.N + BJ - 1) / BJ, 1, 4, threadIdx.x >> 6);
    double c0 = 0.0;
    for (int64_t b = xs.first; b < xs.hi; b += xs.stride) {
        const int64_t q = b * BJ + lane;
        const bool in = q < a.N;
        double y = 0.0;
        if (in) {
            if (S) {
                y = a.r[q] - alpha * a.v[q];
                a.s[q] = y;
                c0 += y * y;
            } else {
                y = a.r[q] + beta * (a.p[q] - omega * a.v[q]);
                a.p[q] = y;
            }
        }
        const half8* B = reinterpret_cast<const half8*>(a.binv + (size_t)b * BJ * BJ) + lane;
        half8 h[BJ / 8];
#pragma unroll
        for (int j8 = 0; j8 < BJ / 8; ++j8) h[j8] = B[(size_t)j8 * BJ];
        const float sc = a.bscale[b * BJ + lane];
        double acc = 0.0;
#pragma unroll
        for (int j8 = 0; j8 < BJ / 8; ++j8)
#pragma unroll
            for (int e = 0; e < 8; ++e) acc = fma((double)(float)h[j8][e], readlane_d(y, 8 * j8 + e), acc);
        if (in) (S ? a.sh : a.ph)[q] = (double)sc * acc;
    }
    if (S) {
        double tot[1] = {c0};
        block_partials<1>(tot, a.part_s);
    }
}

// workgroups of 256 threads for `threads`, at most cap (a multiple of 8); from
// 64 on a multiple of 8, so the work splits by XCD
unsigned blocks_for(int64_t threads, int64_t cap) {
    int64_t b = (threads + 255) / 256;
    if (b >= 64) b = (b + 7) / 8 * 8;
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
    // what: 0 start, 1 iteration it, 2 end-of-chunk check before iteration it,
    // 3 residual of the result, 4 check of a converged x (restart)
    static hipError_t launch(hipStream_t s, SolveArgs a, int what, int it) {
        const dim3 gr(blocks_for(a.N * G, NBMAX)), gv(blocks_for(a.N, NBVEC)), b(256), one(1);
        // one wavefront per node block, at most NBVEC blocks (the |s|^2 block sums)
        const dim3 gb(blocks_for(((a.N + BJ - 1) / BJ) * 64, NBVEC));
        const int nr = (int)gr.x, nv = (int)gv.x, ns = a.binv ? (int)gb.x : nv;
        switch (what) {
            case 0:
                hipLaunchKernelGGL((k_spmv<G, E, U, SP_R0>), gr, b, 0, s, a);
                hipLaunchKernelGGL((k_reduce<RD_R0>), one, b, 0, s, a, nr, 0);
                break;
            case 1:
                if (a.binv)
                    hipLaunchKernelGGL((k_bj_vec<false>), gb, b, 0, s, a, it, nv);
                else
                    hipLaunchKernelGGL((k_vec<VP>), gv, b, 0, s, a, it, nv, 0);
                hipLaunchKernelGGL((k_spmv<G, E, U, SP_V>), gr, b, 0, s, a);
                if (a.binv)
                    hipLaunchKernelGGL((k_bj_vec<true>), gb, b, 0, s, a, it, nr);
                else
                    hipLaunchKernelGGL((k_vec<VS>), gv, b, 0, s, a, it, nr, 0);
                hipLaunchKernelGGL((k_spmv<G, E, U, SP_T>), gr, b, 0, s, a);
                hipLaunchKernelGGL((k_vec<VX>), gv, b, 0, s, a, it, nr, ns);
                break;
            case 2:
                hipLaunchKernelGGL((k_reduce<RD_CHECK>), one, b, 0, s, a, nv, it);
                break;
            case 4:
                hipLaunchKernelGGL((k_spmv<G, E, U, SP_R0>), gr, b, 0, s, a);
                hipLaunchKernelGGL((k_reduce<RD_RESTART>), one, b, 0, s, a, nr, 0);
                break;
            default:
                hipLaunchKernelGGL((k_spmv<G, E, U, SP_TRUE>), gr, b, 0, s, a);
                hipLaunchKernelGGL((k_reduce<RD_TRUE>), one, b, 0, s, a, nr, 0);
                break;
        }
        return hipGetLastError();
    }
};

// Row-product shape of the solver (measured on 1M-row systems): two lanes per
// row for rows of at most 10 entries, eight lanes with two rows in flight up
// to 64, then 16 and 64 lanes.  Longer rows than n_max are still summed whole.
hipError_t solver_launch(int n_max, hipStream_t s, SolveArgs a, int what, int it = 0) {
    switch (n_max <= 10 ? (n_max + 1) / 2 : 0) {
        case 1: return SolverL<2, 1, 1>::launch(s, a, what, it);
        case 2: return SolverL<2, 2, 1>::launch(s, a, what, it);
        case 3: return SolverL<2, 3, 1>::launch(s, a, what, it);
        case 4: return SolverL<2, 4, 1>::launch(s, a, what, it);
        case 5: return SolverL<2, 5, 1>::launch(s, a, what, it);
        default: break;
    }
    switch (n_max <= 64 ? (n_max + 7) / 8 : 0) {
        case 2: return SolverL<8, 2, 2>::launch(s, a, what, it);
        case 3: return SolverL<8, 3, 2>::launch(s, a, what, it);
        case 4: return SolverL<8, 4, 2>::launch(s, a, what, it);
        case 5: return SolverL<8, 5, 2>::launch(s, a, what, it);
        case 6: return SolverL<8, 6, 2>::launch(s, a, what, it);
        case 7: return SolverL<8, 7, 2>::launch(s, a, what, it);
        case 8: return SolverL<8, 8, 2>::launch(s, a, what, it);
        default: break;
    }
    if (n_max <= 128) return SolverL<16, 8, 1>::launch(s, a, what, it);
    return SolverL<64, 4, 1>::launch(s, a, what, it);
}

// ------------------------------------------------------------------ block order
// The block-Jacobi solve works on a copy of the system in block order: row q of
// the copy is row perm[q] of M with every column c replaced by inv[c] (invalid
// columns stay invalid, -1); a row with an invalid range becomes the single
// invalid entry -1, so the row products still give NaN for it.  The copy holds
// nnz + N entries: enough for rows that partition [0, nnz) plus one entry per
// invalid row; rows of overlapping ranges past that capacity are not copied
// and fall outside the copy's range check (NaN rows), as invalid rows do.
constexpr int SCAN_B = 1024;  // elements per block of the offset scan

// len[q] = length of row perm[q] (1 for an invalid range), written to poff[q + 1]
__global__ __launch_bounds__(256) void k_perm_len(int64_t N, const int64_t* __restrict__ offsets, int64_t nnz,
                                                  const int32_t* __restrict__ perm, int64_t* __restrict__ poff) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q == 0) poff[0] = 0;
    if (q >= N) return;
    const int64_t src = perm[q];
    if (src < 0 || src >= N) {  // not a permutation of [0, N): the row is invalid
        poff[q + 1] = 1;
        return;
    }
    const int64_t o = offsets[src], e = offsets[src + 1];
    poff[q + 1] = (o < 0 || e < o || e > nnz) ? 1 : e - o;
}

// Inclusive scan of v[0, n) in blocks of SCAN_B: scan within each block, block
// totals to bsum (k_scan_local); exclusive scan of the totals by one block
// (k_scan_top); totals of the preceding blocks added (k_scan_add).
__global__ __launch_bounds__(256) void k_scan_local(int64_t* __restrict__ v, int64_t n, int64_t* __restrict__ bsum) {
    __shared__ int64_t wsum[4];
    const int64_t base = (int64_t)blockIdx.x * SCAN_B + threadIdx.x * 4;
    int64_t e[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) e[k] = base + k < n ? v[base + k] : 0;
#pragma unroll
    for (int k = 1; k < 4; ++k) e[k] += e[k - 1];
    // inclusive scan of the thread totals across the wave, then across the waves
    int64_t t = e[3];
    const int lane = lane_id(), wv = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t u = __shfl_up(t, o);
        if (lane >= o) t += u;
    }
    if (lane == 63) wsum[wv] = t;
    __syncthreads();
    int64_t before = t - e[3];
    for (int w2 = 0; w2 < wv; ++w2) before += wsum[w2];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + k < n) v[base + k] = e[k] + before;
    if (threadIdx.x == 255) bsum[blockIdx.x] = before + e[3];
}

__global__ __launch_bounds__(256) void k_scan_top(int64_t* __restrict__ bsum, int64_t nb) {
    __shared__ int64_t wsum[4];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    for (int64_t b0 = 0; b0 < nb; b0 += 256) {
        const int64_t i = b0 + threadIdx.x;
        const int64_t x = i < nb ? bsum[i] : 0;
        int64_t t = x;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t u = __shfl_up(t, o);
            if (lane >= o) t += u;
        }
        if (lane == 63) wsum[wv] = t;
        __syncthreads();
        int64_t before = carry + t - x;
        for (int w2 = 0; w2 < wv; ++w2) before += wsum[w2];
        if (i < nb) bsum[i] = before;  // exclusive
        __syncthreads();
        if (threadIdx.x == 255) carry = before + x;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_scan_add(int64_t* __restrict__ v, int64_t n,
                                                  const int64_t* __restrict__ bsum) {
    const int64_t add = bsum[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * SCAN_B;
    for (int k = threadIdx.x; k < SCAN_B; k += 256)
        if (base + k < n) v[base + k] += add;
}

// row q of the copy (eight lanes per row)
__global__ __launch_bounds__(256) void k_perm_rows(int64_t N, const int64_t* __restrict__ offsets,
                                                   const int32_t* __restrict__ idx, const double* __restrict__ vals,
                                                   int64_t nnz, const int32_t* __restrict__ perm,
                                                   const int32_t* __restrict__ inv, const int64_t* __restrict__ poff,
                                                   int32_t* __restrict__ pidx, double* __restrict__ pvals,
                                                   int64_t cap) {
    const int gl = threadIdx.x & 7;
    const int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3;
    if (q >= N) return;
    const int64_t src = perm[q];
    const int64_t dst = poff[q];
    if (poff[q + 1] > cap) return;
    const bool sok = src >= 0 && src < N;
    const int64_t o = sok ? offsets[src] : -1, e = sok ? offsets[src + 1] : -1;
    if (o < 0 || e < o || e > nnz) {
        if (gl == 0) {
            pidx[dst] = -1;
            pvals[dst] = 0.0;
        }
        return;
    }
    for (int64_t k = gl; k < e - o; k += 8) {
        const int32_t c = idx[o + k];
        pidx[dst + k] = (c >= 0 && (int64_t)c < N) ? inv[c] : -1;
        pvals[dst + k] = vals[o + k];
    }
}

// TO: out[q] = in[perm[q]] for the two vectors; else out[perm[q]] = in[q]
template <bool TO>
__global__ __launch_bounds__(256) void k_perm_vec(int64_t N, const int32_t* __restrict__ perm,
                                                  const double* __restrict__ in0, double* __restrict__ out0,
                                                  const double* __restrict__ in1, double* __restrict__ out1) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    const int64_t j = perm[q];
    const bool ok = j >= 0 && j < N;
    if (TO) {
        out0[q] = ok ? in0[j] : kNaN;
        if (in1) out1[q] = ok ? in1[j] : 0.0;
    } else if (ok) {
        out0[j] = in0[q];
    }
}

struct SolveLayout {
    size_t st, part, part_s, part_x, vec[9], poff, pidx, pvals, pb, px, bsum, total;
};

SolveLayout solve_layout(int64_t N, int64_t nnz, bool bj) {
    SolveLayout L;
    size_t o = 0;
    L.st = o;
    o += rbf_align(sizeof(SolveState));
    L.part = o;
    o += rbf_align((size_t)NBMAX * 2 * sizeof(double));
    L.part_s = o;
    o += rbf_align((size_t)NBVEC * sizeof(double));
    L.part_x = o;
    o += rbf_align((size_t)NBVEC * 2 * sizeof(double));
    for (size_t& v : L.vec) {
        v = o;
        o += rbf_align((size_t)N * sizeof(double));
    }
    L.poff = L.pidx = L.pvals = L.pb = L.px = L.bsum = 0;
    if (bj) {
        L.poff = o;
        o += rbf_align((size_t)(N + 1) * sizeof(int64_t));
        L.pidx = o;
        o += rbf_align((size_t)(nnz + N) * sizeof(int32_t));
        L.pvals = o;
        o += rbf_align((size_t)(nnz + N) * sizeof(double));
        L.pb = o;
        o += rbf_align((size_t)N * sizeof(double));
        L.px = o;
        o += rbf_align((size_t)N * sizeof(double));
        L.bsum = o;
        o += rbf_align((size_t)((N + SCAN_B - 1) / SCAN_B) * sizeof(int64_t));
    }
    L.total = o;
    return L;
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
    _Float16* binv = (_Float16*)(w + L.binv);
    float* bscale = (float*)(w + L.bscale);
    RBF_HIP_CHECK(rbf::cell_order_enqueue(s, X, N, d, d == 3 ? BJ_PER_CELL_3D : BJ_PER_CELL_2D, w + L.scratch, perm));
    hipLaunchKernelGGL(k_bj_inverse_perm, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, perm, N, inv);
    hipLaunchKernelGGL(k_bj_setup, dim3((unsigned)((L.nblocks + 3) / 4)), dim3(256), 0, s, N, offsets, idx, vals, nnz,
                       perm, inv, binv, bscale);
    RBF_LAUNCH_CHECK();
    return RBF_OK;
}

extern "C" rbf_status rbf_bicgstab_workspace(int64_t N, int64_t nnz, int precond, size_t* bytes) {
    if (!bytes || N < 1 || nnz < 0) return RBF_EINVAL;
    if (precond != RBF_PRECOND_NONE && precond != RBF_PRECOND_JACOBI && precond != RBF_PRECOND_BLOCK_JACOBI)
        return RBF_EINVAL;
    *bytes = solve_layout(N, nnz, precond == RBF_PRECOND_BLOCK_JACOBI).total;
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
    const bool bj = precond == RBF_PRECOND_BLOCK_JACOBI;
    const SolveLayout WL = solve_layout(N, nnz, bj);
    if (ws_bytes < WL.total) return RBF_EWORKSPACE;
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
    a.st = (SolveState*)(w + WL.st);
    a.part = (double*)(w + WL.part);
    a.part_s = (double*)(w + WL.part_s);
    a.part_x = (double*)(w + WL.part_x);
    double** vecs[9] = {&a.dinv, &a.r, &a.rh, &a.p, &a.v, &a.s, &a.t, &a.ph, &a.sh};
    for (int k = 0; k < 9; ++k) *vecs[k] = (double*)(w + WL.vec[k]);
    const int32_t* perm = nullptr;
    if (bj) {
        const BjLayout L = bj_layout(N, 2);  // perm and inverses sit at the same offsets for d = 2 and 3
        perm = (const int32_t*)((const char*)pc + L.perm);
        const int32_t* inv = (const int32_t*)((const char*)pc + L.inv);
        a.binv = (const _Float16*)((const char*)pc + L.binv);
        a.bscale = (const float*)((const char*)pc + L.bscale);
        // the system in block order
        int64_t* poff = (int64_t*)(w + WL.poff);
        int32_t* pidx = (int32_t*)(w + WL.pidx);
        double* pvals = (double*)(w + WL.pvals);
        int64_t* bsum = (int64_t*)(w + WL.bsum);
        const int64_t nsb = (N + SCAN_B - 1) / SCAN_B;
        const unsigned gN = (unsigned)((N + 255) / 256);
        hipLaunchKernelGGL(k_perm_len, dim3(gN), dim3(256), 0, s, N, offsets, nnz, perm, poff);
        hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nsb), dim3(256), 0, s, poff + 1, N, bsum);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, s, bsum, nsb);
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nsb), dim3(256), 0, s, poff + 1, N, bsum);
        hipLaunchKernelGGL(k_perm_rows, dim3((unsigned)((N * 8 + 255) / 256)), dim3(256), 0, s, N, offsets, idx, vals,
                           nnz, perm, inv, poff, pidx, pvals, nnz + N);
        double* pb = (double*)(w + WL.pb);
        double* px = (double*)(w + WL.px);
        hipLaunchKernelGGL((k_perm_vec<true>), dim3(gN), dim3(256), 0, s, N, perm, rhs, pb, (const double*)x, px);
        RBF_LAUNCH_CHECK();
        a.offsets = poff;
        a.idx = pidx;
        a.vals = pvals;
        a.nnz = nnz + N;
        a.b = pb;
        a.x = px;
    } else {
        a.binv = nullptr;
        a.bscale = nullptr;
    }
    a.xp = bj ? a.ph : a.p;
    a.xs = bj ? a.sh : a.s;

    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, a.st, max_iter, tol);
    RBF_LAUNCH_CHECK();
    if (dispatch_row_shape<DiagL>(n_max, N, s, a, precond == RBF_PRECOND_JACOBI ? 1 : 0) != hipSuccess)
        return RBF_EHIP;
    if (solver_launch(n_max, s, a, 0) != hipSuccess) return RBF_EHIP;

    // iterations 1, 2, ... (counted from the latest start) in chunks; after each
    // chunk the checks that the next iteration's head would make (no iteration
    // past max_iter in all is launched).  A converged x is checked against its
    // recomputed residual and, if that is above twice the tolerance, restarted from.
    SolveState hs;
    int enqueued = 0, restarts = 0;
    for (;;) {
        RBF_HIP_CHECK(hipMemcpyAsync(&hs, a.st, sizeof(hs), hipMemcpyDeviceToHost, s));
        RBF_HIP_CHECK(hipStreamSynchronize(s));
        const int left = max_iter - hs.iter_base - enqueued;
        if (hs.status == RUNNING && left > 0) {
            const int chunk = left < CHECK_EVERY ? left : CHECK_EVERY;
            for (int k = 0; k < chunk; ++k)
                if (solver_launch(n_max, s, a, 1, enqueued + k + 1) != hipSuccess) return RBF_EHIP;
            enqueued += chunk;
            if (solver_launch(n_max, s, a, 2, enqueued + 1) != hipSuccess) return RBF_EHIP;
            continue;
        }
        if (hs.status == RBF_SOLVE_CONVERGED && !hs.verified && restarts < MAX_RESTARTS) {
            if (solver_launch(n_max, s, a, 4) != hipSuccess) return RBF_EHIP;
            ++restarts;
            enqueued = 0;
            continue;
        }
        break;
    }
    if (solver_launch(n_max, s, a, 3) != hipSuccess) return RBF_EHIP;
    if (bj)
        hipLaunchKernelGGL((k_perm_vec<false>), dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, perm,
                           (const double*)a.x, x, (const double*)nullptr, (double*)nullptr);
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
