/*
 * rbffd.h -- C ABI of the MI355X (gfx950) RBF-FD stencil library.
 *
 * The library computes the data-parallel hot path of strong-form mesh-free
 * discretisation (Slak & Kosec, "Medusa", Sec. 2.1, 2.2.2, 2.3.2):
 *   1. stencil selection: for each node the n_i closest nodes, itself first;
 *   2. RBF-FD weights: for each stencil the augmented polyharmonic-spline plus
 *      monomial system of eq. (rbf-system-aug), solved for the Laplacian and
 *      first-derivative weights (or the GWLS weights of Sec. 2.2.1);
 *   3. the sparse operator in CSR form (at most sum n_i nonzeros);
 *   4. explicit evaluation of the operators on a field and the explicit Euler
 *      time step built from it (Sec. 2.3.1);
 *   5. the implicit system M u = r of a boundary value problem and its
 *      iterative solution on the GPU (Sec. 2.3.2, Sec. 5).
 *
 * Conventions shared by every call
 *   - All array arguments are DEVICE pointers unless stated otherwise.  The
 *     caller allocates and owns every buffer, including the workspace; the
 *     library never allocates on these calls.
 *   - Indices are 0-based.  Node coordinates X are row-major [N][d] float64.
 *   - offsets[N+1] (int64) is the exclusive prefix sum of the stencil sizes n_i;
 *     nnz = offsets[N].  Stencil i occupies idx[offsets[i] .. offsets[i+1]).
 *   - Weight arrays are operator-major: w[r * nnz + offsets[i] + j] is the
 *     weight of stencil node j of node i for the r-th operator selected in
 *     op_mask, operators ordered LAP, DX, DY, DZ, DXX, DXY, DXZ, DYY, DYZ, DZZ.
 *     One weights call computes at most four operators (one local solve
 *     serves them all); operators along z need d = 3.
 *   - Every call is asynchronous on the context's HIP stream.  Argument errors
 *     are detected on the host before any launch and returned as negative
 *     codes; numerical trouble is never a call failure but a per-stencil status.
 *   - Calls on one context must not overlap from several host threads.
 */
#ifndef RBFFD_H
#define RBFFD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rbf_status;

/* call return codes */
#define RBF_OK            0
#define RBF_EINVAL       -1  /* null pointer or inconsistent argument            */
#define RBF_ETOOFEW      -2  /* stencil size bound larger than the node count    */
#define RBF_EDIM         -3  /* dimension not 2 or 3                             */
#define RBF_EWORKSPACE   -4  /* workspace smaller than the *_workspace size      */
#define RBF_EHIP         -5  /* HIP runtime error (launch or device)             */
#define RBF_EUNSUPPORTED -6  /* n_max + m beyond the compiled system sizes       */

/* operator selection (op_mask bits); the second derivatives d2/dx_a dx_b are the
 * building blocks of the general second-order operator of eq. (gen-op), Sec. 3.3 */
#define RBF_OP_LAP 1u
#define RBF_OP_DX  2u
#define RBF_OP_DY  4u
#define RBF_OP_DZ  8u
#define RBF_OP_DXX 16u
#define RBF_OP_DXY 32u
#define RBF_OP_DXZ 64u
#define RBF_OP_DYY 128u
#define RBF_OP_DYZ 256u
#define RBF_OP_DZZ 512u

/* per-stencil status values (int8) */
#define RBF_ST_OK                   0  /* FP64 solve, reproduction check passed      */
#define RBF_ST_REFINED              1  /* FP32 LU + FP64 refinement accepted         */
#define RBF_ST_FALLBACK             2  /* refinement rejected, FP64 solve used       */
#define RBF_ST_SURROGATE            3  /* learned weights accepted after projection  */
#define RBF_ST_SURROGATE_REJECTED   4  /* learned weights rejected, FP64 solve used  */
#define RBF_ST_SINGULAR            -1  /* FP64 solve failed its checks: weights NaN  */
#define RBF_ST_BADSIZE             -2  /* n_i outside [1, n_max]: weights NaN        */

/* precision of the local solves */
#define RBF_PREC_F64     0  /* LU with partial pivoting in float64                   */
#define RBF_PREC_F32_IR  1  /* float32 LU + float64-residual iterative refinement   */

typedef struct rbf_ctx rbf_ctx;

typedef struct rbf_options {
    int    precision;    /* RBF_PREC_F64 or RBF_PREC_F32_IR                           */
    int    max_refine;   /* refinement corrections for F32_IR (default 10); 0 sends   */
                         /* every stencil to the FP64 solve                           */
    int    phs_power;    /* odd exponent k of phi(r) = r^k; 3 (default) or 5          */
    int    scale_mode;   /* 0: s = max_j |p_j - p*| (default); 1: closest node        */
    double repro_tol;    /* FP64 reproduction-check tolerance (default 1e-8)          */
    double refine_tol;   /* F32_IR acceptance: max|r| <= tol ||K|| max|x| per RHS with */
                         /* tol = max(sqrt(n+m) 2^-53, refine_tol); 0 (default) is    */
                         /* LAPACK dsgesv's test                                      */
    double surrogate_tol;/* surrogate acceptance: reproduction residual <= tol        */
                         /* (default 1e-6)                                            */
    double surrogate_corr_tol; /* surrogate acceptance: the projection's correction   */
                         /* max|w - y| <= tol max|w| (default 0.25)                   */
} rbf_options;

/* Default options (precision F64, 10 corrections, r^3, stencil-radius scale,
 * reproduction tolerance 1e-8, surrogate tolerances 1e-6 and 0.25). */
rbf_status rbf_options_default(rbf_options* opt);

/* Human-readable text of a return code (static storage). */
const char* rbf_status_string(rbf_status s);

/* Context: device ordinal and the HIP stream (hipStream_t, may be NULL for the
 * default stream) every call is enqueued on.  The context owns no device memory
 * except the autotuner's plan and the surrogate network parameters. */
rbf_status rbf_ctx_create(rbf_ctx** ctx, int device, void* hip_stream);
rbf_status rbf_ctx_set_stream(rbf_ctx* ctx, void* hip_stream);
rbf_status rbf_ctx_destroy(rbf_ctx* ctx);

/* ------------------------------------------------------------------------ *
 * Stencil selection (Sec. 2.1, "closest nodes"; FindClosest of Sec. 3.1).
 *
 * For node i, idx[offsets[i]] = i and the next n_i - 1 entries are the nodes
 * j != i with the smallest key ((dx*dx + dy*dy) + dz*dz) in float64 with
 * dx = x_j - x_i (each operation correctly rounded, no fused multiply-add),
 * in ascending (key, j) order.  The result is exact (not approximate):
 * identical to a brute-force search.
 *
 * n_max bounds every n_i (1 <= n_max <= min(N, 129)); a node with n_i outside
 * [1, n_max] gets idx entries -1.  Workspace: rbf_select_stencils_workspace.
 * ------------------------------------------------------------------------ */
rbf_status rbf_select_stencils_workspace(int64_t N, int d, int n_max, size_t* bytes);
rbf_status rbf_select_stencils(rbf_ctx* ctx, const double* X, int64_t N, int d,
                               const int64_t* offsets, int n_max, int32_t* idx,
                               void* workspace, size_t ws_bytes);

/* ------------------------------------------------------------------------ *
 * Stencil selection that allocates nothing and takes no workspace.
 *
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result, kernels and stream semantics as rbf_select_stencils, with the
 * selection buffers (grid, cell counts, node ids and coordinates in cell order)
 * in a fixed array inside the library, RBF_SELECT_STATIC_BYTES per device,
 * held from the library's load until the process ends.  Sizes whose
 * rbf_select_stencils_workspace exceeds that return RBF_EWORKSPACE (about
 * 1.5M nodes in 3D, 1.8M in 2D); nothing is launched then.  The array is
 * resolved on each device by rbf_ctx_create.  Every call on one device uses
 * the same array: calls that overlap on one device (several streams or
 * contexts, several host threads) race and must be serialised by the caller.
 * The call never calls hipMalloc/hipFree; it clears what must start at zero.
 * ------------------------------------------------------------------------ */
#define RBF_SELECT_STATIC_BYTES (64u * 1024u * 1024u)
rbf_status rbf_select_stencils_static(rbf_ctx* ctx, const double* X, int64_t N, int d,
                                      const int64_t* offsets, int n_max, int32_t* idx);

/* ------------------------------------------------------------------------ *
 * RBF-FD weights, eq. (rbf-system-aug) of Sec. 2.2.2.
 *
 * For each stencil: offsets to the centre p* = X[idx[offsets[i]]], scaled by s
 * (opt->scale_mode); phi(r) = r^k (opt->phs_power); monomials of total degree
 * <= degree (m = C(degree + d, d) of them); right-hand sides of the selected
 * operators at p*; the system is solved (LU with partial pivoting, or FP32 LU
 * with FP64 refinement and FP64 fallback), the Lagrange multipliers are
 * discarded and the weights scaled back by s^-2 (LAP) or s^-1 (DX, DY, DZ).
 * Second derivatives d2/dx_a dx_b (RBF_OP_DXX ..) use
 * (d_ab phi_j)(0) = k r^(k-2) delta_ab + k (k-2) r^(k-4) x_a x_b and are scaled
 * back by s^-2.  Each stencil's weights pass an FP64 polynomial-reproduction
 * check (second block row of the system) before they are accepted.
 *
 * Augmentation degree (Sec. 3.2 takes it as a parameter of the approximation;
 * Sec. 3.1 allows stencils of varying size): degree[N] (int8, device) gives
 * each node its own degree, and degree_max (0..4) bounds them -- a node whose
 * degree lies outside [0, degree_max] gets RBF_ST_BADSIZE; with degree == NULL
 * every node takes degree_max.  n_max bounds every n_i; the system size
 * n_max + C(degree_max + d, d) must be <= 128, and selects the compiled size
 * class every stencil of the call runs in.  F32_IR runs the float32
 * elimination with one row per lane up to 64 unknowns and two rows per lane
 * (one wavefront per stencil) up to 108; the 128 class is solved in float64
 * (four wavefronts per stencil) also when F32_IR is asked for, and then reports
 * RBF_ST_FALLBACK.  status[N] (int8, may be NULL for F64) receives
 * RBF_ST_*.  w: [popcount(op_mask)][nnz] float64, popcount(op_mask) <= 4.
 * No workspace is needed.
 * ------------------------------------------------------------------------ */
rbf_status rbf_compute_weights(rbf_ctx* ctx, const double* X, int64_t N, int d,
                               const int64_t* offsets, const int32_t* idx, int64_t nnz,
                               int n_max, const int8_t* degree, int degree_max, unsigned op_mask,
                               const rbf_options* opt, double* w, int8_t* status);

/* weight functions of the GWLS engine */
#define RBF_WLS_UNIT      0   /* omega = 1: plain least squares                        */
#define RBF_WLS_GAUSSIAN  1   /* omega(x) = exp(-|x|^2 / sigma^2) on the scaled offsets */

/* ------------------------------------------------------------------------ *
 * GWLS weights, Sec. 2.2.1 (the paper's second approximation engine).
 *
 * Basis: the monomials of total degree <= degree (m = C(degree + d, d)) at the
 * scaled offsets x_j = (p_j - p*) / s (s from opt->scale_mode, as for
 * rbf_compute_weights); W = diag(omega(x_j)).  The weights of each operator are
 * w = W y with y the minimum-norm solution of (W B)^T y = (L b)(0), eq. (wbsys),
 * i.e. w^T = (L b)(0)^T (W B)^+ W, scaled back by s^-2 (LAP) or s^-1.  Solved by
 * Householder QR of W B in float64, one stencil per wavefront.  A stencil whose
 * W B is rank deficient (n_i < m included) gets RBF_ST_SINGULAR and NaN
 * weights; accepted weights pass the FP64 reproduction check (opt->repro_tol).
 * n_max <= 64, degree 0..4; weight_fn RBF_WLS_*, sigma > 0 for the Gaussian;
 * opt may be NULL (defaults; its precision and phs_power are not used).
 * status[N] may be NULL.  w: [popcount(op_mask)][nnz].  No workspace.
 * ------------------------------------------------------------------------ */
rbf_status rbf_compute_weights_wls(rbf_ctx* ctx, const double* X, int64_t N, int d,
                                   const int64_t* offsets, const int32_t* idx, int64_t nnz,
                                   int n_max, int degree, unsigned op_mask, int weight_fn,
                                   double sigma, const rbf_options* opt, double* w, int8_t* status);

/* ------------------------------------------------------------------------ *
 * CSR operator (Sec. 2.3.2, internal-node rows of eqs. implicit-start..end).
 *
 * row_ptr[N+1] (int64) = offsets; the columns of each row are the stencil
 * indices in ascending order (equal columns keep their stencil order); vals[r][nnz]
 * holds the weights of operator r permuted the same way.  n_max bounds every n_i
 * (<= 256).  A row whose size lies outside [0, n_max], or that holds a column
 * outside [0, N), gets col = -1 and NaN values over its range; a row whose
 * range lies outside [0, nnz] is left unwritten.  w and vals may not alias.
 * No workspace is needed.
 * ------------------------------------------------------------------------ */
rbf_status rbf_assemble_csr(rbf_ctx* ctx, int64_t N, const int64_t* offsets,
                            const int32_t* idx, const double* w, int n_ops, int64_t nnz,
                            int n_max, int64_t* row_ptr, int32_t* col, double* vals);

/* ------------------------------------------------------------------------ *
 * Batched persistent form: the weights of several node sets at once, mixing
 * dimension (2D/3D), augmentation degree (0..4, per node) and stencil size.
 * The stencils of all domains are sorted into RBF_BATCHED_CLASSES size classes
 * (n_i + m <= 24, 32, 48, 64, 80, 100, 108, 128); each class runs one
 * persistent launch over all domains.  Classes up to 64 unknowns solve one
 * stencil per wavefront (one row per lane); above 64, the float64 form runs one
 * stencil per four-wave workgroup and the FP32+refinement form one stencil per
 * wavefront (two float rows per lane, classes up to 108; the 128 class is
 * solved in float64 and reported FALLBACK); the refined form adds one float64
 * launch per class for its fallbacks.  Each domain is described as for
 * rbf_compute_weights; a stencil with n_i + m > 128 gets BADSIZE.  Results,
 * status codes and layouts are those of rbf_compute_weights.
 * Workspace: rbf_batched_workspace.  The plan of each class (chunk of stencils
 * per grab, waves per compute unit) is the context's, set by
 * rbf_autotune_batched or rbf_set_plan (default chunk 4, 8 waves per CU).
 * Plans change the scheduling only, never the results.  At most 16 domains.
 * ------------------------------------------------------------------------ */
#define RBF_BATCHED_CLASSES 8

typedef struct rbf_domain_desc {
    const double*  X;              /* [N][d] node coordinates                        */
    int64_t        N;
    int            d;              /* 2 or 3                                         */
    const int64_t* offsets;        /* [N+1]                                          */
    const int32_t* idx;            /* [nnz] stencils, centre first                   */
    int64_t        nnz;
    const int8_t*  degree;         /* [N] per-node augmentation degree, or NULL      */
    int            degree_uniform; /* degree of every node when degree == NULL       */
    int            n_max;          /* bound on every n_i                             */
    unsigned       op_mask;        /* RBF_OP_* of this domain                        */
    double*        w;              /* [popcount(op_mask)][nnz] output                */
    int8_t*        status;         /* [N] output (required)                          */
} rbf_domain_desc;

typedef struct rbf_plan {
    int   chunk;         /* stencils taken per atomic grab of the work list   */
    int   waves_per_cu;  /* persistent grid size = compute units x this       */
    float ms;            /* the class's time when the plan was tuned (0 if set) */
} rbf_plan;

/* largest system size n + m of batched class cls (0 .. RBF_BATCHED_CLASSES-1) */
rbf_status rbf_batched_class_size(int cls, int* maxm);

rbf_status rbf_batched_workspace(const rbf_domain_desc* doms, int n_doms, size_t* bytes);
rbf_status rbf_compute_weights_batched(rbf_ctx* ctx, const rbf_domain_desc* doms, int n_doms,
                                       const rbf_options* opt, void* workspace, size_t ws_bytes);

/* Autotuner of the batched form: runs this batch once per candidate plan
 * (chunk in {1,2,4,8,16} x waves per CU in {4,8,12,16}), times every class's
 * launches separately with HIP events, and keeps for EACH class the fastest
 * candidate; the plans go to the context and to best[RBF_BATCHED_CLASSES]
 * (host, may be NULL).  Synchronous.  cache_path (host string, may be NULL): a
 * text file of "signature chunk_0 waves_0 ... chunk_7 waves_7 ms" lines; the
 * signature holds the device, the solver options (precision, PHS power,
 * refinement limit and tolerance, scale mode, reproduction tolerance) and each
 * domain's shape (d, N, nnz, degree, n_max, op_mask).  A stored line for the
 * same signature is reused without timing; a tuned one is appended. */
rbf_status rbf_autotune_batched(rbf_ctx* ctx, const rbf_domain_desc* doms, int n_doms,
                                const rbf_options* opt, void* workspace, size_t ws_bytes,
                                const char* cache_path, rbf_plan* best);
/* plans[RBF_BATCHED_CLASSES] (host); NULL returns every class to the default */
rbf_status rbf_set_plan(rbf_ctx* ctx, const rbf_plan* plans);
rbf_status rbf_get_plan(const rbf_ctx* ctx, rbf_plan* plans);

/* ------------------------------------------------------------------------ *
 * Explicit evaluation (Sec. 2.3.1): an operator applied to a known field is
 * the stencil dot product w_{L,p_i}^T u_{I(i)} at every node.
 *
 * out[r * N + i] = sum_{p = offsets[i]}^{offsets[i+1]-1} w[r * nnz + p] * u[idx[p]]
 * for r < n_ops (1..4), float64.  u[n_u]; out[n_ops][N] may not alias u or w.
 * n_max is the largest n_i and only chooses the lanes per row.  A row whose
 * range lies outside [0, nnz] or holds an index outside [0, n_u) gets NaN; an
 * empty row gets 0.  The summation order is fixed: results are reproducible
 * run to run.  No workspace is needed.
 * ------------------------------------------------------------------------ */
rbf_status rbf_apply_operators(rbf_ctx* ctx, int64_t N, const int64_t* offsets,
                               const int32_t* idx, const double* w, int n_ops, int64_t nnz,
                               int n_max, const double* u, int64_t n_u, double* out);

/* ------------------------------------------------------------------------ *
 * General second-order operator from stored weights, eq. (gen-op), Sec. 3.3:
 * for L = sum_alpha a_alpha(p) d^alpha,
 *   out[p] = sum_{k < n_ops} coef[i * n_ops + k] * w[k * nnz + p]
 * for every position p of row i (w: n_ops stored operator rows, e.g. DX, DY,
 * DXX, DXY, DYY; coef[N][n_ops] the coefficients a_alpha at the nodes).
 * n_ops in 1..10; out[nnz] may not alias w.  n_max only chooses the lanes per
 * row.  Rows whose range lies outside [0, nnz] are left unwritten.
 * ------------------------------------------------------------------------ */
rbf_status rbf_combine_operators(rbf_ctx* ctx, int64_t N, const int64_t* offsets, int64_t nnz,
                                 int n_max, const double* w, int n_ops, const double* coef,
                                 double* out);

/* node kinds of the explicit step (uint8) */
#define RBF_NODE_INTERIOR  0
#define RBF_NODE_DIRICHLET 1
#define RBF_NODE_NEUMANN   2

/* ------------------------------------------------------------------------ *
 * One explicit Euler step of du/dt = L u + s, eqs. (exp-start)-(exp-end):
 *   interior node:  u_new[i] = u[i] + dt * (w_lap_i^T u_{I(i)} + s[i])
 *   Dirichlet node: u_new[i] = g[i]                  (g NULL: u[i])
 *   Neumann node:   with c_j = sum_l normal[i][l] * w_grad[l][offsets[i] + j],
 *                   u_new[i] = (g[i] - sum_{j>=1} c_j u[idx[offsets[i]+j]]) / c_0
 *                   (g NULL: zero flux), the discretised normal derivative of
 *                   eq. (neu) equated to g and solved for u_i.
 * kind[N] uint8 (RBF_NODE_*); w_lap[nnz]; w_grad: d rows of nnz values at
 * w_grad + l * nnz (the DX..DZ rows of an rbf_compute_weights output), needed
 * only when some node is Neumann; normals[N][d] (outward unit normals, read at
 * Neumann nodes only); g[N] holds g_d((k+1) dt) at Dirichlet and g_n((k+1) dt)
 * at Neumann nodes; s[N] the source (NULL: 0).  g and s may be NULL.
 * Stencil position 0 must be node i itself (rbf_select_stencils puts it
 * there).  A node with an invalid kind, row range or index, or a Neumann node
 * whose first entry is not itself, gets NaN.  u_new may not alias u.
 * d is 2 or 3.  No workspace is needed.
 * ------------------------------------------------------------------------ */
rbf_status rbf_explicit_step(rbf_ctx* ctx, int64_t N, int d, const int64_t* offsets,
                             const int32_t* idx, int64_t nnz, int n_max,
                             const double* w_lap, const double* w_grad, const uint8_t* kind,
                             const double* normals, const double* g, const double* s,
                             const double* u, double dt, double* u_new);

/* ------------------------------------------------------------------------ *
 * Implicit system, eqs. (implicit-start)-(implicit-end) of Sec. 2.3.2, for
 * L u = f in the domain, u = g_d on Dirichlet and du/dn = g_n on Neumann nodes:
 *   interior row i:  M[i][idx[p]] = w_lap[p],                     r[i] = f[i]
 *   Dirichlet row i: M[i][i] = 1,                                  r[i] = g[i]
 *   Neumann row i:   M[i][idx[p]] = sum_l normals[i][l] w_grad[l][p], r[i] = g[i]
 * for p in the row's range.  M is written in the stencil layout (the same
 * offsets and idx; vals[nnz] float64): a Dirichlet row keeps its n_i slots,
 * 1 at position 0 (the node itself) and explicit zeros elsewhere.
 * rbf_assemble_csr turns it into CSR with ascending columns.  kind, w_grad,
 * normals as for rbf_explicit_step; f and g may be NULL (zero).  A row with an
 * invalid kind or range, or a Dirichlet / Neumann row whose position 0 is not
 * the node itself, gets NaN in r (and in its vals where the range is valid).
 * No workspace is needed.
 * ------------------------------------------------------------------------ */
rbf_status rbf_assemble_implicit(rbf_ctx* ctx, int64_t N, int d, const int64_t* offsets,
                                 const int32_t* idx, int64_t nnz, const double* w_lap,
                                 const double* w_grad, const uint8_t* kind, const double* normals,
                                 const double* f, const double* g, double* vals, double* rhs);

/* iterative solver preconditioners and outcomes */
#define RBF_PRECOND_NONE          0
#define RBF_PRECOND_JACOBI        1   /* rows scaled by the inverse diagonal              */
#define RBF_PRECOND_BLOCK_JACOBI  2   /* inverses of 64 x 64 diagonal blocks of nodes in  */
                                      /* cell order (rbf_block_jacobi_setup), right side  */

#define RBF_SOLVE_CONVERGED  0
#define RBF_SOLVE_MAXITER    1
#define RBF_SOLVE_BREAKDOWN  2  /* a BiCGStab denominator vanished or a value is not finite */
#define RBF_SOLVE_BADDIAG    3  /* Jacobi: a row without a finite nonzero diagonal entry */
#define RBF_SOLVE_DIVERGED   4  /* the residual grew past 10^6 times the initial one      */

typedef struct rbf_solve_info {
    int32_t status;          /* RBF_SOLVE_*                                               */
    int32_t iterations;      /* BiCGStab iterations taken                                 */
    double  residual;        /* ||D^-1 (r - M x)|| / ||D^-1 r||, the monitored residual   */
    double  true_residual;   /* ||r - M x|| / ||r|| of the returned x, recomputed         */
} rbf_solve_info;

/* ------------------------------------------------------------------------ *
 * Solution of M x = r (Sec. 2.3.2) by BiCGStab (van der Vorst 1992), the
 * Krylov method the paper's benchmark uses (Sec. 5; there with an incomplete-LU
 * preconditioner on the CPU), in float64 on the GPU.
 *
 * M: N rows in the stencil layout or CSR (row_ptr = offsets, col = idx, vals
 * [nnz]); n_max bounds the row lengths.  x[N]: initial guess in, solution out.
 * Preconditioner: RBF_PRECOND_JACOBI solves D^-1 M x = D^-1 r with D the
 * diagonal of M (the first entry of row i in column i), RBF_PRECOND_NONE with
 * D = I; both stop when ||D^-1 (r - M x)|| <= tol ||D^-1 r||.
 * RBF_PRECOND_BLOCK_JACOBI solves M P^-1 y = r, x = P^-1 y, with P the block
 * diagonal of M over the node blocks of rbf_block_jacobi_setup (pc, built from
 * the same M), and stops when ||r - M x|| <= tol ||r||; it copies M, r and x
 * into the node order of pc inside the workspace (x is copied back on return),
 * so its iterations read every vector contiguously.  pc/pc_bytes are ignored by
 * the other preconditioners (may be NULL).  The monitored residual is updated
 * by the recursion; once it meets tol, the residual is recomputed from x in the
 * same norm and, if that exceeds 2 tol, the iteration restarts from x (at
 * most 3 times; iterations counts all of them; after the last restart the
 * monitored residual decides).  Any form also stops
 * after max_iter iterations, or with RBF_SOLVE_DIVERGED once the monitored
 * residual exceeds 10^6 times its initial value.  Every step runs on the
 * device (no host round trip inside an iteration); the call waits for the
 * context stream every 16 iterations and on return, when *info (host memory,
 * may be NULL) is filled.  Deterministic: every dot product is reduced in a
 * fixed order.  Workspace: rbf_bicgstab_workspace for the same N, nnz and
 * preconditioner (9 N + 5,120 float64 values and 256 bytes; block-Jacobi adds
 * the copy of M, about 12 (nnz + N) + 24 N bytes).
 * ------------------------------------------------------------------------ */
rbf_status rbf_bicgstab_workspace(int64_t N, int64_t nnz, int precond, size_t* bytes);
rbf_status rbf_bicgstab(rbf_ctx* ctx, int64_t N, const int64_t* offsets, const int32_t* idx,
                        const double* vals, int64_t nnz, int n_max, const double* rhs, double* x,
                        double tol, int max_iter, int precond, const void* pc, size_t pc_bytes,
                        void* workspace, size_t ws_bytes, rbf_solve_info* info);

/* ------------------------------------------------------------------------ *
 * Block-Jacobi preconditioner of rbf_bicgstab (a parallel replacement for the
 * incomplete LU the paper's benchmark uses, Sec. 5).  The nodes X[N][d] are
 * ordered by a uniform grid of cells (about 8 nodes per cell in 2D, 16 in 3D;
 * ascending ids inside a cell) and cut into blocks of 64 consecutive nodes;
 * for every block the 64 x 64 submatrix of M (rows and columns of its nodes;
 * entries of other columns dropped, repeated columns added) is inverted in
 * float32 (Gauss-Jordan, partial pivoting); a block with a zero pivot keeps
 * the inverse of its diagonal.  pc (device, caller-owned, at least
 * rbf_block_jacobi_size bytes) receives the node order and the inverses, each
 * row stored as float16 divided by its largest magnitude with that scale in
 * float32 (about 140 B per node).  M as for rbf_bicgstab.
 * ------------------------------------------------------------------------ */
rbf_status rbf_block_jacobi_size(int64_t N, int d, size_t* bytes);
rbf_status rbf_block_jacobi_setup(rbf_ctx* ctx, const double* X, int64_t N, int d,
                                  const int64_t* offsets, const int32_t* idx, const double* vals,
                                  int64_t nnz, void* pc, size_t pc_bytes);

/* ------------------------------------------------------------------------ *
 * Learned surrogate of the 2D, 15-node Laplacian weights (degree-2
 * augmentation, m = 6).  Not part of the paper's method: a network replaces
 * the local solve of eq. (rbf-system-aug) and its output is projected onto the
 * second block row of that system (polynomial reproduction), which the plain
 * weights satisfy exactly.
 *
 * Network: 30 -> 128 -> 128 -> 128 -> 15, erf-GELU after the hidden layers
 * (erf by Abramowitz & Stegun 7.1.26, |error| <= 1.5e-7).  Input: the scaled offsets (x_j - x_i)/s, s = max_j |x_j - x_i|,
 * in stencil order (x, y interleaved, the centre's zeros included), in the
 * canonical frame of the stencil: rotated so that node 1 lies on +x, then
 * y reflected so that node 2 has y >= 0 (float64, c = o_1x/|o_1|,
 * s_ = o_1y/|o_1|, f = sign(c o_2y - s_ o_2x) (+1 at 0), x' = (c o_x + s_ o_y)/s,
 * y' = f (c o_y - s_ o_x)/s, each operation rounded, no fused multiply-add,
 * then rounded to float32).  Output: the scaled weights w_j s^2.  Parameters: one float32 array of
 * RBF_MLP_NPARAM values, row-major W1[128][30], b1[128], W2[128][128], b2,
 * W3[128][128], b3, W4[15][128], b4[15].  Products use bfloat16 operands and
 * float32 accumulation; x, W and the hidden activations (forward) and the
 * output and pre-activation gradients (backward) are rounded to bfloat16,
 * round-to-nearest-even.  The "packed" array (RBF_MLP_PACKED_BYTES, caller
 * owned, 16-byte aligned) holds the bfloat16 weights in the operand order of
 * the kernels; it is derived from the parameters by rbf_mlp_pack and must be
 * refreshed after every parameter change (rbf_mlp_adam does it).
 * ------------------------------------------------------------------------ */
#define RBF_MLP_NPARAM       38927
#define RBF_MLP_PACKED_BYTES (148 * 1024)

rbf_status rbf_mlp_pack(rbf_ctx* ctx, const float* params, void* packed);

/* y[B][15] = network(x[B][30]) (float32 row-major). */
rbf_status rbf_mlp_forward(rbf_ctx* ctx, const float* params, const void* packed,
                           const float* x, int64_t B, float* y);

/* Mean-squared-error loss over the batch, sum_{b,o} (y_bo - t_bo)^2 / (15 B),
 * and its gradient with respect to every parameter (grads[RBF_MLP_NPARAM]).
 * x[n_rows][30], t[n_rows][15]; the batch rows are sel[0..B) (sel may be NULL:
 * rows 0..B-1, then B <= n_rows); a sel entry outside [0, n_rows) contributes
 * nothing.  loss (device float, may be NULL).  Deterministic: per-block partial
 * sums reduced in a fixed order.  Workspace: rbf_mlp_grad_workspace. */
rbf_status rbf_mlp_grad_workspace(int64_t B, size_t* bytes);
rbf_status rbf_mlp_grad(rbf_ctx* ctx, const float* params, const void* packed,
                        const float* x, const float* t, int64_t n_rows, const int64_t* sel, int64_t B,
                        float* grads, float* loss, void* workspace, size_t ws_bytes);

/* One Adam step (step = 1, 2, ...; bias-corrected moments m, v, float32) on
 * params in place; packed (may be NULL) is refreshed from the new values. */
rbf_status rbf_mlp_adam(rbf_ctx* ctx, float* params, const float* grads, float* m, float* v,
                        int step, float lr, float beta1, float beta2, float eps, void* packed);

/* Training pairs from 2D 15-node stencils: feat[N][30] (float32 scaled
 * offsets), target[N][15] = w_lap * s^2 (may be NULL; w_lap the plain
 * Laplacian weights [nnz] from rbf_compute_weights, or NULL), scale[N] = s
 * (may be NULL).  Stencils of another size or with invalid indices get NaN rows. */
rbf_status rbf_surrogate_dataset(rbf_ctx* ctx, const double* X, int64_t N,
                                 const int64_t* offsets, const int32_t* idx, int64_t nnz,
                                 const double* w_lap, float* feat, float* target, double* scale);

/* Copy parameters (device float32 [RBF_MLP_NPARAM]) into the context and pack
 * them; the context allocates its copy on the first call. */
rbf_status rbf_surrogate_load(rbf_ctx* ctx, const float* params);

/* Laplacian weights of 2D stencils through the loaded network: features,
 * network, float64 projection w = y + Q (Q^T Q)^{-1} (l_q - Q^T y) onto the
 * reproduction conditions, and the residual
 * rho = max_l |(Q^T w - l_q)_l| / max(1, max |l_q|).  A stencil is accepted
 * (status RBF_ST_SURROGATE) when rho <= opt->surrogate_tol (a consistency check
 * of the float64 projection, which the network cannot fail) AND the correction
 * the projection made is small against the result, max_j |w_j - y_j| <=
 * opt->surrogate_corr_tol max_j |w_j| (what the network controls: the zero
 * network needs a correction of the whole weights, ratio 1); otherwise (and for
 * stencils that are not
 * 15-node) the plain float64 solve runs and the status is
 * RBF_ST_SURROGATE_REJECTED (or RBF_ST_SINGULAR / RBF_ST_BADSIZE from that
 * solve).  w[nnz] float64, status[N] required.  n_max bounds every n_i. */
rbf_status rbf_surrogate_weights(rbf_ctx* ctx, const double* X, int64_t N, int d,
                                 const int64_t* offsets, const int32_t* idx, int64_t nnz,
                                 int n_max, const rbf_options* opt, double* w, int8_t* status);

#ifdef __cplusplus
}
#endif
#endif /* RBFFD_H */
