// RBF-FD weights of one stencil per wavefront (gfx950): assembly of the
// augmented system of eq. (rbf-system-aug), its solution, back-scaling, the
// FP64 polynomial-reproduction check and the store.
//
// Only the register-array size MAXM is a template parameter; dimension (2D is
// run as 3D with z = 0), augmentation degree and stencil size are runtime
// values, so one solver serves every (d, degree) pair.
//
// Unknown / row order inside the kernel: the m polynomial multipliers first,
// then the n stencil weights, i.e. K' = [0 Q^T; Q A] acting on [lambda; w] --
// the paper's K with rows and columns permuted alike (same solution).  Row r of
// K' lives in lane r (one row per lane, MAXM <= 64) and is held in registers;
// padding rows r in [n + m, MAXM) are identity rows.
//
// Solvers:
//   * FP64: Gauss-Jordan with partial pivoting (the paper's LU continued
//     upwards, which costs nothing extra when every lane holds one row and
//     leaves no back substitution).  Per step the pivot search is a DPP max on
//     float magnitudes and the pivot row reaches the other lanes by lane reads
//     into scalar registers.
//   * FP32 + FP64 refinement: float32 Gauss-Jordan that keeps each row's
//     multipliers in its eliminated columns; corrections replay the recorded
//     row operations on the float64 residual (K recomputed in float64 from the
//     scaled offsets kept in LDS).
//   * n + m in (64, 128]: wsolve_quad.hpp (one stencil on four waves).
#pragma once

#include "common.hpp"

namespace rbf {

constexpr int NR = 4;  // right-hand-side slots; each holds one operator (StencilArgs::opc)

// Monomial exponents of total degree <= 4 in graded order (degree ascending,
// then x-power descending, then y-power descending); the first C(P+d, d)
// entries span the polynomials of degree <= P.
struct MonoTable {
    int e2[15][2];
    int e3[35][3];
    constexpr MonoTable() : e2(), e3() {
        int c = 0;
        for (int deg = 0; deg <= 4; ++deg)
            for (int a = deg; a >= 0; --a) {
                e2[c][0] = a;
                e2[c][1] = deg - a;
                ++c;
            }
        c = 0;
        for (int deg = 0; deg <= 4; ++deg)
            for (int a = deg; a >= 0; --a)
                for (int b = deg - a; b >= 0; --b) {
                    e3[c][0] = a;
                    e3[c][1] = b;
                    e3[c][2] = deg - a - b;
                    ++c;
                }
    }
};
__constant__ constexpr MonoTable kMono{};

__device__ __forceinline__ void mono_exp(int d, int l, int& a, int& b, int& c) {
    if (d == 2) {
        a = kMono.e2[l][0];
        b = kMono.e2[l][1];
        c = 0;
    } else {
        a = kMono.e3[l][0];
        b = kMono.e3[l][1];
        c = kMono.e3[l][2];
    }
}

__device__ __forceinline__ double ipow4(double x, int e) {
    const double x2 = x * x;
    return e == 0 ? 1.0 : e == 1 ? x : e == 2 ? x2 : e == 3 ? x2 * x : x2 * x2;
}

// q_l(x) for the graded monomial basis
__device__ __forceinline__ double mono(int d, int l, const double (&x)[3]) {
    int a, b, c;
    mono_exp(d, l, a, b, c);
    return ipow4(x[0], a) * ipow4(x[1], b) * ipow4(x[2], c);
}

// (L q_l)(0): Laplacian (op 0): 2 for q = x_a^2; first derivative d/dx_a (op a+1): 1 for q = x_a
__device__ __forceinline__ double mono_lq(int d, int l, int op) {
    int e[3];
    mono_exp(d, l, e[0], e[1], e[2]);
    const int s = e[0] + e[1] + e[2];
    if (op == 0) return (s == 2 && (e[0] == 2 || e[1] == 2 || e[2] == 2)) ? 2.0 : 0.0;
    return (op - 1 < d && s == 1 && e[op - 1] == 1) ? 1.0 : 0.0;
}

// Operator codes of the right-hand-side slots (one 4-bit code per slot in
// StencilArgs::opc, the bit index of the operator in rbffd.h): 0 Laplacian,
// 1..3 d/dx_a, 4..9 the second derivatives xx, xy, xz, yy, yz, zz.
__host__ __device__ constexpr int op_order(int code) { return (code >= 1 && code <= 3) ? 1 : 2; }
__device__ __forceinline__ int slot_op(unsigned opc, int q) { return (int)((opc >> (4 * q)) & 15u); }
__device__ __forceinline__ void op_axes(int code, int& ax, int& bx) {
    switch (code) {
        case 4: ax = 0; bx = 0; break;
        case 5: ax = 0; bx = 1; break;
        case 6: ax = 0; bx = 2; break;
        case 7: ax = 1; bx = 1; break;
        case 8: ax = 1; bx = 2; break;
        default: ax = 2; bx = 2; break;
    }
}

// (L q_l)(0) for every operator code, dimension and monomial, tabulated at
// compile time (a table lookup keeps the solvers' registers free): Laplacian 2
// for x_a^2; d_a 1 for x_a; d_ab 1 for x_a x_b (a != b), 2 for x_a^2 (a = b).
struct MonoOpTable {
    double v[10][2][35];
    constexpr MonoOpTable() : v() {
        constexpr int A[6] = {0, 0, 0, 1, 1, 2}, B[6] = {0, 1, 2, 1, 2, 2};
        for (int dd = 0; dd < 2; ++dd) {
            int e[35][3] = {};
            int c = 0;
            for (int deg = 0; deg <= 4; ++deg) {
                if (dd == 0) {
                    for (int a = deg; a >= 0; --a) {
                        e[c][0] = a;
                        e[c][1] = deg - a;
                        e[c][2] = 0;
                        ++c;
                    }
                } else {
                    for (int a = deg; a >= 0; --a)
                        for (int b = deg - a; b >= 0; --b) {
                            e[c][0] = a;
                            e[c][1] = b;
                            e[c][2] = deg - a - b;
                            ++c;
                        }
                }
            }
            for (int l = 0; l < c; ++l) {
                const int s = e[l][0] + e[l][1] + e[l][2];
                v[0][dd][l] = (s == 2 && (e[l][0] == 2 || e[l][1] == 2 || e[l][2] == 2)) ? 2.0 : 0.0;
                for (int a = 0; a < 3; ++a) v[1 + a][dd][l] = (a < dd + 2 && s == 1 && e[l][a] == 1) ? 1.0 : 0.0;
                for (int k = 0; k < 6; ++k) {
                    const int ax = A[k], bx = B[k];
                    double t = 0.0;
                    if (s == 2) {
                        if (ax == bx) t = e[l][ax] == 2 ? 2.0 : 0.0;
                        else t = (e[l][ax] == 1 && e[l][bx] == 1) ? 1.0 : 0.0;
                    }
                    v[4 + k][dd][l] = t;
                }
            }
        }
    }
};
__constant__ constexpr MonoOpTable kMonoOp{};

__device__ __forceinline__ double mono_lop(int d, int l, int code) { return kMonoOp.v[code][d - 2][l]; }

// (L phi_j)(0) for phi(r) = r^k about the scaled offset x = x_j, r2 = |x_j|^2,
// pw = |x_j|^(k-2):  Laplacian k (k + d - 2) pw;  d_a: -k pw x_a;
// d_ab: k pw delta_ab + k (k - 2) pw / r2 x_a x_b (the second term is 0 at x_j = 0).
// Written branch-free (alpha pw + beta pw x_a + gamma x_a x_b with per-code
// constants): with branches per code the one-row-per-lane solvers spill.
__device__ __forceinline__ double phs_lop(int code, const double (&x)[3], double r2, double pw, int kpow, int d) {
    const bool lap = code == 0, first = code >= 1 && code <= 3, second = code >= 4;
    const int ia = first ? code - 1 : (code <= 6 ? 0 : (code <= 8 ? 1 : 2));
    const int ib = (code == 4) ? 0 : (code == 5 || code == 7) ? 1 : 2;
    const double xa = ia == 0 ? x[0] : (ia == 1 ? x[1] : x[2]);
    const double xb = ib == 0 ? x[0] : (ib == 1 ? x[1] : x[2]);
    const double alpha = lap ? (double)(kpow * (kpow + d - 2)) : ((second && ia == ib) ? (double)kpow : 0.0);
    const double beta = (first && code <= d) ? -(double)kpow : 0.0;
    const double gamma = (second && r2 > 0.0) ? (double)(kpow * (kpow - 2)) * (pw / r2) : 0.0;
    return alpha * pw + beta * pw * xa + gamma * xa * xb;
}

// fixed coefficients of the test polynomial of the reproduction check
__host__ __device__ constexpr double check_coef(int l) { return 1.0 + 0.6180339887498949 * ((l * 7 + 3) % 11) / 11.0; }

// Square root of a finite x >= 0 (squared scaled offsets): the hardware
// reciprocal square-root estimate, one Goldschmidt iteration on the coupled pair
// g ~ sqrt(x), h ~ 1 / (2 sqrt(x)), and a final Newton correction
// g += (x - g^2) h (Markstein), which leaves g within about an ulp of the rounded
// square root; x = 0 gives 0.  A third of the correctly rounded sequence, whose
// extra work scales denormal and huge arguments; one is evaluated per matrix entry.
__device__ __forceinline__ double sqrt_basis(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    g = fma(fma(-g, g, x), h, g);
    return x > 0.0 ? g : 0.0;
}

// phi(r) = r^k for odd k in {3, 5}, from r^2
__device__ __forceinline__ double phs_from_r2(double r2, int k) {
    const double r = sqrt_basis(r2);
    return (k == 5) ? r2 * r2 * r : r2 * r;
}

struct StencilArgs {
    const double* X;
    int64_t N;
    int d;
    int P;       // uniform augmentation degree, or the bound on the per-node degrees
    const int8_t* degree = nullptr;  // per-node augmentation degree [N], or NULL (every node P)
    const int64_t* offsets;
    const int32_t* idx;
    int64_t nnz;
    int n_max;
    unsigned op_mask;   // active right-hand-side slots (bits 0..NR-1)
    unsigned opc = 0x3210u;  // operator code of each slot (4 bits per slot), see slot_op
    int phs_power;
    int scale_mode;
    double repro_tol;
    double* w;
    int8_t* status;
};

// Augmentation degree of a node: the per-node value when one is given (a value
// outside [0, P] gives -1, which the prologue rejects as BADSIZE), else P.
__device__ __forceinline__ int node_degree(const StencilArgs& a, int64_t node) {
    if (!a.degree) return a.P;
    const int p = a.degree[node];
    return (p >= 0 && p <= a.P) ? p : -1;
}

// NaN weights and a status for a stencil rejected up front
__device__ inline void reject_stencil(const StencilArgs& a, int64_t node, int64_t off, int64_t n, int8_t st) {
    const int R = __builtin_popcount(a.op_mask);
    for (int r = 0; r < R; ++r)
        for (int64_t e = lane_id(); e < n; e += WAVE) a.w[r * a.nnz + off + e] = __builtin_nan("");
    if (a.status && lane_id() == 0) a.status[node] = st;
}

// Scaled offsets x_j = (p_j - p*) / s of the node held by each row slot (row
// m + j holds node j), the scale s and 1/s.  Returns false (wave-uniform) if a
// stencil index is outside [0, N).
template <int RPL>
struct FrameG {
    double xh[RPL][3];
    double s, inv_s;
};

template <int RPL>
__device__ __forceinline__ bool load_frame_g(const StencilArgs& a, int64_t off, int n, int m, FrameG<RPL>& F) {
    const int lane = lane_id();
    const int d = a.d;
    const int c = a.idx[off];
    bool bad = !(c >= 0 && c < a.N);
    double cx[3] = {0, 0, 0};
    if (!bad)
        for (int q = 0; q < d; ++q) cx[q] = a.X[(int64_t)c * d + q];
    double o[RPL][3];
    double r2max = 0.0, r2min = INFINITY;
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
        const int j = lane + 64 * t - m;
        o[t][0] = o[t][1] = o[t][2] = 0.0;
        if (j >= 0 && j < n) {
            const int id = a.idx[off + j];
            if (id >= 0 && id < a.N) {
                for (int q = 0; q < d; ++q) o[t][q] = a.X[(int64_t)id * d + q] - cx[q];
            } else {
                bad = true;
            }
            const double r2 = o[t][0] * o[t][0] + o[t][1] * o[t][1] + o[t][2] * o[t][2];
            r2max = fmax(r2max, r2);
            if (j >= 1) r2min = fmin(r2min, r2);
        }
    }
    const double r2 = (a.scale_mode == 1) ? wave_min_d(r2min) : wave_max_d(r2max);
    F.s = sqrt(r2);
    F.inv_s = 1.0 / F.s;
#pragma unroll
    for (int t = 0; t < RPL; ++t)
        for (int q = 0; q < 3; ++q) F.xh[t][q] = o[t][q] * F.inv_s;
    return ballot64(bad) == 0;
}

// LDS layout (in doubles) of the one-row-per-lane solvers, sized for any m.
template <int MAXM>
struct RowLds {
    static constexpr int QT = (MAXM / 2) * (MAXM - MAXM / 2) + 1;  // max over m of m (MAXM - m)
    static constexpr int QTE = QT + (QT & 1);
    static constexpr int XH = MAXM * 4;                  // scaled offsets, padded to 4 doubles
    static constexpr int SOL = MAXM * NR;                // solution permuted to unknown order
    static constexpr int F32 = (MAXM * NR + 1) / 2;      // FP32 solution (in doubles)
    static constexpr int TOTAL = QTE + XH + SOL + F32;
    static constexpr int o_qt = 0, o_xh = QTE, o_sol = QTE + XH, o_f32 = QTE + XH + SOL;
};

// Assembly of this lane's row of K' (entries computed in float64, stored as T)
// and its FP64 right-hand sides.  Q^T goes to qt[c * (MAXM - m) + j] and the
// scaled offsets to xh[4 j ..] (both stay valid for the refinement residuals).
template <int MAXM, typename T>
__device__ __forceinline__ void assemble_row(const StencilArgs& a, const FrameG<1>& F, int n, int m, double* lds,
                                             T (&row)[MAXM], double (&rhs)[NR]) {
    using L = RowLds<MAXM>;
    double* qt = lds + L::o_qt;
    double* xh = lds + L::o_xh;
    const int d = a.d;
    const int kpow = a.phs_power;
    const int QW = MAXM - m;
    const int r = lane_id();
    const int j = r - m;
    const bool wrow = (j >= 0 && j < n);
    if (wrow) {
        *reinterpret_cast<double2*>(xh + 4 * j) = make_double2(F.xh[0][0], F.xh[0][1]);
        *reinterpret_cast<double2*>(xh + 4 * j + 2) = make_double2(F.xh[0][2], 0.0);
    }
#pragma unroll
    for (int c = 0; c < MAXM; ++c) {
        if (c < m) {  // uniform
            const double q = wrow ? mono(d, c, F.xh[0]) : 0.0;
            row[c] = (T)q;
            if (wrow) qt[c * QW + j] = q;
        }
    }
    wave_lds_sync();
#pragma unroll
    for (int c = 0; c < MAXM; ++c) {
        if (c >= m) {  // uniform
            const int k = c - m;
            const double2 p01 = *reinterpret_cast<const double2*>(xh + 4 * k);
            const double2 p2 = *reinterpret_cast<const double2*>(xh + 4 * k + 2);
            double v;
            if (wrow) {
                const double dx = F.xh[0][0] - p01.x, dy = F.xh[0][1] - p01.y, dz = F.xh[0][2] - p2.x;
                v = (k < n) ? phs_from_r2(dx * dx + dy * dy + dz * dz, kpow) : 0.0;
            } else if (r < m) {
                v = (k < n) ? qt[r * QW + k] : 0.0;
            } else {
                v = (r == c) ? 1.0 : 0.0;  // padding row
            }
            row[c] = (T)v;
        }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) rhs[q] = 0.0;
    if (wrow) {
        const double r2 = F.xh[0][0] * F.xh[0][0] + F.xh[0][1] * F.xh[0][1] + F.xh[0][2] * F.xh[0][2];
        const double rr = sqrt(r2);
        const double pw = (kpow == 5) ? r2 * rr : rr;  // ||x_j||^(k-2)
#pragma unroll
        for (int q = 0; q < NR; ++q) rhs[q] = phs_lop(slot_op(a.opc, q), F.xh[0], r2, pw, kpow, d);
    } else if (r < m) {
#pragma unroll
        for (int q = 0; q < NR; ++q) rhs[q] = mono_lop(d, r, slot_op(a.opc, q));
    }
}

// FP64 reproduction check of the weights held by the weight rows (sol[t][q] is
// the solution of unknown lane + 64 t) and the store of the accepted weights.
template <int RPL>
__device__ __forceinline__ bool repro_check(const StencilArgs& a, int n, int m, const FrameG<RPL>& F,
                                            const double (&sol)[RPL][NR]) {
    const int lane = lane_id();
    const int d = a.d;
    double S[NR], A[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) S[q] = A[q] = 0.0;
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
        const int j = lane + 64 * t - m;
        if (j >= 0 && j < n) {
            double pv = 0.0;
            for (int l = 0; l < m; ++l) pv += check_coef(l) * mono(d, l, F.xh[t]);
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                const double v = sol[t][q] * pv;
                S[q] += v;
                A[q] += fabs(v);
            }
        }
    }
    bool ok = true;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const double s = wave_sum_dpp_d(S[q]);
        const double ab = wave_sum_dpp_d(A[q]);
        if (!(a.op_mask & (1u << q))) continue;
        double lp = 0.0;
        for (int l = 0; l < m; ++l) lp += check_coef(l) * mono_lop(d, l, slot_op(a.opc, q));
        ok = ok && (fabs(s - lp) / (ab + fabs(lp)) <= a.repro_tol);
    }
    return ok;
}

template <int RPL>
__device__ __forceinline__ void store_weights(const StencilArgs& a, int64_t node, int64_t off, int n, int m,
                                              const FrameG<RPL>& F, const double (&sol)[RPL][NR], bool ok,
                                              int8_t good_status) {
    const int lane = lane_id();
    const double sc2 = F.inv_s * F.inv_s;
    int ro = 0;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        if (!(a.op_mask & (1u << q))) continue;
        const double sc = op_order(slot_op(a.opc, q)) == 2 ? sc2 : F.inv_s;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
            const int j = lane + 64 * t - m;
            if (j >= 0 && j < n) a.w[ro * a.nnz + off + j] = ok ? sol[t][q] * sc : __builtin_nan("");
        }
        ++ro;
    }
    if (a.status && lane == 0) a.status[node] = ok ? good_status : (int8_t)RBF_ST_SINGULAR;
}

// 1/x from the hardware reciprocal estimate refined by Newton steps
// (e' = e (2 - x e)); two steps for float64, one for float32.
__device__ __forceinline__ double recip(double x) {
    double e = __builtin_amdgcn_rcp(x);
    e = fma(e, fma(-x, e, 1.0), e);
    e = fma(e, fma(-x, e, 1.0), e);
    return e;
}
__device__ __forceinline__ float recip(float x) {
    const float e = __builtin_amdgcn_rcpf(x);
    return fmaf(e, fmaf(-x, e, 1.0f), e);
}

// Gauss-Jordan with partial pivoting on the rows held in registers (one row per
// lane).  With GUARD, steps and columns past the runtime system size M are
// skipped (uniform branches); without it all MAXM steps run branch-free and
// the padding rows pivot on themselves.  A zero or non-finite pivot is
// recorded and reported at the end.  On return sol[q] holds the solution of
// unknown `lane` (permuted through LDS), mystep the lane's pivot step and invd
// 1/U_kk of that step; with keep_multipliers each row keeps its multipliers in
// the columns it has eliminated (for gj_replay).
//
// The pivot row reaches the other lanes value by value through scalar
// registers (a lane read of the pivot lane, used directly as the FMA operand):
// no LDS store, wait and broadcast read per step.
template <typename T, int MAXM, bool GUARD>
__device__ __forceinline__ bool gauss_jordan(T (&row)[MAXM], T (&rhs)[NR], T* sol_lds, T (&sol)[NR],
                                             bool keep_multipliers, int& step_out, T& invd_out, int M) {
    const int lane = lane_id();
    bool piv = lane >= MAXM;
    int mystep = -1;
    T invd = (T)0;
    int pmin = 0x7F7FFFFF, pmax = 0;  // bit patterns of the smallest / largest pivot magnitude
    // Pivot search on float magnitudes (partial pivoting needs a large pivot, not
    // the exact maximum), compared as bit patterns (a NaN wins and marks the system
    // bad); the first lane with the maximum wins.  The search of step k + 1 runs as
    // soon as column k + 1 is updated, overlapping the rest of step k's update.
    int cand = piv ? -1 : __float_as_int((float)fabs(row[0]));
    int mi = wave_max_dpp_i(cand);
#pragma unroll
    for (int k = 0; k < MAXM; ++k) {
        if (GUARD && k >= M) continue;
        pmin = min(pmin, mi);  // a zero pivot: singular
        pmax = max(pmax, mi);  // an infinite or NaN pivot
        const uint64_t b = ballot64(!piv && cand == mi);
        const int p = first_lane(b);
        const bool me = (lane == p);
        if (me) {
            piv = true;
            mystep = k;
        }
        // values of the pivot lane are read before this step updates them (the
        // pivot lane's own update is by a zero multiplier)
        const T inv = recip(readlane_t<T>(row[k], p));
        if (me) invd = inv;
        const T l = me ? (T)0 : row[k] * inv;
        if (keep_multipliers && !me) row[k] = l;
#pragma unroll
        for (int j = k + 1; j < MAXM; ++j) {
            if (GUARD && j >= M) continue;
            row[j] = fma(-l, readlane_t<T>(row[j], p), row[j]);
            if (j == k + 1) {  // column k + 1 is done: search step k + 1
                cand = piv ? -1 : __float_as_int((float)fabs(row[k + 1]));
                mi = wave_max_dpp_i(cand);
            }
        }
#pragma unroll
        for (int q = 0; q < NR; ++q) rhs[q] = fma(-l, readlane_t<T>(rhs[q], p), rhs[q]);
    }
    step_out = mystep;
    invd_out = invd;
    if (mystep >= 0)
#pragma unroll
        for (int q = 0; q < NR; ++q) sol_lds[mystep * NR + q] = rhs[q] * invd;
    wave_lds_sync();
    if (lane < MAXM)
#pragma unroll
        for (int q = 0; q < NR; ++q) sol[q] = sol_lds[lane * NR + q];
    wave_lds_sync();
    return pmin > 0 && pmax < 0x7F800000;  // wave-uniform
}

// Replay of the recorded float32 elimination on right-hand sides b (one per
// row lane); returns in b the solution component of unknown `mystep`.
template <int MAXM, bool GUARD>
__device__ __forceinline__ void gj_replay(const float (&row)[MAXM], float (&b)[NR], int mystep, float invd, int M) {
    const int lane = lane_id();
#pragma unroll
    for (int k = 0; k < MAXM; ++k) {
        if (GUARD && k >= M) continue;
        const int p = first_lane(ballot64(mystep == k));
        const float l = (lane == p) ? 0.0f : row[k];
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const float y = readlane_f(b[q], p);
            b[q] = fmaf(-l, y, b[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) b[q] *= invd;
}

// Common prologue: sizes, rejection of bad stencils, frame.  Returns false if
// the stencil was rejected (status already written).
template <int RPL>
__device__ __forceinline__ bool stencil_prologue(const StencilArgs& a, int64_t node, int P, int maxm, int64_t& off,
                                                 int& n, int& m, FrameG<RPL>& F) {
    off = a.offsets[node];
    const int64_t n64 = a.offsets[node + 1] - off;
    m = (P >= 0 && P <= 4) ? binom(P + a.d, a.d) : 1 << 20;
    if (n64 < 1 || n64 > a.n_max || n64 + m > maxm || off < 0 || off + n64 > a.nnz) {
        reject_stencil(a, node, off, (n64 < 0 || off < 0 || off + n64 > a.nnz) ? 0 : n64, RBF_ST_BADSIZE);
        return false;
    }
    n = (int)n64;
    if (!load_frame_g<RPL>(a, off, n, m, F)) {
        reject_stencil(a, node, off, n, RBF_ST_BADSIZE);
        return false;
    }
    return true;
}

// ---------------------------------------------------------------- FP64 (<= 64)
template <int MAXM, bool GUARD>
__device__ __forceinline__ void stencil_f64_rows(const StencilArgs& a, int64_t node, int P, double* lds) {
    static_assert(MAXM <= 64, "one row per lane");
    using L = RowLds<MAXM>;
    int64_t off;
    int n, m;
    FrameG<1> F;
    if (!stencil_prologue<1>(a, node, P, MAXM, off, n, m, F)) return;
    double row[MAXM];
    double rhs[NR];
    assemble_row<MAXM, double>(a, F, n, m, lds, row, rhs);
    double s1[NR];
    int mystep;
    double invd;
    const bool ok = gauss_jordan<double, MAXM, GUARD>(row, rhs, lds + L::o_sol, s1, false, mystep, invd, n + m);
    double sol[1][NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) sol[0][q] = ok ? s1[q] : 0.0;
    const bool good = ok && repro_check<1>(a, n, m, F, sol);
    store_weights<1>(a, node, off, n, m, F, sol, good, (int8_t)RBF_ST_OK);
}

// float64 right-hand sides of this lane's row (as assemble_row)
__device__ __forceinline__ void rhs_row(const StencilArgs& a, const FrameG<1>& F, int n, int m, double (&rhs)[NR]) {
    const int d = a.d, kpow = a.phs_power;
    const int r = lane_id();
    const bool wrow = r >= m && r < m + n;
#pragma unroll
    for (int q = 0; q < NR; ++q) rhs[q] = 0.0;
    if (wrow) {
        const double r2 = F.xh[0][0] * F.xh[0][0] + F.xh[0][1] * F.xh[0][1] + F.xh[0][2] * F.xh[0][2];
        const double rr = sqrt(r2);
        const double pw = (kpow == 5) ? r2 * rr : rr;  // ||x_j||^(k-2)
#pragma unroll
        for (int q = 0; q < NR; ++q) rhs[q] = phs_lop(slot_op(a.opc, q), F.xh[0], r2, pw, kpow, d);
    } else if (r < m) {
#pragma unroll
        for (int q = 0; q < NR; ++q) rhs[q] = mono_lop(d, r, slot_op(a.opc, q));
    }
}

// ------------------------------------------------------- FP32 + refine (<= 64)
// Acceptance: every right-hand side satisfies
//     max|r| <= tol * ||K||_inf * max|x|,  tol = max(sqrt(M) 2^-53, refine_tol)
// after at least one correction; otherwise the stencil is marked FALLBACK.
template <int MAXM, bool GUARD>
__device__ __forceinline__ void stencil_ir_rows(const StencilArgs& a, int64_t node, int P, double* lds, int max_refine,
                                                double refine_tol) {
    static_assert(MAXM <= 64, "one row per lane");
    using L = RowLds<MAXM>;
    const int lane = lane_id();
    int64_t off;
    int n, m;
    FrameG<1> F;
    if (!stencil_prologue<1>(a, node, P, MAXM, off, n, m, F)) return;
    const int M = n + m;
    const int QW = MAXM - m;
    double* qt = lds + L::o_qt;
    double* xh = lds + L::o_xh;
    double* x64 = lds + L::o_sol;
    float* sol32 = reinterpret_cast<float*>(lds + L::o_f32);

    float row[MAXM];
    float b32[NR];
    {
        double B0[NR];
        assemble_row<MAXM, float>(a, F, n, m, lds, row, B0);
#pragma unroll
        for (int q = 0; q < NR; ++q) b32[q] = (float)B0[q];
    }
    float s32[NR];
    int mystep;
    float invd;
    const bool ok32 = gauss_jordan<float, MAXM, GUARD>(row, b32, sol32, s32, true, mystep, invd, M);
    // the float64 right-hand side again (cheaper than keeping it live through the elimination)
    double B[NR];
    rhs_row(a, F, n, m, B);

    bool accepted = false;
    double x[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) x[q] = (double)s32[q];
    if (ok32) {
        const double tolc0 = sqrt((double)M) * 0x1p-53;
        const double tolc = refine_tol > tolc0 ? refine_tol : tolc0;
        double knorm = 0.0;
        const int j = lane - m;
        const bool wrow = (j >= 0 && j < n);
        const bool live = lane < M;
        for (int it = 0; it <= max_refine; ++it) {
            if (lane < MAXM)
#pragma unroll
                for (int q = 0; q < NR; ++q) x64[lane * NR + q] = x[q];
            wave_lds_sync();
            // r = B - K x in float64, K's row recomputed (Q^T and offsets from LDS)
            double r[NR];
#pragma unroll
            for (int q = 0; q < NR; ++q) r[q] = B[q];
            double rowabs = 0.0;
            if (wrow) {
                for (int c = 0; c < m; ++c) {
                    const double qv = qt[c * QW + j];
                    const double2 x01 = *reinterpret_cast<const double2*>(x64 + c * NR);
                    const double2 x23 = *reinterpret_cast<const double2*>(x64 + c * NR + 2);
                    r[0] = fma(-qv, x01.x, r[0]);
                    r[1] = fma(-qv, x01.y, r[1]);
                    r[2] = fma(-qv, x23.x, r[2]);
                    r[3] = fma(-qv, x23.y, r[3]);
                    rowabs += fabs(qv);
                }
            }
            for (int c = m; c < M; ++c) {
                const int k = c - m;
                double kv;
                if (wrow) {
                    const double2 p01 = *reinterpret_cast<const double2*>(xh + 4 * k);
                    const double2 p2 = *reinterpret_cast<const double2*>(xh + 4 * k + 2);
                    const double dx = F.xh[0][0] - p01.x, dy = F.xh[0][1] - p01.y, dz = F.xh[0][2] - p2.x;
                    kv = phs_from_r2(dx * dx + dy * dy + dz * dz, a.phs_power);
                } else if (lane < m) {
                    kv = qt[lane * QW + k];
                } else {
                    kv = 0.0;
                }
                const double2 x01 = *reinterpret_cast<const double2*>(x64 + c * NR);
                const double2 x23 = *reinterpret_cast<const double2*>(x64 + c * NR + 2);
                r[0] = fma(-kv, x01.x, r[0]);
                r[1] = fma(-kv, x01.y, r[1]);
                r[2] = fma(-kv, x23.x, r[2]);
                r[3] = fma(-kv, x23.y, r[3]);
                rowabs += fabs(kv);
            }
            if (it == 0) knorm = wave_max_dpp_d(live ? rowabs : 0.0);
            if (it >= 1) {
                bool conv = true;
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    if (!(a.op_mask & (1u << q))) continue;  // slots without an operator
                    const double rn = wave_max_dpp_d(live ? fabs(r[q]) : 0.0);
                    const double xn = wave_max_dpp_d(live ? fabs(x[q]) : 0.0);
                    conv = conv && (rn <= tolc * knorm * xn);
                }
                if (conv) {
                    accepted = true;
                    break;
                }
            }
            if (it == max_refine) break;
            float rb[NR];
#pragma unroll
            for (int q = 0; q < NR; ++q) rb[q] = live ? (float)r[q] : 0.0f;
            gj_replay<MAXM, GUARD>(row, rb, mystep, invd, M);
            wave_lds_sync();
            if (mystep >= 0)
#pragma unroll
                for (int q = 0; q < NR; ++q) sol32[mystep * NR + q] = rb[q];
            wave_lds_sync();
            if (lane < MAXM)
#pragma unroll
                for (int q = 0; q < NR; ++q) x[q] += (double)sol32[lane * NR + q];
            wave_lds_sync();
        }
    }
    double sol[1][NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) sol[0][q] = x[q];
    if (accepted) accepted = repro_check<1>(a, n, m, F, sol);
    if (!accepted) {
        if (a.status && lane == 0) a.status[node] = (int8_t)RBF_ST_FALLBACK;
        return;
    }
    store_weights<1>(a, node, off, n, m, F, sol, true, (int8_t)RBF_ST_REFINED);
}

}  // namespace rbf
