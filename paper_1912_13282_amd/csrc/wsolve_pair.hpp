// RBF-FD weights of systems of 64 < n + m <= MAXM unknowns in float32 with
// float64 refinement, one stencil per wavefront, two rows per lane.
//
// Lane l holds rows l (slot 0) and l + 64 (slot 1) of K' = [0 Q^T; Q A] in
// float32 registers (the row order of wsolve.hpp).  Float rows halve the
// register footprint of the float64 four-wave solver, so one wave holds the
// whole system and the elimination needs no workgroup barrier and no LDS:
// the pivot row reaches the other lanes by lane reads into scalar registers,
// and every value read serves both rows of a lane.
//
//   * Elimination: Gauss-Jordan with partial pivoting (float magnitudes; on
//     ties the first lane, slot 0 before slot 1); each row keeps its
//     multiplier of step k in column k.
//     The pivot row is always read from slot 0: when it sits in slot 1, its lane
//     first exchanges the two slots from column k on (with their right-hand
//     sides and pivot records).  A slot's column u then holds the multiplier of
//     the row that occupied the slot at step u; the replay repeats the
//     exchanges at the same steps (recorded in LDS), so it pairs every
//     multiplier with the right row.
//   * Refinement: r = b - K x in float64 with K's entries recomputed from the
//     scaled offsets in LDS (no n^2 array is kept); the correction replays the
//     recorded row operations on float32(r).  Acceptance as the one-row form:
//     every right-hand side satisfies max|r| <= tol ||K||_inf max|x| after at
//     least one correction, tol = max(sqrt(n + m) 2^-53, refine_tol);
//     otherwise the stencil is marked FALLBACK for the float64 solve.
#pragma once

#include "wsolve.hpp"

namespace rbf {

// largest size class with this refined form (two float rows per lane: 2 x 108
// values next to the working registers of the wave)
constexpr int PAIR_MAXM = 108;

// Stencils of up to PAIR_TRI_N nodes keep the float64 PHS block A (symmetric,
// upper triangle, row-major packed) in LDS from the assembly, so the refinement
// residuals read it instead of recomputing every entry's square root; larger
// stencils recompute it.
constexpr int PAIR_TRI_N = 72;
__host__ __device__ constexpr int tri_row(int j, int n) { return j * n - (j * (j - 1)) / 2; }

template <int MAXM>
struct PairLds {
    static_assert(MAXM > 64 && MAXM <= 128, "two rows per lane");
    static constexpr int XH = MAXM * 4;       // scaled offsets, 4 doubles per node
    static constexpr int X64 = 128 * NR;      // float64 iterate, unknown order
    static constexpr int F32 = 128 * NR / 2;  // float32 solution / correction, unknown order
    static constexpr int PIV = MAXM / 2;      // pivot lane and slot swap of each step (int)
    static constexpr int TRI = PAIR_TRI_N * (PAIR_TRI_N + 1) / 2;  // float64 PHS block, upper triangle
    static constexpr int TOTAL = XH + X64 + F32 + PIV + TRI;
    static constexpr int o_xh = 0, o_x = XH, o_f32 = XH + X64, o_piv = XH + X64 + F32, o_tri = XH + X64 + F32 + PIV;
};

// exchange of two registers in place (on the active lanes)
__device__ __forceinline__ void vswap(float& x, float& y) { asm volatile("v_swap_b32 %0, %1" : "+v"(x), "+v"(y)); }

// x^e for a per-lane exponent e in 0..4
__device__ __forceinline__ double ipow4_v(double x, int e) {
    const double x2 = x * x;
    double v = (e & 1) ? x : 1.0;
    v = (e & 2) ? v * x2 : v;
    return (e & 4) ? x2 * x2 : v;
}

// One row of K' (float64): row r, column c; xr = the scaled offset of the
// row's node (weight rows), xk from LDS.  e[3]: exponents of monomial r (poly rows).
__device__ __forceinline__ double pair_entry(int d, int kpow, int m, int n, int r, int c, const double (&xr)[3],
                                             const int (&e)[3], const double* xh) {
    const int M = n + m;
    if (c >= M) return r == c ? 1.0 : 0.0;
    if (r < m) {
        if (c < m) return 0.0;
        const double* xk = xh + 4 * (c - m);
        return ipow4_v(xk[0], e[0]) * ipow4_v(xk[1], e[1]) * ipow4_v(xk[2], e[2]);
    }
    if (r >= M) return r == c ? 1.0 : 0.0;
    if (c < m) return mono(d, c, xr);
    const double* xk = xh + 4 * (c - m);
    const double dx = xr[0] - xk[0], dy = xr[1] - xk[1], dz = xr[2] - xk[2];
    return phs_from_r2(dx * dx + dy * dy + dz * dz, kpow);
}

// float64 right-hand sides of row r (node offsets xr for weight rows)
__device__ __forceinline__ void pair_rhs(const StencilArgs& a, int m, int n, int r, const double (&xr)[3],
                                         double (&B)[NR]) {
    const int d = a.d, kpow = a.phs_power;
    const int j = r - m;
#pragma unroll
    for (int q = 0; q < NR; ++q) B[q] = 0.0;
    if (j >= 0 && j < n) {
        const double r2 = xr[0] * xr[0] + xr[1] * xr[1] + xr[2] * xr[2];
        const double rr = sqrt(r2);
        const double pw = (kpow == 5) ? r2 * rr : rr;
#pragma unroll
        for (int q = 0; q < NR; ++q) B[q] = phs_lop(slot_op(a.opc, q), xr, r2, pw, kpow, d);
    } else if (r < m) {
#pragma unroll
        for (int q = 0; q < NR; ++q) B[q] = mono_lop(d, r, slot_op(a.opc, q));
    }
}

// scaled offset of the node of row r (zeros for polynomial and padding rows)
__device__ __forceinline__ void pair_xr(const double* xh, int m, int n, int r, double (&xr)[3]) {
    const int j = r - m;
    xr[0] = xr[1] = xr[2] = 0.0;
    if (j >= 0 && j < n) {
        const double2 p01 = *reinterpret_cast<const double2*>(xh + 4 * j);
        xr[0] = p01.x;
        xr[1] = p01.y;
        xr[2] = xh[4 * j + 2];
    }
}

template <int MAXM>
__device__ __forceinline__ void stencil_ir_pair(const StencilArgs& a, int64_t node, int P, double* lds, int max_refine,
                                                double refine_tol) {
    using L = PairLds<MAXM>;
    const int lane = lane_id();
    int64_t off;
    int n, m;
    double inv_s;
    double* xh = lds + L::o_xh;
    double* x64 = lds + L::o_x;
    float* c32 = reinterpret_cast<float*>(lds + L::o_f32);
    {
        FrameG<2> F;
        if (!stencil_prologue<2>(a, node, P, MAXM, off, n, m, F)) return;
        inv_s = F.inv_s;
        // scaled offsets of every node to LDS (weight row m + j holds node j)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int j = lane + 64 * t - m;
            if (j >= 0 && j < n) {
                *reinterpret_cast<double2*>(xh + 4 * j) = make_double2(F.xh[t][0], F.xh[t][1]);
                *reinterpret_cast<double2*>(xh + 4 * j + 2) = make_double2(F.xh[t][2], 0.0);
            }
        }
    }
    wave_lds_sync();
    const int M = n + m;
    const int d = a.d, kpow = a.phs_power;
    double* tri = lds + L::o_tri;
    const bool tri_ok = n <= PAIR_TRI_N;
    // ---- assembly in float64, rounded to float32.  Order chosen for register
    // pressure: right-hand sides first, then the PHS columns, then the cheap
    // monomial columns, so few temporaries are live next to the full rows.
    float row0[MAXM], row1[MAXM];
    float b0[NR], b1[NR];
    {
        double x0[3], x1[3];
        pair_xr(xh, m, n, lane, x0);
        pair_xr(xh, m, n, lane + 64, x1);
        {
            double B[NR];
            pair_rhs(a, m, n, lane, x0, B);
#pragma unroll
            for (int q = 0; q < NR; ++q) b0[q] = (float)B[q];
            pair_rhs(a, m, n, lane + 64, x1, B);
#pragma unroll
            for (int q = 0; q < NR; ++q) b1[q] = (float)B[q];
        }
        const int r0 = lane, r1 = lane + 64;
        const int j0 = r0 - m, j1 = r1 - m;
        const bool w0 = j0 >= 0 && j0 < n, w1 = j1 >= 0 && j1 < n;
        const bool q0 = r0 < m;  // polynomial row (slot 0 only: m <= 35 < 64)
        int e[3] = {0, 0, 0};    // its monomial's exponents
        if (q0) mono_exp(d, lane, e[0], e[1], e[2]);
        // columns c >= m: node k = c - m; branch-free per lane (the entry of every
        // row kind is formed and the row's own one selected)
#pragma unroll
        for (int c = 0; c < MAXM; ++c) {
            if (c >= m) {  // uniform
                const int k = c - m;
                const bool live = k < n;
                const int kk = live ? k : 0;
                const double2 p01 = *reinterpret_cast<const double2*>(xh + 4 * kk);
                const double p2 = xh[4 * kk + 2];
                const double dx0 = x0[0] - p01.x, dy0 = x0[1] - p01.y, dz0 = x0[2] - p2;
                const double dx1 = x1[0] - p01.x, dy1 = x1[1] - p01.y, dz1 = x1[2] - p2;
                const double a0 = phs_from_r2(dx0 * dx0 + dy0 * dy0 + dz0 * dz0, kpow);
                const double a1 = phs_from_r2(dx1 * dx1 + dy1 * dy1 + dz1 * dz1, kpow);
                if (tri_ok) {  // uniform
                    if (w0 && live && k >= j0) tri[tri_row(j0, n) + k - j0] = a0;
                    if (w1 && live && k >= j1) tri[tri_row(j1, n) + k - j1] = a1;
                }
                const double qv = ipow4_v(p01.x, e[0]) * ipow4_v(p01.y, e[1]) * ipow4_v(p2, e[2]);
                const float pad0 = (r0 == c) ? 1.0f : 0.0f, pad1 = (r1 == c) ? 1.0f : 0.0f;
                row0[c] = !live ? pad0 : (w0 ? (float)a0 : (q0 ? (float)qv : pad0));
                row1[c] = !live ? pad1 : (w1 ? (float)a1 : pad1);
            }
        }
        // columns c < m (uniform phase): monomial c at the weight rows' nodes; the
        // polynomial and padding rows are 0 there.  m <= 35 bounds the phase.
#pragma unroll
        for (int c = 0; c < MAXM; ++c) {
            if (c < 35 && c < m) {
                row0[c] = w0 ? (float)mono(d, c, x0) : 0.0f;
                row1[c] = w1 ? (float)mono(d, c, x1) : 0.0f;
            }
        }
    }

    // ---- float32 Gauss-Jordan, multipliers kept in the eliminated columns
    int* pinfo = reinterpret_cast<int*>(lds + L::o_piv);
    bool piv0 = lane >= M, piv1 = lane + 64 >= M;  // padding rows never pivot
    int step0 = -1, step1 = -1;
    float invd0 = 0.0f, invd1 = 0.0f;
    int pmin = 0x7F7FFFFF, pmax = 0;
    int c0 = piv0 ? -1 : __float_as_int(fabsf(row0[0]));
    int c1 = piv1 ? -1 : __float_as_int(fabsf(row1[0]));
    int mi = wave_max_dpp_i(max(c0, c1));
#pragma unroll
    for (int k = 0; k < MAXM; ++k) {
        if (k < M) {  // uniform
            pmin = min(pmin, mi);
            pmax = max(pmax, mi);
            // among the maxima: the first lane, slot 0 before slot 1
            const uint64_t bs0 = ballot64(!piv0 && c0 == mi);
            const bool sub = bs0 == 0;
            const int p = first_lane(sub ? ballot64(!piv1 && c1 == mi) : bs0);
            if (lane == 0) pinfo[k] = p | (sub ? 256 : 0);
            if (sub) {  // uniform: move the pivot row of lane p into slot 0
                if (lane == p) {
                    // in-place exchanges on the one active lane (a renaming swap would
                    // leave both versions of every register live where the branch joins)
#pragma unroll
                    for (int c = k; c < MAXM; ++c) vswap(row0[c], row1[c]);
#pragma unroll
                    for (int q = 0; q < NR; ++q) vswap(b0[q], b1[q]);
                    const bool tp = piv0;
                    piv0 = piv1;
                    piv1 = tp;
                    const int ts = step0;
                    step0 = step1;
                    step1 = ts;
                    const float ti = invd0;
                    invd0 = invd1;
                    invd1 = ti;
                }
            }
            const bool me = lane == p;
            const float inv = recip(readlane_f(row0[k], p));
            if (me) {
                piv0 = true;
                step0 = k;
                invd0 = inv;
            }
            const float l0 = me ? 0.0f : row0[k] * inv;
            const float l1 = row1[k] * inv;
            if (!me) row0[k] = l0;
            row1[k] = l1;
#pragma unroll
            for (int j = k + 1; j < MAXM; ++j) {
                const float u = readlane_f(row0[j], p);
                row0[j] = fmaf(-l0, u, row0[j]);
                row1[j] = fmaf(-l1, u, row1[j]);
                if (j == k + 1) {  // column k + 1 is done: search step k + 1
                    c0 = piv0 ? -1 : __float_as_int(fabsf(row0[k + 1]));
                    c1 = piv1 ? -1 : __float_as_int(fabsf(row1[k + 1]));
                    mi = wave_max_dpp_i(max(c0, c1));
                }
                // keep the lane reads next to their multiply-adds (hoisting them
                // ahead runs out of scalar registers)
                if ((j & 7) == 7) __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                const float u = readlane_f(b0[q], p);
                b0[q] = fmaf(-l0, u, b0[q]);
                b1[q] = fmaf(-l1, u, b1[q]);
            }
        }
    }
    const bool ok32 = pmin > 0 && pmax < 0x7F800000;

    // v / U_kk of each pivot row, to the unknown of its step, in LDS (float32)
    auto scatter = [&](const float (&v0)[NR], const float (&v1)[NR]) {
        wave_lds_sync();
        if (step0 >= 0)
#pragma unroll
            for (int q = 0; q < NR; ++q) c32[step0 * NR + q] = v0[q] * invd0;
        if (step1 >= 0)
#pragma unroll
            for (int q = 0; q < NR; ++q) c32[step1 * NR + q] = v1[q] * invd1;
        wave_lds_sync();
    };
    // the iterate lives in LDS (float64, unknown order): x64[u * NR + q]
    scatter(b0, b1);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int u = lane + 64 * t;
        if (u < M)
#pragma unroll
            for (int q = 0; q < NR; ++q) x64[u * NR + q] = (double)c32[u * NR + q];
    }
    wave_lds_sync();

    bool accepted = false;
    if (ok32) {
        const double tolc0 = sqrt((double)M) * 0x1p-53;
        const double tolc = refine_tol > tolc0 ? refine_tol : tolc0;
        double knorm = 0.0;
        int e[3] = {0, 0, 0};  // exponents of the polynomial row in slot 0
        if (lane < m) mono_exp(d, lane, e[0], e[1], e[2]);
        for (int it = 0; it <= max_refine; ++it) {
            // r = B - K x in float64 (K's rows recomputed), one row slot at a time;
            // the norms of the acceptance test are taken from float32(r) and x in LDS
            float y0[NR], y1[NR];
            double rowabs = 0.0;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int rr = lane + 64 * t;
                double xr[3];
                pair_xr(xh, m, n, rr, xr);
                double r[NR];
                pair_rhs(a, m, n, rr, xr, r);
                double ra = 0.0;
                if (tri_ok) {  // uniform
                    const int j = rr - m;
                    const bool wr = j >= 0 && j < n, qr = t == 0 && rr < m;  // m <= 35: no polynomial row in slot 1
                    // columns c < m: monomials at the weight row's node (0 in the other rows)
                    for (int c = 0; c < m; ++c) {
                        const double kv = wr ? mono(d, c, xr) : 0.0;
                        const double2 x01 = *reinterpret_cast<const double2*>(x64 + c * NR);
                        r[0] = fma(-kv, x01.x, r[0]);
                        r[1] = fma(-kv, x01.y, r[1]);
                        const double2 x23 = *reinterpret_cast<const double2*>(x64 + c * NR + 2);
                        r[2] = fma(-kv, x23.x, r[2]);
                        r[3] = fma(-kv, x23.y, r[3]);
                        if (it == 0) ra += fabs(kv);
                    }
                    // columns m + k: A_jk from the stored triangle, or monomial rr at node k
                    const int tj = wr ? tri_row(j, n) - j : 0;
                    for (int k = 0; k < n; ++k) {
                        const int tk = tri_row(k, n) - k;
                        const int ti = wr ? ((k >= j) ? tj + k : tk + j) : 0;
                        const double av = tri[ti];
                        double qv = 0.0;
                        if (t == 0) {
                            const double2 p01 = *reinterpret_cast<const double2*>(xh + 4 * k);
                            qv = ipow4_v(p01.x, e[0]) * ipow4_v(p01.y, e[1]) * ipow4_v(xh[4 * k + 2], e[2]);
                        }
                        const double kv = wr ? av : (qr ? qv : 0.0);
                        const int c = m + k;
                        const double2 x01 = *reinterpret_cast<const double2*>(x64 + c * NR);
                        r[0] = fma(-kv, x01.x, r[0]);
                        r[1] = fma(-kv, x01.y, r[1]);
                        const double2 x23 = *reinterpret_cast<const double2*>(x64 + c * NR + 2);
                        r[2] = fma(-kv, x23.x, r[2]);
                        r[3] = fma(-kv, x23.y, r[3]);
                        if (it == 0) ra += fabs(kv);
                    }
                } else if (rr < M) {
                    for (int c = 0; c < M; ++c) {
                        const double kv = pair_entry(d, kpow, m, n, rr, c, xr, e, xh);
                        const double2 x01 = *reinterpret_cast<const double2*>(x64 + c * NR);
                        r[0] = fma(-kv, x01.x, r[0]);
                        r[1] = fma(-kv, x01.y, r[1]);
                        const double2 x23 = *reinterpret_cast<const double2*>(x64 + c * NR + 2);
                        r[2] = fma(-kv, x23.x, r[2]);
                        r[3] = fma(-kv, x23.y, r[3]);
                        if (it == 0) ra += fabs(kv);
                    }
                }
                rowabs = fmax(rowabs, ra);
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    const float v = rr < M ? (float)r[q] : 0.0f;
                    if (t == 0) y0[q] = v;
                    else y1[q] = v;
                }
            }
            if (it == 0) knorm = wave_max_dpp_d(rowabs);
            if (it >= 1) {
                bool conv = true;
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    if (!(a.op_mask & (1u << q))) continue;  // slots without an operator
                    const double xa = (lane < M) ? fabs(x64[lane * NR + q]) : 0.0;
                    const double xb = (lane + 64 < M) ? fabs(x64[(lane + 64) * NR + q]) : 0.0;
                    const double rn = wave_max_dpp_d((double)fmaxf(fabsf(y0[q]), fabsf(y1[q])));
                    conv = conv && (rn <= tolc * knorm * wave_max_dpp_d(fmax(xa, xb)));
                }
                if (conv) {
                    accepted = true;
                    break;
                }
            }
            if (it == max_refine) break;
            // correction: replay the recorded elimination on float32(r)
#pragma unroll
            for (int k = 0; k < MAXM; ++k) {
                if (k < M) {  // uniform
                    const int info = __builtin_amdgcn_readfirstlane(pinfo[k]);
                    const int p = info & 255;
                    if ((info & 256) && lane == p)  // the exchange of the elimination, at the same step
#pragma unroll
                        for (int q = 0; q < NR; ++q) vswap(y0[q], y1[q]);
                    // the multipliers of step k sit in column k of each slot
                    const float l0 = (lane == p) ? 0.0f : row0[k];
                    const float l1 = row1[k];
#pragma unroll
                    for (int q = 0; q < NR; ++q) {
                        const float u = readlane_f(y0[q], p);
                        y0[q] = fmaf(-l0, u, y0[q]);
                        y1[q] = fmaf(-l1, u, y1[q]);
                    }
                }
            }
            scatter(y0, y1);
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int u = lane + 64 * t;
                if (u < M)
#pragma unroll
                    for (int q = 0; q < NR; ++q) x64[u * NR + q] += (double)c32[u * NR + q];
            }
            wave_lds_sync();
        }
    }
    // FP64 reproduction check and store (the weights are the unknowns m .. M-1)
    double sol[2][NR];
    FrameG<2> G;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int u = lane + 64 * t;
        pair_xr(xh, m, n, u, G.xh[t]);
#pragma unroll
        for (int q = 0; q < NR; ++q) sol[t][q] = (u < M) ? x64[u * NR + q] : 0.0;
    }
    G.inv_s = inv_s;
    G.s = 1.0 / inv_s;
    if (accepted) accepted = repro_check<2>(a, n, m, G, sol);
    if (!accepted) {
        if (a.status && lane == 0) a.status[node] = (int8_t)RBF_ST_FALLBACK;
        return;
    }
    store_weights<2>(a, node, off, n, m, G, sol, true, (int8_t)RBF_ST_REFINED);
}

}  // namespace rbf
