// RBF-FD weights of one stencil per 4-wave workgroup, for systems of
// 64 < n + m <= 2H unknowns (float64 Gauss-Jordan with partial pivoting).
//
// Layout.  Wave w of the workgroup holds row r = 64 (w & 1) + lane of K'
// (row group w & 1) restricted to the column half c in [H (w >> 1), H (w >> 1) + H)
// (column half w >> 1): 2H rows x 2H columns over 256 lanes, H doubles per lane,
// all in registers.  The right-hand sides live with column half 0.
//
// Step k (one fully unrolled iteration; k < n + m):
//   1. the two waves of the column half owning column k search their 64 rows
//      for the pivot (DPP max on float magnitudes) and publish their candidate
//      and their whole column k in LDS                              -- barrier
//   2. every lane reads the winning row, the pivot value and its own column-k
//      entry, so it forms its multiplier itself; the two lanes holding the
//      pivot row write their halves of it                          -- barrier
//   3. every lane updates its columns > k (and the right-hand sides).
// The LDS buffers of consecutive steps alternate, so a step never overwrites
// data another wave may still read.  Rows are never swapped (Gauss-Jordan in
// the one-row-per-lane form): a pivoted row keeps its step number, and at the
// end x_k = rhs / U_kk of the row pivoted at step k.
#pragma once

#include "wsolve.hpp"

namespace rbf {

constexpr int QB = 8;  // pivot-row reads in flight per batch of the update

template <int H>
struct QuadLds {
    static constexpr int M2 = 2 * H;
    static constexpr int XH = M2 * 4;               // scaled offsets, 4 doubles per node
    static constexpr int COL = 2 * 128;             // column k of all 128 rows (two row groups), two buffers
    static constexpr int PRW = M2 + NR;             // one pivot row + right-hand sides
    static constexpr int PR = 2 * PRW;              // two buffers
    static constexpr int SOL = M2 * NR;             // solution in unknown order
    static constexpr int RED = 64;                  // reductions and candidates
    static constexpr int TOTAL = XH + COL + PR + SOL + RED;
    static constexpr int o_xh = 0, o_col = XH, o_pr = XH + COL, o_sol = XH + COL + PR, o_red = XH + COL + PR + SOL;
};

// Gauss-Jordan steps k < M for the waves of column half CH (see the header
// comment); every wave of the workgroup runs the same sequence of barriers.
template <int H, int CH>
__device__ __forceinline__ void quad_eliminate(double (&row)[H], double (&rhs)[NR], double* lds, int r, int rg,
                                               int lane, int M, int& mystep, double& invd, int& pmin, int& pmax) {
    using L = QuadLds<H>;
    constexpr int M2 = 2 * H;
    int* redi = reinterpret_cast<int*>(lds + L::o_red);
    bool piv = r >= M;  // padding rows (r >= n + m) take no part
#pragma unroll
    for (int k = 0; k < M2; ++k) {
        if (k < M) {  // uniform
            const int par = k & 1;
            double* col = lds + L::o_col + par * 128;
            double* prow = lds + L::o_pr + par * L::PRW;
            int* cand = redi + 16 + 8 * par;  // [rg][2]: max bits, lane
            if (CH == k / H) {
                const double ck = row[k % H];
                col[r] = ck;
                const int cb = piv ? -1 : __float_as_int((float)fabs(ck));
                const int mi = wave_max_dpp_i(cb);
                const uint64_t b = ballot64(!piv && cb == mi);
                if (lane == 0) {
                    cand[2 * rg] = mi;
                    cand[2 * rg + 1] = b ? first_lane(b) : 0;
                }
            }
            __syncthreads();
            const int m0 = cand[0], m1 = cand[2];
            const int prg = (m1 > m0) ? 1 : 0;  // ties: the smaller row
            const int mi = prg ? m1 : m0;
            const int pr = 64 * prg + cand[2 * prg + 1];
            pmin = min(pmin, mi);
            pmax = max(pmax, mi);
            const double inv = recip(col[pr]);
            const bool me = (r == pr);
            const double l = me ? 0.0 : col[r] * inv;
            if (me) {
                piv = true;
                mystep = k;
                invd = inv;
                // one 8-byte store per value, kept apart by an empty asm: merged stores
                // need their data in an aligned register tuple (a copy of every value)
#pragma unroll
                for (int cl = 0; cl < H; ++cl) {
                    if (H * CH + cl > k) prow[H * CH + cl] = row[cl];
                    asm volatile("" ::: "memory");
                }
                if (CH == 0)
#pragma unroll
                    for (int q = 0; q < NR; ++q) {
                        prow[M2 + q] = rhs[q];
                        asm volatile("" ::: "memory");
                    }
            }
            __syncthreads();
            // the pivot row in batches of QB 16-byte reads issued ahead of their
            // FMAs, so that a batch's LDS latency is paid once
#pragma unroll
            for (int cb = 0; cb < H; cb += 2 * QB) {
                double2 u[QB];
#pragma unroll
                for (int b = 0; b < QB; ++b) {
                    const int cl0 = cb + 2 * b;
                    if (cl0 < H && H * CH + cl0 + 1 > k)  // a column of the pair is still live
                        u[b] = *reinterpret_cast<const double2*>(prow + H * CH + cl0);
                }
#pragma unroll
                for (int b = 0; b < QB; ++b) {
                    const int cl0 = cb + 2 * b;
                    if (cl0 < H && H * CH + cl0 + 1 > k) {
                        if (H * CH + cl0 > k) row[cl0] = fma(-l, u[b].x, row[cl0]);
                        row[cl0 + 1] = fma(-l, u[b].y, row[cl0 + 1]);
                    }
                }
            }
            if (CH == 0) {
                const double2 u0 = *reinterpret_cast<const double2*>(prow + M2);
                const double2 u1 = *reinterpret_cast<const double2*>(prow + M2 + 2);
                rhs[0] = fma(-l, u0.x, rhs[0]);
                rhs[1] = fma(-l, u0.y, rhs[1]);
                rhs[2] = fma(-l, u1.x, rhs[2]);
                rhs[3] = fma(-l, u1.y, rhs[3]);
            }
        }
    }
}

// all 256 threads of the workgroup call this with the same node
template <int H>
__device__ __forceinline__ void stencil_f64_quad(const StencilArgs& a, int64_t node, int P, double* lds) {
    using L = QuadLds<H>;
    constexpr int M2 = 2 * H;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int rg = wv & 1, ch = wv >> 1;
    const int r = 64 * rg + lane;  // this lane's row of K'
    double* xh = lds + L::o_xh;
    double* red = lds + L::o_red;
    int* redi = reinterpret_cast<int*>(red);

    const int64_t off = a.offsets[node];
    const int64_t n64 = a.offsets[node + 1] - off;
    const int d = a.d;
    const int m = (P >= 0 && P <= 4) ? binom(P + d, d) : 1 << 20;
    if (n64 < 1 || n64 > a.n_max || n64 + m > M2 || off < 0 || off + n64 > a.nnz) {
        const int R = __builtin_popcount(a.op_mask);
        const int64_t nn = (n64 < 0 || off < 0 || off + n64 > a.nnz) ? 0 : n64;
        for (int q = 0; q < R; ++q)
            for (int64_t e = tid; e < nn; e += 256) a.w[q * a.nnz + off + e] = __builtin_nan("");
        if (a.status && tid == 0) a.status[node] = RBF_ST_BADSIZE;
        return;
    }
    const int n = (int)n64, M = n + m;

    // ---- frame: scaled offsets of all nodes (threads 0..n-1), scale s
    double o3[3] = {0.0, 0.0, 0.0};
    bool bad = false;
    double r2 = 0.0, r2n = INFINITY;
    {
        const int c = a.idx[off];
        bad = !(c >= 0 && c < a.N);
        if (tid < n && !bad) {
            const int id = a.idx[off + tid];
            if (id >= 0 && id < a.N) {
                for (int q = 0; q < d; ++q) o3[q] = a.X[(int64_t)id * d + q] - a.X[(int64_t)c * d + q];
            } else {
                bad = true;
            }
            r2 = o3[0] * o3[0] + o3[1] * o3[1] + o3[2] * o3[2];
            if (tid >= 1) r2n = r2;
        }
    }
    {
        const double vmax = wave_max_d(r2), vmin = wave_min_d(r2n);
        const uint64_t bb = ballot64(bad);
        if (lane == 0) {
            red[2 * wv] = vmax;
            red[2 * wv + 1] = vmin;
            redi[32 + wv] = bb != 0;
        }
    }
    __syncthreads();
    const double s2 = (a.scale_mode == 1) ? fmin(fmin(red[1], red[3]), fmin(red[5], red[7]))
                                          : fmax(fmax(red[0], red[2]), fmax(red[4], red[6]));
    const bool badidx = (redi[32] | redi[33] | redi[34] | redi[35]) != 0;
    const double s = sqrt(s2), inv_s = 1.0 / s;
    if (tid < n) {
        *reinterpret_cast<double2*>(xh + 4 * tid) = make_double2(o3[0] * inv_s, o3[1] * inv_s);
        *reinterpret_cast<double2*>(xh + 4 * tid + 2) = make_double2(o3[2] * inv_s, 0.0);
    }
    __syncthreads();
    if (badidx) {
        const int R = __builtin_popcount(a.op_mask);
        for (int q = 0; q < R; ++q)
            for (int e = tid; e < n; e += 256) a.w[q * a.nnz + off + e] = __builtin_nan("");
        if (a.status && tid == 0) a.status[node] = RBF_ST_BADSIZE;
        return;
    }

    // ---- assembly of this lane's half row (float64)
    const int kpow = a.phs_power;
    const int jr = r - m;  // node of this row, if a weight row
    double xr[3] = {0.0, 0.0, 0.0};
    if (jr >= 0 && jr < n) {
        xr[0] = xh[4 * jr];
        xr[1] = xh[4 * jr + 1];
        xr[2] = xh[4 * jr + 2];
    }
    double row[H];
#pragma unroll
    for (int cl = 0; cl < H; ++cl) {
        const int c = H * ch + cl;
        double v = 0.0;
        if (r < m) {  // polynomial row r: [0 | Q^T]
            if (c >= m && c < M) {
                const int k = c - m;
                const double xk[3] = {xh[4 * k], xh[4 * k + 1], xh[4 * k + 2]};
                v = mono(d, r, xk);
            }
        } else if (r < M) {  // weight row of node jr: [Q | A]
            if (c < m) {
                v = mono(d, c, xr);
            } else if (c < M) {
                const int k = c - m;
                const double dx = xr[0] - xh[4 * k], dy = xr[1] - xh[4 * k + 1], dz = xr[2] - xh[4 * k + 2];
                v = phs_from_r2(dx * dx + dy * dy + dz * dz, kpow);
            }
        } else {
            v = (r == c) ? 1.0 : 0.0;  // padding row
        }
        row[cl] = v;
    }
    double rhs[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) rhs[q] = 0.0;
    if (ch == 0) {
        if (jr >= 0 && jr < n) {
            const double rr2 = xr[0] * xr[0] + xr[1] * xr[1] + xr[2] * xr[2];
            const double rr = sqrt(rr2);
            const double pw = (kpow == 5) ? rr2 * rr : rr;  // ||x_j||^(k-2)
#pragma unroll
            for (int q = 0; q < NR; ++q) rhs[q] = phs_lop(slot_op(a.opc, q), xr, rr2, pw, kpow, d);
        } else if (r < m) {
#pragma unroll
            for (int q = 0; q < NR; ++q) rhs[q] = mono_lop(d, r, slot_op(a.opc, q));
        }
    }

    // ---- Gauss-Jordan (the column half is uniform per wave: one specialised
    // copy per half, so every column test below is a compile-time constant)
    int mystep = -1;
    double invd = 0.0;
    int pmin = 0x7F7FFFFF, pmax = 0;
    if (ch == 0) quad_eliminate<H, 0>(row, rhs, lds, r, rg, lane, M, mystep, invd, pmin, pmax);
    else quad_eliminate<H, 1>(row, rhs, lds, r, rg, lane, M, mystep, invd, pmin, pmax);
    const bool ok = pmin > 0 && pmax < 0x7F800000;

    // ---- solution in unknown order, reproduction check, store
    double* sol = lds + L::o_sol;
    if (ch == 0 && mystep >= 0)
#pragma unroll
        for (int q = 0; q < NR; ++q) sol[mystep * NR + q] = rhs[q] * invd;
    __syncthreads();
    double w4[NR] = {0.0, 0.0, 0.0, 0.0};
    double S[NR] = {0.0, 0.0, 0.0, 0.0}, A[NR] = {0.0, 0.0, 0.0, 0.0};
    if (tid < n) {
        const double x3[3] = {xh[4 * tid], xh[4 * tid + 1], xh[4 * tid + 2]};
        double pvl = 0.0;
        for (int l2 = 0; l2 < m; ++l2) pvl += check_coef(l2) * mono(d, l2, x3);
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            w4[q] = ok ? sol[(m + tid) * NR + q] : 0.0;
            const double v = w4[q] * pvl;
            S[q] = v;
            A[q] = fabs(v);
        }
    }
    __syncthreads();  // red is reused below
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const double sq = wave_sum_dpp_d(S[q]), aq = wave_sum_dpp_d(A[q]);
        if (lane == 0) {
            red[8 * wv + 2 * q] = sq;
            red[8 * wv + 2 * q + 1] = aq;
        }
    }
    __syncthreads();
    bool good = ok;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        if (!(a.op_mask & (1u << q))) continue;
        const double sq = (red[2 * q] + red[8 + 2 * q]) + (red[16 + 2 * q] + red[24 + 2 * q]);
        const double aq = (red[2 * q + 1] + red[8 + 2 * q + 1]) + (red[16 + 2 * q + 1] + red[24 + 2 * q + 1]);
        double lp = 0.0;
        for (int l2 = 0; l2 < m; ++l2) lp += check_coef(l2) * mono_lop(d, l2, slot_op(a.opc, q));
        good = good && (fabs(sq - lp) / (aq + fabs(lp)) <= a.repro_tol);
    }
    if (tid < n) {
        int ro = 0;
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            if (!(a.op_mask & (1u << q))) continue;
            const double sc = op_order(slot_op(a.opc, q)) == 2 ? inv_s * inv_s : inv_s;
            a.w[ro * a.nnz + off + tid] = good ? w4[q] * sc : __builtin_nan("");
            ++ro;
        }
    }
    if (a.status && tid == 0) a.status[node] = good ? (int8_t)RBF_ST_OK : (int8_t)RBF_ST_SINGULAR;
    __syncthreads();  // the LDS is reused by the next stencil
}

}  // namespace rbf
