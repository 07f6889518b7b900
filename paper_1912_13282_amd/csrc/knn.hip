// Exact k-nearest-neighbour stencil selection on a uniform cell grid (gfx950).
//
// Stencil of node i (Sec. 2.1 of the Medusa paper, FindClosest of Sec. 3.1):
// i itself, then the n_i - 1 nodes j != i with the smallest float64 key
// ((dx*dx + dy*dy) + dz*dz), dx = x_j - x_i, ties broken by the smaller j.
//
// Pipeline (all on the caller's stream, no host synchronisation):
//   k_bbox_partial / k_grid_setup : bounding box, cell side, grid dimensions
//   k_bin_count                   : cell of every node + rank inside its cell
//   k_scan_*                      : exclusive scan of the cell counts
//   k_bin_scatter                 : node ids and SoA coordinates in cell order
//   k_knn_radius_group<QW, SPL>   : 64 / QW query nodes per wavefront (n_i <= 41):
//   k_knn_radius                  : one wavefront per query node (n_i <= 101):
//       every node within a radius estimated from the local density is
//       filtered by its key, the survivors compacted in LDS and ordered once on
//       (key, index) (exact: at least k survivors prove the radius sufficient)
//   k_knn<T>, k_knn_list          : one wavefront per query node, n_i <= 129
//       (and the queries the radius search leaves unsettled): candidates of the surrounding
//       cells are streamed in chunks of 64*T, bitonic-sorted across the wave on
//       (key, index) and merged into a sorted top list of 64*T entries; rings of
//       cells are added until the k-th key is below the squared distance to
//       the unsearched region (exact termination).
#include "cellorder.hpp"
#include "common.hpp"

#include <math.h>

#include <algorithm>
#include <mutex>

namespace {

struct GridParams {
    double origin[3];
    double cell;
    double inv_cell;
    int dims[3];
    int ncell;
};

constexpr int BBOX_BLOCKS = 512;
// mean nodes per cell relative to n_max / (unit-ball volume), i.e. the cell
// volume relative to the stencil ball: cells a fraction of the ball keep the
// cells gathered around a search radius close to the ball itself
constexpr double CELL_FILL_2D = 0.5;
constexpr double CELL_FILL_3D = 0.25;
constexpr int SCAN_CHUNK = 1024;  // elements per scan block (256 threads x 4)

__global__ __launch_bounds__(256) void k_zero_ints(int* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Bounding-box partials of the nodes (grid-stride, four nodes per thread and
// pass so their loads are in flight together; an index clamped into range
// repeats a node, which leaves a minimum or maximum unchanged).
template <int D>
__global__ __launch_bounds__(256) void k_bbox_partial(const double* __restrict__ X, int64_t N,
                                                      double* __restrict__ part) {
    __shared__ double sm[4][6];
    double mn[3] = {INFINITY, INFINITY, INFINITY};
    double mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < N; i0 += 4 * stride) {
        double v[4][D];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = min(i0 + u * stride, N - 1);
#pragma unroll
            for (int a = 0; a < D; ++a) v[u][a] = X[i * D + a];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int a = 0; a < D; ++a) {
                mn[a] = fmin(mn[a], v[u][a]);
                mx[a] = fmax(mx[a], v[u][a]);
            }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        mn[a] = wave_min_d(mn[a]);
        mx[a] = wave_max_d(mx[a]);
    }
    const int w = threadIdx.x / WAVE;
    if (lane_id() == 0)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            sm[w][a] = mn[a];
            sm[w][3 + a] = mx[a];
        }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int a = threadIdx.x;
        double v = sm[0][a];
        for (int k = 1; k < 4; ++k) v = (a < 3) ? fmin(v, sm[k][a]) : fmax(v, sm[k][a]);
        part[blockIdx.x * 6 + a] = v;
    }
}

inline void bbox_enqueue(hipStream_t s, int nbb, const double* X, int64_t N, int d, double* part) {
    if (d == 3)
        hipLaunchKernelGGL(k_bbox_partial<3>, dim3(nbb), dim3(256), 0, s, X, N, part);
    else
        hipLaunchKernelGGL(k_bbox_partial<2>, dim3(nbb), dim3(256), 0, s, X, N, part);
}

__global__ __launch_bounds__(64) void k_grid_setup(const double* __restrict__ part, int nb, int64_t N, int d,
                                                   double target_per_cell, int64_t cap, GridParams* gp) {
    double mn[3], mx[3];
    for (int a = 0; a < 3; ++a) {
        double lo = INFINITY, hi = -INFINITY;
        for (int b = lane_id(); b < nb; b += WAVE) {
            lo = fmin(lo, part[b * 6 + a]);
            hi = fmax(hi, part[b * 6 + 3 + a]);
        }
        mn[a] = wave_min_d(lo);
        mx[a] = wave_max_d(hi);
    }
    if (threadIdx.x != 0) return;
    double ext[3] = {0, 0, 0}, emax = 0;
    for (int a = 0; a < d; ++a) {
        ext[a] = mx[a] - mn[a];
        emax = fmax(emax, ext[a]);
    }
    double cell;
    if (!(emax > 0)) {
        cell = 1.0;
    } else {
        double vol = 1.0;
        for (int a = 0; a < d; ++a) vol *= fmax(ext[a], emax * 1e-3);
        cell = pow(target_per_cell * vol / (double)N, 1.0 / d);
        cell = fmax(cell, emax * 1e-7);
    }
    int dims[3] = {1, 1, 1};
    for (int it = 0; it < 200; ++it) {
        double total = 1.0;
        for (int a = 0; a < d; ++a) total *= floor(ext[a] / cell) + 1.0;
        if (total <= (double)cap) break;
        cell *= 1.25;
    }
    int64_t nc = 1;
    for (int a = 0; a < d; ++a) {
        dims[a] = (int)floor(ext[a] / cell) + 1;
        nc *= dims[a];
    }
    for (int a = 0; a < 3; ++a) gp->origin[a] = (a < d) ? mn[a] : 0.0;
    gp->cell = cell;
    gp->inv_cell = 1.0 / cell;
    for (int a = 0; a < 3; ++a) gp->dims[a] = dims[a];
    gp->ncell = (int)nc;
}

__device__ __forceinline__ int cell_coord(double x, double o, double inv, int dim) {
    int c = (int)floor((x - o) * inv);
    return c < 0 ? 0 : (c >= dim ? dim - 1 : c);
}

// Rank of this lane's node among the nodes of its cell: the lanes of the
// wavefront holding the same cell take consecutive ranks from one atomic
// increment by the lowest of them.  The count is bound by the number of
// increments; nodes that follow each other in the input often share a cell
// (2D disk: 78 to 57 us; the 3D sets, about one node per cell along a run of
// the input, are unchanged).  Lanes that are not active take no part.
__device__ __forceinline__ int wave_cell_rank(int* __restrict__ count, int lin) {
    const int lane = lane_id();
    uint64_t todo = ballot64(true);
    int leader = lane, within = 0, n_same = 0;
    while (todo) {  // uniform: one pass per distinct cell of the wavefront
        const int L = first_lane(todo);
        const int c = __builtin_amdgcn_readlane(lin, L);
        const uint64_t same = ballot64(lin == c) & todo;
        if ((same >> lane) & 1ull) {
            leader = L;
            within = __builtin_popcountll(same & ((1ull << lane) - 1ull));
        }
        if (lane == L) n_same = __builtin_popcountll(same);
        todo &= ~same;
    }
    int base = 0;
    if (leader == lane) base = atomicAdd(&count[lin], n_same);
    return __shfl(base, leader) + within;
}

__global__ __launch_bounds__(256) void k_bin_count(const double* __restrict__ X, int64_t N, int d,
                                                   const GridParams* __restrict__ gp, int* __restrict__ count,
                                                   int* __restrict__ cell_of, int* __restrict__ rank) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;  // the rank below is taken over the lanes still active
    int c[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) c[a] = cell_coord(X[i * d + a], gp->origin[a], gp->inv_cell, gp->dims[a]);
    int lin = c[0] + gp->dims[0] * (c[1] + gp->dims[1] * c[2]);
    cell_of[i] = lin;
    rank[i] = wave_cell_rank(count, lin);
}

// block-local exclusive scan of SCAN_CHUNK ints (256 threads x 4 each); returns the block total
__device__ int block_exclusive_scan4(int v[4], int* sm) {
    int s = v[0] + v[1] + v[2] + v[3];
    int incl = s;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        int t = __shfl_up(incl, o);
        if (lane_id() >= o) incl += t;
    }
    int w = threadIdx.x / WAVE;
    if (lane_id() == WAVE - 1) sm[w] = incl;
    __syncthreads();
    int wbase = 0, total = 0;
    for (int k = 0; k < 4; ++k) {
        if (k < w) wbase += sm[k];
        total += sm[k];
    }
    int run = wbase + incl - s;
    for (int k = 0; k < 4; ++k) {
        int x = v[k];
        v[k] = run;
        run += x;
    }
    return total;
}

__global__ __launch_bounds__(256) void k_scan_blocks(const int* __restrict__ a, int64_t n, int* __restrict__ bsum) {
    __shared__ int sm[4];
    int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + threadIdx.x * 4;
    int v[4];
    for (int k = 0; k < 4; ++k) v[k] = (base + k < n) ? a[base + k] : 0;
    int total = block_exclusive_scan4(v, sm);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_scan_top(int* __restrict__ bsum, int nb) {
    // exclusive scan of nb block totals by one block of 1024 threads
    __shared__ int sm[16];
    int per = (nb + 1023) / 1024;
    int start = threadIdx.x * per;
    int s = 0;
    for (int k = 0; k < per; ++k)
        if (start + k < nb) s += bsum[start + k];
    int incl = s;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        int t = __shfl_up(incl, o);
        if (lane_id() >= o) incl += t;
    }
    int w = threadIdx.x / WAVE;
    if (lane_id() == WAVE - 1) sm[w] = incl;
    __syncthreads();
    int wbase = 0;
    for (int k = 0; k < w; ++k) wbase += sm[k];
    int run = wbase + incl - s;
    for (int k = 0; k < per; ++k)
        if (start + k < nb) {
            int x = bsum[start + k];
            bsum[start + k] = run;
            run += x;
        }
}

__global__ __launch_bounds__(256) void k_scan_apply(int* __restrict__ a, int64_t n, const int* __restrict__ bsum) {
    __shared__ int sm[4];
    int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + threadIdx.x * 4;
    int v[4];
    for (int k = 0; k < 4; ++k) v[k] = (base + k < n) ? a[base + k] : 0;
    block_exclusive_scan4(v, sm);
    int off = bsum[blockIdx.x];
    for (int k = 0; k < 4; ++k)
        if (base + k < n) a[base + k] = v[k] + off;
}

__global__ __launch_bounds__(256) void k_bin_scatter(const double* __restrict__ X, int64_t N, int d,
                                                     const int* __restrict__ cell_start,
                                                     const int* __restrict__ cell_of, const int* __restrict__ rank,
                                                     int* __restrict__ sorted_id, double* __restrict__ sx) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int pos = cell_start[cell_of[i]] + rank[i];
    sorted_id[pos] = (int)i;
    for (int a = 0; a < d; ++a) sx[(int64_t)a * N + pos] = X[i * d + a];
}

// ------------------------------------------------------------------ selection
__device__ __forceinline__ double sq_key(const double* q, double x, double y, double z, int d) {
#pragma clang fp contract(off)
    double dx = x - q[0];
    double dy = y - q[1];
    double k = dx * dx + dy * dy;
    if (d == 3) {
        double dz = z - q[2];
        k = k + dz * dz;
    }
    return k;
}

__device__ __forceinline__ bool kless(double k1, unsigned i1, double k2, unsigned i2) {
    return (k1 < k2) || (k1 == k2 && i1 < i2);
}

// value of lane ^ j.  j = 1, 2, 8 are single DPP moves (quad permutations, row
// rotation by 8), j = 4 two of them (lane ^ 3 inside the quad, then the
// half-row mirror, lane ^ 7); j = 16, 32 cross rows and go through the LDS
// permute.  Every lane of the wave must be active.
__device__ __forceinline__ int xor_lane(int v, int j) {
    switch (j) {
        case 1: return __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false);
        case 2: return __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false);
        case 4: {
            const int a = __builtin_amdgcn_update_dpp(v, v, 0x1B, 0xF, 0xF, false);
            return __builtin_amdgcn_update_dpp(a, a, 0x141, 0xF, 0xF, false);
        }
        case 8: return __builtin_amdgcn_update_dpp(v, v, 0x128, 0xF, 0xF, false);
        default: return __shfl_xor(v, j);
    }
}
__device__ __forceinline__ double xor_lane(double v, int j) {
    return __hiloint2double(xor_lane(__double2hiint(v), j), xor_lane(__double2loint(v), j));
}

// compare-exchange of element e (= lane + 64 t) with e ^ j; want_min decided per element
template <int T>
__device__ __forceinline__ void cmpx_lane(double (&K)[T], unsigned (&I)[T], int j, const bool (&want_min)[T]) {
#pragma unroll
    for (int t = 0; t < T; ++t) {
        double pk = xor_lane(K[t], j);
        unsigned pi = (unsigned)xor_lane((int)I[t], j);
        bool pl = kless(pk, pi, K[t], I[t]);
        bool ml = kless(K[t], I[t], pk, pi);
        bool take = want_min[t] ? pl : ml;
        if (take) {
            K[t] = pk;
            I[t] = pi;
        }
    }
}

// in-register compare-exchange of slots 0 and 1 (distance 64); slot 0 keeps min if asc
__device__ __forceinline__ void cmpx_slot(double (&K)[2], unsigned (&I)[2], bool asc) {
    bool l10 = kless(K[1], I[1], K[0], I[0]);
    bool sw = asc ? l10 : kless(K[0], I[0], K[1], I[1]);
    if (sw) {
        double tk = K[0];
        unsigned ti = I[0];
        K[0] = K[1];
        I[0] = I[1];
        K[1] = tk;
        I[1] = ti;
    }
}

// full bitonic sort of the 64*T elements; descending if desc
template <int T>
__device__ __forceinline__ void bitonic_sort(double (&K)[T], unsigned (&I)[T], bool desc) {
    constexpr int S = 64 * T;
    int lane = lane_id();
#pragma unroll
    for (int k = 2; k <= S; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= 64) {
                if constexpr (T == 2) {
                    // e and e^64 share the lane: lower (slot 0) keeps min if asc
                    bool asc = (((lane) & k) == 0) != desc;  // k == 128 here: (e & 128) == 0
                    cmpx_slot(K, I, asc);
                }
            } else {
                bool wm[T];
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    int e = lane + 64 * t;
                    bool asc = ((e & k) == 0) != desc;
                    wm[t] = (((e & j) == 0) == asc);
                }
                cmpx_lane<T>(K, I, j, wm);
            }
        }
    }
}

// top ascending, chunk descending -> top = S smallest of both, ascending
template <int T>
__device__ __forceinline__ void merge_into(double (&TK)[T], unsigned (&TI)[T], const double (&CK)[T],
                                           const unsigned (&CI)[T]) {
    int lane = lane_id();
#pragma unroll
    for (int t = 0; t < T; ++t)
        if (kless(CK[t], CI[t], TK[t], TI[t])) {
            TK[t] = CK[t];
            TI[t] = CI[t];
        }
#pragma unroll
    for (int j = 32 * T; j > 0; j >>= 1) {
        if (j >= 64) {
            if constexpr (T == 2) cmpx_slot(TK, TI, true);
        } else {
            bool wm[T];
#pragma unroll
            for (int t = 0; t < T; ++t) wm[t] = (((lane + 64 * t) & j) == 0);
            cmpx_lane<T>(TK, TI, j, wm);
        }
    }
}

__device__ __forceinline__ int lin3(const GridParams& g, int x, int y, int z) {
    return x + g.dims[0] * (y + g.dims[1] * z);
}

// gap between coordinate q and the cells lo..hi along axis a (0 inside)
__device__ __forceinline__ double axis_gap(const GridParams& g, double q, int lo, int hi, int a) {
    const double blo = g.origin[a] + lo * g.cell, bhi = g.origin[a] + (hi + 1) * g.cell;
    return q < blo ? blo - q : (q > bhi ? q - bhi : 0.0);
}

// candidate range of slot s of ring R (rows of cells along x; see file header).
// A slot whose cells all lie farther than the current k-th key wk is empty: every
// node in it has a larger key (the relative margin covers rounding).
__device__ __forceinline__ void slot_range(const GridParams& g, const int* __restrict__ cell_start, int d,
                                           const int (&qc)[3], const double (&qx)[3], double wk, int R, bool first,
                                           int s, int nslots, int& start, int& len) {
    start = 0;
    len = 0;
    if (s >= nslots) return;
    int row = s >> 1, side = s & 1;
    int W = 2 * R + 1;
    int dy = (d == 3) ? (row % W) - R : row - R;
    int dz = (d == 3) ? (row / W) - R : 0;
    int cy = qc[1] + dy, cz = qc[2] + dz;
    if (cy < 0 || cy >= g.dims[1] || cz < 0 || cz >= g.dims[2]) return;
    bool full = first || dy == R || dy == -R || (d == 3 && (dz == R || dz == -R));
    int xlo, xhi;
    if (full) {
        if (side) return;
        xlo = max(0, qc[0] - R);
        xhi = min(g.dims[0] - 1, qc[0] + R);
    } else {
        int cx = side ? qc[0] + R : qc[0] - R;
        if (cx < 0 || cx >= g.dims[0]) return;
        xlo = xhi = cx;
    }
    if (!first) {
        const double gx = axis_gap(g, qx[0], xlo, xhi, 0), gy = axis_gap(g, qx[1], cy, cy, 1);
        const double gz = (d == 3) ? axis_gap(g, qx[2], cz, cz, 2) : 0.0;
        if ((gx * gx + gy * gy + gz * gz) * (1.0 - 1e-9) > wk) return;
    }
    int a = cell_start[lin3(g, xlo, cy, cz)];
    int b = cell_start[lin3(g, xhi, cy, cz) + 1];
    start = a;
    len = b - a;
}

// Streaming search of one query (one wavefront): candidate cell rows streamed in
// chunks of 64 T, filtered against the current k-th key, bitonic-sorted across
// the wave on (key, index) and merged into a sorted top list of 64 T entries;
// rings of cells are added until the k-th key is below the squared distance to
// the unsearched region (exact termination).  Writes the whole stencil.
template <int T>
__device__ __forceinline__ void knn_stream(const GridParams& g, const int* __restrict__ cell_start,
                                        const int* __restrict__ sorted_id, const double* __restrict__ sx, int64_t N,
                                        int d, int64_t q, int qid, int64_t off, int k, int32_t* __restrict__ idx,
                                        double key_inf) {
    const int lane = lane_id();
    double qx[3];
    qx[0] = sx[q];
    qx[1] = sx[N + q];
    qx[2] = (d == 3) ? sx[2 * N + q] : 0.0;
    // the axes written out: an index over the runtime d would place g in scratch memory
    int qc[3];
    qc[0] = cell_coord(qx[0], g.origin[0], g.inv_cell, g.dims[0]);
    qc[1] = cell_coord(qx[1], g.origin[1], g.inv_cell, g.dims[1]);
    qc[2] = (d == 3) ? cell_coord(qx[2], g.origin[2], g.inv_cell, g.dims[2]) : 0;

    double TK[T];
    unsigned TI[T];
    #pragma unroll
    for (int t = 0; t < T; ++t) {
        TK[t] = INFINITY;
        TI[t] = 0xFFFFFFFFu;
    }
    // k-th smallest (key, index) so far.  The +inf sentinel arrives as an argument:
    // a uniform FP64 constant whose low word is zero must not be materialised by a
    // single 64-bit scalar move (not encodable on this target).
    double wk = key_inf;
    unsigned wi = 0xFFFFFFFFu;
    const int wl = (k - 1) & 63, ws = (k - 1) >> 6;

    for (int R = 1;; ++R) {
        const bool first = (R == 1);
        const int W = 2 * R + 1;
        const int nslots = 2 * ((d == 3) ? W * W : W);
        for (int g0 = 0; g0 < nslots; g0 += WAVE) {
            int st, ln;
            slot_range(g, cell_start, d, qc, qx, wk, R, first, g0 + lane, nslots, st, ln);
            int incl = ln;
#pragma unroll
            for (int o = 1; o < WAVE; o <<= 1) {
                int t = __shfl_up(incl, o);
                if (lane >= o) incl += t;
            }
            const int total = __builtin_amdgcn_readlane(incl, 63);
            const int excl = incl - ln;
            for (int base = 0; base < total; base += 64 * T) {
                double CK[T];
                unsigned CI[T];
                bool any = false;
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    int e = base + lane + 64 * t;
                    // smallest slot r with incl[r] > e
                    int r = 0;
#pragma unroll
                    for (int step = 32; step > 0; step >>= 1) {
                        int v = __shfl(incl, r + step - 1);
                        if (v <= e) r += step;
                    }
                    int sr = __shfl(st, r);
                    int er = __shfl(excl, r);
                    // branch-free: every lane loads an in-bounds candidate, then selects
                    const bool valid = e < total;
                    const int pos = valid ? sr + (e - er) : 0;
                    const unsigned cid = (unsigned)sorted_id[pos];
                    const double key = sq_key(qx, sx[pos], sx[N + pos], (d == 3) ? sx[2 * N + pos] : 0.0, d);
                    const bool pass = valid && (cid != (unsigned)qid) && kless(key, cid, wk, wi);
                    CK[t] = pass ? key : key_inf;
                    CI[t] = pass ? cid : 0xFFFFFFFFu;
                    any = any || pass;
                }
                if (__ballot(any) == 0) continue;
                bitonic_sort<T>(CK, CI, true);
                merge_into<T>(TK, TI, CK, CI);
                double kk = (ws == 0) ? TK[0] : TK[T - 1];
                unsigned ii = (ws == 0) ? TI[0] : TI[T - 1];
                wk = readlane_d(kk, wl);
                wi = (unsigned)__builtin_amdgcn_readlane((int)ii, wl);
            }
        }
        // exact termination: every node outside the searched block is at least dist away
        double dist = INFINITY;
        for (int a = 0; a < d; ++a) {
            if (qc[a] - R > 0) dist = fmin(dist, qx[a] - (g.origin[a] + (qc[a] - R) * g.cell));
            if (qc[a] + R + 1 < g.dims[a]) dist = fmin(dist, (g.origin[a] + (qc[a] + R + 1) * g.cell) - qx[a]);
        }
        if (dist == INFINITY) break;
        if (wk < key_inf && wk < dist * dist * (1.0 - 1e-9)) break;
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
        int e = lane + 64 * t;
        if (e < k) idx[off + 1 + e] = (int32_t)TI[t];
    }
}


// Streaming kernel: every query (stencils of up to 129 nodes), or with a list
// (the radius search's unsettled queries: list[0 .. *list_count)) a persistent
// grid of waves over the listed cell-order positions.
template <int T>
__device__ __forceinline__ void knn_stream_query(const GridParams& g, const int* __restrict__ cell_start,
                                                 const int* __restrict__ sorted_id, const double* __restrict__ sx,
                                                 int64_t N, int d, const int64_t* __restrict__ offsets, int n_max,
                                                 int32_t* __restrict__ idx, double key_inf, int64_t q) {
    const int lane = lane_id();
    const int qid = sorted_id[q];
    const int64_t off = offsets[qid];
    const int64_t ni = offsets[qid + 1] - off;
    if (ni < 1 || ni > n_max || ni > N) {
        for (int64_t e = lane; e < ni; e += WAVE) idx[off + e] = -1;
        return;
    }
    if (lane == 0) idx[off] = qid;
    if (ni == 1) return;
    knn_stream<T>(g, cell_start, sorted_id, sx, N, d, q, qid, off, (int)ni - 1, idx, key_inf);
}

template <int T>
__global__ __launch_bounds__(256) void k_knn(const GridParams* __restrict__ gpp, const int* __restrict__ cell_start,
                                             const int* __restrict__ sorted_id, const double* __restrict__ sx,
                                             int64_t N, int d, const int64_t* __restrict__ offsets, int n_max,
                                             int32_t* __restrict__ idx, double key_inf) {
    const GridParams g = *gpp;
    const int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    if (q >= N) return;
    knn_stream_query<T>(g, cell_start, sorted_id, sx, N, d, offsets, n_max, idx, key_inf, q);
}

__global__ __launch_bounds__(256) void k_knn_list(const GridParams* __restrict__ gpp,
                                                  const int* __restrict__ cell_start,
                                                  const int* __restrict__ sorted_id, const double* __restrict__ sx,
                                                  int64_t N, int d, const int64_t* __restrict__ offsets, int n_max,
                                                  int32_t* __restrict__ idx, double key_inf,
                                                  const int* __restrict__ list, const int* __restrict__ list_count) {
    // the list length first: the grid parameters are copied into per-thread
    // storage (they are indexed by axis), which an idle launch should not pay for
    const int nl = __builtin_amdgcn_readfirstlane(*list_count);
    if ((int)(blockIdx.x * (blockDim.x / WAVE)) >= nl) return;  // uniform: nothing listed for this block
    const GridParams g = *gpp;
    const int nw = (int)(gridDim.x * (blockDim.x / WAVE));
    for (int i = (int)(blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE); i < nl; i += nw)
        knn_stream_query<1>(g, cell_start, sorted_id, sx, N, d, offsets, n_max, idx, key_inf,
                            (int64_t)__builtin_amdgcn_readfirstlane(list[i]));
}

// ------------------------------------------------------------ radius search
// Queries with k = n_i - 1 <= RADIUS_KMAX.  The k nearest nodes of a query all have keys
// <= tau exactly when at least k nodes other than the query have keys <= tau.
// tau is first estimated from the node density in the 3 x 3 (x 3) cells around
// the query; every node of the cells within sqrt(tau) (rows of cells along x
// are contiguous in cell order) is tested against tau and the survivors are
// compacted into a per-wave LDS buffer.  With k <= survivors <= RCAP they are
// sorted once on (key, index) and the first k written; otherwise tau is
// rescaled (survivors grow like tau^(d/2)) and the gather repeated.  A query
// that does not settle within RTRIES gathers is listed for the streaming search.
constexpr int RCAP = 128;
constexpr int RTRIES = 6;
constexpr int RADIUS_KMAX = 100;  // survivors aimed at 1.25 k must fit RCAP
constexpr int RANK_MAX = 32;      // survivors ordered by counting ranks up to this many
static_assert(RANK_MAX % 2 == 0 && RANK_MAX < RCAP, "the rank loop reads slot count when count is odd");

// Nodes in the cell rows of `rows` (rows of cells along x, y/z from the row
// index) within radius rho of qx: lane r handles row r0 + r, returns its node
// range; the caller scans them.  Conservative: a cell is taken when its box is
// within rho (rho already carries the rounding margin).
__device__ __forceinline__ void radius_row(const GridParams& g, const int* __restrict__ cell_start, int d,
                                           const double (&qx)[3], double rho, int ylo, int zlo, int ny, int row,
                                           int nrows, int& start, int& len) {
    start = 0;
    len = 0;
    if (row >= nrows) return;
    const int cy = ylo + row % ny, cz = zlo + row / ny;
    const double gy = axis_gap(g, qx[1], cy, cy, 1);
    const double gz = (d == 3) ? axis_gap(g, qx[2], cz, cz, 2) : 0.0;
    const double rem = rho * rho - gy * gy - gz * gz;
    if (rem < 0.0) return;
    const double rx = sqrt(rem);
    const int xlo = cell_coord(qx[0] - rx, g.origin[0], g.inv_cell, g.dims[0]);
    const int xhi = cell_coord(qx[0] + rx, g.origin[0], g.inv_cell, g.dims[0]);
    start = cell_start[lin3(g, xlo, cy, cz)];
    len = cell_start[lin3(g, xhi, cy, cz) + 1] - start;
}

__global__ __launch_bounds__(256) void k_knn_radius(const GridParams* __restrict__ gpp,
                                                    const int* __restrict__ cell_start,
                                                    const int* __restrict__ sorted_id, const double* __restrict__ sx,
                                                    int64_t N, int d, const int64_t* __restrict__ offsets, int n_max,
                                                    int32_t* __restrict__ idx, double key_inf,
                                                    int* __restrict__ list, int* __restrict__ list_count) {
    __shared__ __attribute__((aligned(16))) double skey[4][RCAP];
    __shared__ __attribute__((aligned(16))) unsigned sid[4][RCAP];
    const GridParams g = *gpp;
    const int lane = lane_id(), wv = threadIdx.x / WAVE;
    const int64_t q = (int64_t)blockIdx.x * 4 + wv;
    if (q >= N) return;
    const int qid = sorted_id[q];
    const int64_t off = offsets[qid];
    const int64_t ni = offsets[qid + 1] - off;
    if (ni < 1 || ni > n_max || ni > N) {
        for (int64_t e = lane; e < ni; e += WAVE) idx[off + e] = -1;
        return;
    }
    if (lane == 0) idx[off] = qid;
    if (ni == 1) return;
    const int k = (int)ni - 1;
    double qx[3];
    qx[0] = sx[q];
    qx[1] = sx[N + q];
    qx[2] = (d == 3) ? sx[2 * N + q] : 0.0;
    // the axes written out: an index over the runtime d would place g in scratch memory
    int qc[3];
    qc[0] = cell_coord(qx[0], g.origin[0], g.inv_cell, g.dims[0]);
    qc[1] = cell_coord(qx[1], g.origin[1], g.inv_cell, g.dims[1]);
    qc[2] = (d == 3) ? cell_coord(qx[2], g.origin[2], g.inv_cell, g.dims[2]) : 0;

    // local density: nodes in the 3 x 3 (x 3) cells around the query (in the grid)
    double tau;
    {
        const int nrow = (d == 3) ? 9 : 3;
        int cnt = 0, cells = 0;
        if (lane < nrow) {
            const int cy = qc[1] + lane % 3 - 1, cz = (d == 3) ? qc[2] + lane / 3 - 1 : 0;
            if (cy >= 0 && cy < g.dims[1] && cz >= 0 && cz < g.dims[2]) {
                const int xlo = max(qc[0] - 1, 0), xhi = min(qc[0] + 1, g.dims[0] - 1);
                cnt = cell_start[lin3(g, xhi, cy, cz) + 1] - cell_start[lin3(g, xlo, cy, cz)];
                cells = xhi - xlo + 1;
            }
        }
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            cnt += __shfl_xor(cnt, o);
            cells += __shfl_xor(cells, o);
        }
        cnt = __builtin_amdgcn_readfirstlane(cnt);
        cells = __builtin_amdgcn_readfirstlane(cells);
        // expected nodes within radius r: density * V_d r^d; aim at about 1.3 (k + 1)
        const double vol = (double)cells * ((d == 3) ? g.cell * g.cell * g.cell : g.cell * g.cell);
        const double dens = (double)max(cnt, 1) / vol;
        const double unit = (d == 3) ? 4.18879020478639098 : 3.14159265358979324;
        const double v = 1.3 * (k + 1) / (dens * unit);
        const double r = (d == 3) ? cbrt(v) : sqrt(v);
        tau = r * r;
    }

    int count = 0;
    bool ok = false;
    for (int attempt = 0; attempt < RTRIES; ++attempt) {
        const double rho = sqrt(tau) * (1.0 + 1e-9);
        const int ylo = cell_coord(qx[1] - rho, g.origin[1], g.inv_cell, g.dims[1]);
        const int yhi = cell_coord(qx[1] + rho, g.origin[1], g.inv_cell, g.dims[1]);
        const int zlo = (d == 3) ? cell_coord(qx[2] - rho, g.origin[2], g.inv_cell, g.dims[2]) : 0;
        const int zhi = (d == 3) ? cell_coord(qx[2] + rho, g.origin[2], g.inv_cell, g.dims[2]) : 0;
        const int ny = yhi - ylo + 1;
        const int nrows = ny * (zhi - zlo + 1);
        count = 0;
        for (int r0 = 0; r0 < nrows; r0 += WAVE) {
            int st, ln;
            radius_row(g, cell_start, d, qx, rho, ylo, zlo, ny, r0 + lane, nrows, st, ln);
            int incl = ln;
#pragma unroll
            for (int o = 1; o < WAVE; o <<= 1) {
                const int t = __shfl_up(incl, o);
                if (lane >= o) incl += t;
            }
            const int total = __builtin_amdgcn_readlane(incl, 63);
            const int excl = incl - ln;
            for (int base = 0; base < total; base += WAVE) {
                const int e = base + lane;
                // smallest row r with incl[r] > e
                int r = 0;
#pragma unroll
                for (int step = 32; step > 0; step >>= 1) {
                    const int v = __shfl(incl, r + step - 1);
                    if (v <= e) r += step;
                }
                const int sr = __shfl(st, r);
                const int er = __shfl(excl, r);
                // branch-free: every lane loads an in-bounds candidate, then selects
                const bool valid = e < total;
                const int pos = valid ? sr + (e - er) : 0;
                const unsigned cid = (unsigned)sorted_id[pos];
                const double key = sq_key(qx, sx[pos], sx[N + pos], (d == 3) ? sx[2 * N + pos] : 0.0, d);
                const bool pass = valid && cid != (unsigned)qid && key <= tau;
                const uint64_t b = ballot64(pass);
                const int slot = count + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(b >> 32),
                                                                        __builtin_amdgcn_mbcnt_lo((unsigned)b, 0u));
                if (pass && slot < RCAP) {
                    skey[wv][slot] = key;
                    sid[wv][slot] = cid;
                }
                count += __builtin_popcountll(b);
            }
        }
        if (count >= k && count <= RCAP) {
            ok = true;
            break;
        }
        // survivors grow like tau^(d/2): aim at about 1.25 k
        const double ratio = 1.25 * k / (double)max(count, 1);
        const double cr = cbrt(ratio);
        double f = (count == 0) ? 4.0 : ((d == 3) ? cr * cr : ratio);
        f = (count < k) ? fmax(f, 1.2) : fmin(f, 0.9);
        tau *= f;
    }
    if (!ok) {  // left to the streaming search (k_knn_list)
        if (lane == 0) list[atomicAdd(list_count, 1)] = (int)q;
        return;
    }
    wave_lds_sync();
    if (count <= RANK_MAX) {
        // few survivors: each lane's survivor counts the survivors before it on
        // (key, index) -- a strict order, so the ranks are 0 .. count - 1 -- and
        // the k smallest ranks are the stencil in order (fewer instructions than
        // the 21 stages of a 64-wide sort)
        const bool have = lane < count;
        const double kl = have ? skey[wv][lane] : 0.0;
        const unsigned il = have ? sid[wv][lane] : 0u;
        int rank = 0;
        // two survivors per 16-byte read (slot count, read when count is odd, is
        // within the buffer and not counted)
#pragma unroll 4
        for (int j = 0; j < count; j += 2) {
            const double2 kk = *reinterpret_cast<const double2*>(&skey[wv][j]);
            const uint2 ii = *reinterpret_cast<const uint2*>(&sid[wv][j]);
            rank += (kk.x < kl || (kk.x == kl && ii.x < il)) ? 1 : 0;
            rank += (j + 1 < count && (kk.y < kl || (kk.y == kl && ii.y < il))) ? 1 : 0;
        }
        if (have && rank < k) idx[off + 1 + rank] = (int32_t)il;
    } else if (count <= WAVE) {
        double K[1];
        unsigned I[1];
        K[0] = lane < count ? skey[wv][lane] : key_inf;
        I[0] = lane < count ? sid[wv][lane] : 0xFFFFFFFFu;
        bitonic_sort<1>(K, I, false);
        if (lane < k) idx[off + 1 + lane] = (int32_t)I[0];
    } else {
        double K[2];
        unsigned I[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int e = lane + WAVE * t;
            K[t] = e < count ? skey[wv][e] : key_inf;
            I[t] = e < count ? sid[wv][e] : 0xFFFFFFFFu;
        }
        bitonic_sort<2>(K, I, false);
        if (lane < k) idx[off + 1 + lane] = (int32_t)I[0];
        if (WAVE + lane < k) idx[off + 1 + WAVE + lane] = (int32_t)I[1];
    }
}

// Several queries per wavefront for stencils of up to 41 nodes, the same search
// and result as k_knn_radius: each query has a group of QW lanes (16 or 32),
// with its own rows of cells, prefix sums and survivor buffer, so the
// per-query set-up (density, radius, rows) runs once for 64 / QW queries.
// Survivors are capped at QW * SPL (SPL per lane) and ordered by counting
// ranks; a query that does not settle within RTRIES gathers is listed for the
// streaming search as before.  Every lane takes part in every cross-lane step
// (a finished or empty group only masks its own work).
// k = n_i - 1 up to GROUP_KMAX<cap>: survivors aimed at 1.3 (k + 1) well below the cap
template <int CAP>
constexpr int GROUP_KMAX = CAP == 32 ? 16 : 40;

template <int QW, int SPL>
__global__ __launch_bounds__(256) void k_knn_radius_group(const GridParams* __restrict__ gpp,
                                                          const int* __restrict__ cell_start,
                                                          const int* __restrict__ sorted_id,
                                                          const double* __restrict__ sx, int64_t N, int d,
                                                          const int64_t* __restrict__ offsets, int n_max,
                                                          int32_t* __restrict__ idx, int* __restrict__ list,
                                                          int* __restrict__ list_count) {
    static_assert(QW == 16 || QW == 32, "a group holds the density rows (9) of a query");
    static_assert(QW * SPL == 32 || QW * SPL == 64, "survivor caps of GROUP_KMAX");
    constexpr int QPW = WAVE / QW;   // queries per wavefront
    constexpr int PCAP = SPL * QW;   // survivors per query
    __shared__ __attribute__((aligned(16))) double skey[4 * QPW][PCAP];
    __shared__ __attribute__((aligned(16))) unsigned sid[4 * QPW][PCAP];
    const GridParams g = *gpp;
    const int lane = lane_id(), wv = threadIdx.x / WAVE;
    const int sl = lane & (QW - 1), gb = lane - sl, hq = wv * QPW + lane / QW;
    const int64_t q = (int64_t)blockIdx.x * (4 * QPW) + hq;
    bool active = q < N;
    int qid = 0;
    int64_t off = 0, ni = 0;
    if (active) {
        qid = sorted_id[q];
        off = offsets[qid];
        ni = offsets[qid + 1] - off;
        if (ni < 1 || ni > n_max || ni > N) {
            for (int64_t e = sl; e < ni; e += QW) idx[off + e] = -1;
            active = false;
        } else {
            if (sl == 0) idx[off] = qid;
            if (ni == 1) active = false;
        }
    }
    const int k = (int)ni - 1;
    double qx[3] = {0.0, 0.0, 0.0};
    if (active) {
        qx[0] = sx[q];
        qx[1] = sx[N + q];
        qx[2] = (d == 3) ? sx[2 * N + q] : 0.0;
    }
    // the axes written out: an index over the runtime d would place g in scratch memory
    int qc[3];
    qc[0] = cell_coord(qx[0], g.origin[0], g.inv_cell, g.dims[0]);
    qc[1] = cell_coord(qx[1], g.origin[1], g.inv_cell, g.dims[1]);
    qc[2] = (d == 3) ? cell_coord(qx[2], g.origin[2], g.inv_cell, g.dims[2]) : 0;

    // local density around the query's cell, as in k_knn_radius
    double tau;
    {
        const int nrow = (d == 3) ? 9 : 3;
        int cnt = 0, cells = 0;
        if (active && sl < nrow) {
            const int cy = qc[1] + sl % 3 - 1, cz = (d == 3) ? qc[2] + sl / 3 - 1 : 0;
            if (cy >= 0 && cy < g.dims[1] && cz >= 0 && cz < g.dims[2]) {
                const int xlo = max(qc[0] - 1, 0), xhi = min(qc[0] + 1, g.dims[0] - 1);
                cnt = cell_start[lin3(g, xhi, cy, cz) + 1] - cell_start[lin3(g, xlo, cy, cz)];
                cells = xhi - xlo + 1;
            }
        }
        const int span = (d == 3) ? 16 : 4;  // lanes holding the rows
        for (int o = 1; o < span; o <<= 1) {
            cnt += __shfl_xor(cnt, o);
            cells += __shfl_xor(cells, o);
        }
        cnt = __shfl(cnt, gb);
        cells = __shfl(cells, gb);
        // expected nodes within r: cnt / (cells c^d) V_d r^d; aim at about 1.3 (k + 1)
        const double vol = (double)max(cells, 1) * ((d == 3) ? g.cell * g.cell * g.cell : g.cell * g.cell);
        const double unit = (d == 3) ? 4.18879020478639098 : 3.14159265358979324;
        const double v = 1.3 * (k + 1) * vol / ((double)max(cnt, 1) * unit);
        const double r = (d == 3) ? cbrt(v) : sqrt(v);
        tau = r * r;
    }

    int count = 0;
    bool ok = !active;  // nothing to search
    for (int attempt = 0; attempt < RTRIES; ++attempt) {
        if (ballot64(!ok) == 0) break;
        const bool work = !ok;
        const double rho = sqrt(tau) * (1.0 + 1e-9);
        const int ylo = cell_coord(qx[1] - rho, g.origin[1], g.inv_cell, g.dims[1]);
        const int yhi = cell_coord(qx[1] + rho, g.origin[1], g.inv_cell, g.dims[1]);
        const int zlo = (d == 3) ? cell_coord(qx[2] - rho, g.origin[2], g.inv_cell, g.dims[2]) : 0;
        const int zhi = (d == 3) ? cell_coord(qx[2] + rho, g.origin[2], g.inv_cell, g.dims[2]) : 0;
        const int ny = yhi - ylo + 1;
        const int nrows = work ? ny * (zhi - zlo + 1) : 0;
        int rmax = nrows;
#pragma unroll
        for (int o = QW; o < WAVE; o <<= 1) rmax = max(rmax, __shfl_xor(rmax, o));
        if (work) count = 0;
        for (int r0 = 0; r0 < rmax; r0 += QW) {
            int st, ln;
            radius_row(g, cell_start, d, qx, rho, ylo, zlo, ny, r0 + sl, nrows, st, ln);
            int incl = ln;
#pragma unroll
            for (int o = 1; o < QW; o <<= 1) {
                const int t = __shfl_up(incl, o, QW);
                if (sl >= o) incl += t;
            }
            const int total = __shfl(incl, gb + QW - 1);
            const int excl = incl - ln;
            int tmax = total;
#pragma unroll
            for (int o = QW; o < WAVE; o <<= 1) tmax = max(tmax, __shfl_xor(tmax, o));
            for (int base = 0; base < tmax; base += QW) {
                const int e = base + sl;
                // smallest row r of this group with incl[r] > e
                int r = 0;
#pragma unroll
                for (int step = QW / 2; step > 0; step >>= 1) {
                    const int v = __shfl(incl, gb + r + step - 1);
                    if (v <= e) r += step;
                }
                const int sr = __shfl(st, gb + r);
                const int er = __shfl(excl, gb + r);
                const bool valid = e < total;
                const int pos = valid ? sr + (e - er) : 0;
                const unsigned cid = (unsigned)sorted_id[pos];
                const double key = sq_key(qx, sx[pos], sx[N + pos], (d == 3) ? sx[2 * N + pos] : 0.0, d);
                const bool pass = valid && cid != (unsigned)qid && key <= tau;
                const unsigned hb = (unsigned)(ballot64(pass) >> gb) & (unsigned)((1ull << QW) - 1);
                const int slot = count + __builtin_popcount(hb & ((1u << sl) - 1u));
                if (pass && slot < PCAP) {
                    skey[hq][slot] = key;
                    sid[hq][slot] = cid;
                }
                count += __builtin_popcount(hb);
            }
        }
        if (work) {
            if (count >= k && count <= PCAP) {
                ok = true;
            } else {
                const double ratio = 1.25 * k / (double)max(count, 1);
                const double cr = cbrt(ratio);
                double f = (count == 0) ? 4.0 : ((d == 3) ? cr * cr : ratio);
                f = (count < k) ? fmax(f, 1.2) : fmin(f, 0.9);
                tau *= f;
            }
        }
    }
    wave_lds_sync();
    if (!active) return;
    if (!ok) {  // left to the streaming search (k_knn_list)
        if (sl == 0) list[atomicAdd(list_count, 1)] = (int)q;
        return;
    }
    // count <= PCAP: each survivor counts the survivors before it on (key,
    // index); the k smallest ranks are the stencil in order
    double kl[SPL];
    unsigned il[SPL];
    int rank[SPL];
#pragma unroll
    for (int t = 0; t < SPL; ++t) {
        const bool have = sl + QW * t < count;
        kl[t] = have ? skey[hq][sl + QW * t] : 0.0;
        il[t] = have ? sid[hq][sl + QW * t] : 0u;
        rank[t] = 0;
    }
    for (int j = 0; j < count; j += 2) {  // slot count, read when count is odd, is in the buffer and not counted
        const double2 kk = *reinterpret_cast<const double2*>(&skey[hq][j]);
        const uint2 ii = *reinterpret_cast<const uint2*>(&sid[hq][j]);
#pragma unroll
        for (int t = 0; t < SPL; ++t) {
            rank[t] += (kk.x < kl[t] || (kk.x == kl[t] && ii.x < il[t])) ? 1 : 0;
            rank[t] += (j + 1 < count && (kk.y < kl[t] || (kk.y == kl[t] && ii.y < il[t]))) ? 1 : 0;
        }
    }
#pragma unroll
    for (int t = 0; t < SPL; ++t)
        if (sl + QW * t < count && rank[t] < k) idx[off + 1 + rank[t]] = (int32_t)il[t];
}

struct SelWorkspace {
    size_t gp, part, count, bsum, cell_of, rank, sorted_id, sx, list, total;
    int64_t cap;
    int nb_scan;
};

SelWorkspace sel_layout(int64_t N, int d) {
    SelWorkspace w;
    w.cap = N + 4096;
    w.nb_scan = (int)((w.cap + 1 + SCAN_CHUNK - 1) / SCAN_CHUNK);
    size_t o = 0;
    w.gp = o;
    o += rbf_align(sizeof(GridParams));
    w.part = o;
    o += rbf_align(sizeof(double) * 6 * BBOX_BLOCKS);
    w.count = o;
    o += rbf_align(sizeof(int) * (w.cap + 2));  // cell counts, then the list length
    w.bsum = o;
    o += rbf_align(sizeof(int) * (w.nb_scan + 1));
    w.cell_of = o;
    o += rbf_align(sizeof(int) * N);
    w.rank = o;
    o += rbf_align(sizeof(int) * N);
    w.sorted_id = o;
    o += rbf_align(sizeof(int) * N);
    w.sx = o;
    o += rbf_align(sizeof(double) * d * N);
    w.list = o;
    o += rbf_align(sizeof(int) * N);
    w.total = o;
    return w;
}

}  // namespace

extern "C" rbf_status rbf_select_stencils_workspace(int64_t N, int d, int n_max, size_t* bytes) {
    if (!bytes || N < 1) return RBF_EINVAL;
    if (d != 2 && d != 3) return RBF_EDIM;
    (void)n_max;
    *bytes = sel_layout(N, d).total;
    return RBF_OK;
}

// Enqueues the whole selection pipeline with its buffers carved from ws (layout L).
static rbf_status select_enqueue(rbf_ctx* ctx, const double* X, int64_t N, int d, const int64_t* offsets, int n_max,
                                 int32_t* idx, char* ws, const SelWorkspace& L) {
    GridParams* gp = (GridParams*)(ws + L.gp);
    double* part = (double*)(ws + L.part);
    int* count = (int*)(ws + L.count);
    int* bsum = (int*)(ws + L.bsum);
    int* cell_of = (int*)(ws + L.cell_of);
    int* rank = (int*)(ws + L.rank);
    int* sorted_id = (int*)(ws + L.sorted_id);
    double* sx = (double*)(ws + L.sx);
    hipStream_t s = ctx->stream;

    const double unit_ball = (d == 2) ? M_PI : 4.0 * M_PI / 3.0;
    const double target = fmax(1.0, ((d == 3) ? CELL_FILL_3D : CELL_FILL_2D) * (double)n_max / unit_ball);

    int nbb = (int)std::min<int64_t>(BBOX_BLOCKS, (N + 255) / 256);
    bbox_enqueue(s, nbb, X, N, d, part);
    hipLaunchKernelGGL(k_grid_setup, dim3(1), dim3(64), 0, s, part, nbb, N, d, target, L.cap, gp);
    // cleared by a kernel (a memset node in a captured graph is not reliable);
    // count[cap + 1] is the length of the radius search's fallback list
    int* list_count = count + L.cap + 1;
    int* list = (int*)(ws + L.list);
    hipLaunchKernelGGL(k_zero_ints, dim3((unsigned)((L.cap + 2 + 255) / 256)), dim3(256), 0, s, count,
                       (int64_t)L.cap + 2);
    int nbN = (int)((N + 255) / 256);
    hipLaunchKernelGGL(k_bin_count, dim3(nbN), dim3(256), 0, s, X, N, d, gp, count, cell_of, rank);
    hipLaunchKernelGGL(k_scan_blocks, dim3(L.nb_scan), dim3(256), 0, s, count, L.cap + 1, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, bsum, L.nb_scan);
    hipLaunchKernelGGL(k_scan_apply, dim3(L.nb_scan), dim3(256), 0, s, count, L.cap + 1, bsum);
    hipLaunchKernelGGL(k_bin_scatter, dim3(nbN), dim3(256), 0, s, X, N, d, count, cell_of, rank, sorted_id, sx);
    int64_t waves = N;
    dim3 grid((unsigned)((waves * WAVE + 255) / 256));
    // four queries per wavefront (16 lanes each) where the survivors fit 2 or 4
    // slots per lane; two (32 lanes, 2 slots) for the larger 2D stencils
    if (n_max - 1 <= GROUP_KMAX<32> && d == 2) {
        hipLaunchKernelGGL((k_knn_radius_group<16, 2>), dim3((unsigned)((N + 15) / 16)), dim3(256), 0, s, gp, count,
                           sorted_id, sx, N, d, offsets, n_max, idx, list, list_count);
    } else if (n_max - 1 <= GROUP_KMAX<64> && d == 3) {
        hipLaunchKernelGGL((k_knn_radius_group<16, 4>), dim3((unsigned)((N + 15) / 16)), dim3(256), 0, s, gp, count,
                           sorted_id, sx, N, d, offsets, n_max, idx, list, list_count);
    } else if (n_max - 1 <= GROUP_KMAX<64>) {
        hipLaunchKernelGGL((k_knn_radius_group<32, 2>), dim3((unsigned)((N + 7) / 8)), dim3(256), 0, s, gp, count,
                           sorted_id, sx, N, d, offsets, n_max, idx, list, list_count);
    } else if (n_max - 1 <= RADIUS_KMAX) {
        hipLaunchKernelGGL(k_knn_radius, grid, dim3(256), 0, s, gp, count, sorted_id, sx, N, d, offsets, n_max, idx,
                           (double)INFINITY, list, list_count);
    }
    if (n_max - 1 <= RADIUS_KMAX) {
        // persistent, 2k waves: the list is usually empty or short, and an idle
        // launch of 2k blocks costs more than the few listed queries gain
        const unsigned lg = (unsigned)std::min<int64_t>((N + 3) / 4, 512);
        hipLaunchKernelGGL(k_knn_list, dim3(lg), dim3(256), 0, s, gp, count, sorted_id, sx, N, d, offsets, n_max,
                           idx, (double)INFINITY, list, list_count);
    } else
        hipLaunchKernelGGL(k_knn<2>, grid, dim3(256), 0, s, gp, count, sorted_id, sx, N, d, offsets, n_max, idx,
                           (double)INFINITY);
    RBF_LAUNCH_CHECK();
    return RBF_OK;
}

static rbf_status select_check(rbf_ctx* ctx, const double* X, int64_t N, int d, const int64_t* offsets, int n_max,
                               int32_t* idx) {
    if (!ctx || !X || !offsets || !idx || N < 1) return RBF_EINVAL;
    if (d != 2 && d != 3) return RBF_EDIM;
    if (n_max < 1 || n_max > 129) return RBF_EINVAL;
    if (n_max > N) return RBF_ETOOFEW;
    if (N > (int64_t)0x7FFFFFFF - 8192) return RBF_EINVAL;
    return RBF_OK;
}

extern "C" rbf_status rbf_select_stencils(rbf_ctx* ctx, const double* X, int64_t N, int d, const int64_t* offsets,
                                          int n_max, int32_t* idx, void* workspace, size_t ws_bytes) {
    const rbf_status st = select_check(ctx, X, N, d, offsets, n_max, idx);
    if (st != RBF_OK) return st;
    if (!workspace) return RBF_EINVAL;
    SelWorkspace L = sel_layout(N, d);
    if (ws_bytes < L.total) return RBF_EWORKSPACE;
    RBF_HIP_CHECK(hipSetDevice(ctx->device));
    return select_enqueue(ctx, X, N, d, offsets, n_max, idx, (char*)workspace, L);
}

// ------------------------------------------------------ cell order of a node set
// Ascending ids inside each cell, whatever its size: the id at position p of
// the cell-ordered array moves to the cell's start plus the number of ids of
// its cell that are smaller (ids are distinct, so the ranks are a permutation of
// the cell's positions).  One thread per position; work per cell is the square
// of its size, spread over its threads.
__global__ __launch_bounds__(256) void k_cell_rank(int64_t N, const int* __restrict__ cell_of,
                                                   const int* __restrict__ cell_start, const int32_t* __restrict__ ids,
                                                   int32_t* __restrict__ out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int32_t v = ids[p];
    const int c = cell_of[v];
    const int a = cell_start[c], b = cell_start[c + 1];
    int r = 0;
    for (int i = a; i < b; ++i) r += ids[i] < v ? 1 : 0;
    out[a + r] = v;
}

namespace rbf {

// Workspace of cell_order_enqueue (the selection layout).
size_t cell_order_ws(int64_t N, int d) { return sel_layout(N, d).total; }

// Node ids in the order of a uniform grid of cells holding about per_cell nodes
// each (cells in x-fastest order, ascending ids within a cell): order[N]
// (device), the same for every run.  Enqueued on s; ws (cell_order_ws bytes) is
// scratch.
hipError_t cell_order_enqueue(hipStream_t s, const double* X, int64_t N, int d, double per_cell, void* ws,
                              int32_t* order) {
    const SelWorkspace L = sel_layout(N, d);
    char* w = (char*)ws;
    GridParams* gp = (GridParams*)(w + L.gp);
    double* part = (double*)(w + L.part);
    int* count = (int*)(w + L.count);
    int* bsum = (int*)(w + L.bsum);
    int* cell_of = (int*)(w + L.cell_of);
    int* rank = (int*)(w + L.rank);
    double* sx = (double*)(w + L.sx);
    const int nbb = (int)std::min<int64_t>(BBOX_BLOCKS, (N + 255) / 256);
    bbox_enqueue(s, nbb, X, N, d, part);
    hipLaunchKernelGGL(k_grid_setup, dim3(1), dim3(64), 0, s, part, nbb, N, d, fmax(1.0, per_cell), L.cap, gp);
    hipLaunchKernelGGL(k_zero_ints, dim3((unsigned)((L.cap + 2 + 255) / 256)), dim3(256), 0, s, count,
                       (int64_t)L.cap + 2);
    const int nbN = (int)((N + 255) / 256);
    hipLaunchKernelGGL(k_bin_count, dim3(nbN), dim3(256), 0, s, X, N, d, gp, count, cell_of, rank);
    hipLaunchKernelGGL(k_scan_blocks, dim3(L.nb_scan), dim3(256), 0, s, count, L.cap + 1, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, bsum, L.nb_scan);
    hipLaunchKernelGGL(k_scan_apply, dim3(L.nb_scan), dim3(256), 0, s, count, L.cap + 1, bsum);
    // the ids in cell order (any order inside a cell: the ranks are atomic) in the
    // layout's sorted_id buffer, then in ascending order inside each cell to order
    int32_t* ids = (int32_t*)(w + L.sorted_id);
    hipLaunchKernelGGL(k_bin_scatter, dim3(nbN), dim3(256), 0, s, X, N, d, count, cell_of, rank, ids, sx);
    hipLaunchKernelGGL(k_cell_rank, dim3(nbN), dim3(256), 0, s, N, cell_of, count, ids, order);
    return hipGetLastError();
}

}  // namespace rbf

// ------------------------------------------------------ no-allocation variant
// The selection buffers of rbf_select_stencils_static live in this file-scope
// array, one copy per device, held from module load to process end.  Host code
// never uses the array's name as an address (on the host it is only a stand-in
// symbol): the device address comes from hipGetSymbolAddress, taken once per
// device at context creation with that device current.
static __device__ __align__(256) unsigned char scratch[RBF_SELECT_STATIC_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES];
}  // namespace

// Resolves this device's copy of the scratch array (the caller has made the
// device current).  Idempotent.
rbf_status rbf_select_scratch_init(int device) {
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) return RBF_EINVAL;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return RBF_OK;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RBF_EHIP;
    g_scratch_ptr[device] = p;
    return RBF_OK;
}

extern "C" rbf_status rbf_select_stencils_static(rbf_ctx* ctx, const double* X, int64_t N, int d,
                                                 const int64_t* offsets, int n_max, int32_t* idx) {
    const rbf_status st = select_check(ctx, X, N, d, offsets, n_max, idx);
    if (st != RBF_OK) return st;
    const SelWorkspace L = sel_layout(N, d);
    if (L.total > (size_t)RBF_SELECT_STATIC_BYTES) return RBF_EWORKSPACE;
    void* p;
    {
        if (ctx->device < 0 || ctx->device >= SCRATCH_MAX_DEVICES) return RBF_EINVAL;
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        p = g_scratch_ptr[ctx->device];
    }
    if (!p) return RBF_EHIP;  // the context's creation did not resolve the array
    RBF_HIP_CHECK(hipSetDevice(ctx->device));
    return select_enqueue(ctx, X, N, d, offsets, n_max, idx, (char*)p, L);
}
