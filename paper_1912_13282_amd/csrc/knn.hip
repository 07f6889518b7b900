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
//   k_knn<T>                      : one wavefront per query node; candidates of
//       the surrounding cells are streamed in chunks of 64*T, bitonic-sorted
//       across the wave on (key, index) and merged into a sorted top list of
//       64*T entries; rings of cells are added until the k-th key is below the
//       squared distance to the unsearched region (exact termination).
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
// mean nodes per cell relative to n_max / (unit-ball volume), i.e. the cell side
// relative to the stencil radius (measured: 2D is fastest at about one stencil
// radius per cell, 3D at half the volume, which cuts the 27-cell candidate set)
constexpr double CELL_FILL_2D = 1.0;
constexpr double CELL_FILL_3D = 0.5;
constexpr int SCAN_CHUNK = 1024;  // elements per scan block (256 threads x 4)

__global__ __launch_bounds__(256) void k_zero_ints(int* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ __launch_bounds__(256) void k_bbox_partial(const double* __restrict__ X, int64_t N, int d,
                                                      double* __restrict__ part) {
    __shared__ double sm[4][6];
    double mn[3] = {INFINITY, INFINITY, INFINITY};
    double mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        for (int a = 0; a < d; ++a) {
            double v = X[i * d + a];
            mn[a] = fmin(mn[a], v);
            mx[a] = fmax(mx[a], v);
        }
    }
    for (int a = 0; a < 3; ++a) {
        mn[a] = wave_min_d(mn[a]);
        mx[a] = wave_max_d(mx[a]);
    }
    int w = threadIdx.x / WAVE;
    if (lane_id() == 0)
        for (int a = 0; a < 3; ++a) {
            sm[w][a] = mn[a];
            sm[w][3 + a] = mx[a];
        }
    __syncthreads();
    if (threadIdx.x < 6) {
        int a = threadIdx.x;
        double v = sm[0][a];
        for (int k = 1; k < 4; ++k) v = (a < 3) ? fmin(v, sm[k][a]) : fmax(v, sm[k][a]);
        part[blockIdx.x * 6 + a] = v;
    }
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

__global__ __launch_bounds__(256) void k_bin_count(const double* __restrict__ X, int64_t N, int d,
                                                   const GridParams* __restrict__ gp, int* __restrict__ count,
                                                   int* __restrict__ cell_of, int* __restrict__ rank) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int c[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) c[a] = cell_coord(X[i * d + a], gp->origin[a], gp->inv_cell, gp->dims[a]);
    int lin = c[0] + gp->dims[0] * (c[1] + gp->dims[1] * c[2]);
    cell_of[i] = lin;
    rank[i] = atomicAdd(&count[lin], 1);
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

template <int T>
__global__ __launch_bounds__(256) void k_knn(const GridParams* __restrict__ gpp, const int* __restrict__ cell_start,
                                             const int* __restrict__ sorted_id, const double* __restrict__ sx,
                                             int64_t N, int d, const int64_t* __restrict__ offsets, int n_max,
                                             int32_t* __restrict__ idx, double key_inf) {
    const GridParams g = *gpp;
    int lane = lane_id();
    int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    if (q >= N) return;
    const int qid = sorted_id[q];
    const int64_t off = offsets[qid];
    const int64_t ni = offsets[qid + 1] - off;
    if (ni < 1 || ni > n_max || ni > N) {
        for (int64_t e = lane; e < ni; e += WAVE) idx[off + e] = -1;
        return;
    }
    if (lane == 0) idx[off] = qid;
    const int k = (int)ni - 1;
    if (k == 0) return;

    double qx[3];
    qx[0] = sx[q];
    qx[1] = sx[N + q];
    qx[2] = (d == 3) ? sx[2 * N + q] : 0.0;
    int qc[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) qc[a] = cell_coord(qx[a], g.origin[a], g.inv_cell, g.dims[a]);

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

struct SelWorkspace {
    size_t gp, part, count, bsum, cell_of, rank, sorted_id, sx, total;
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
    o += rbf_align(sizeof(int) * (w.cap + 1));
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
    hipLaunchKernelGGL(k_bbox_partial, dim3(nbb), dim3(256), 0, s, X, N, d, part);
    hipLaunchKernelGGL(k_grid_setup, dim3(1), dim3(64), 0, s, part, nbb, N, d, target, L.cap, gp);
    // cleared by a kernel (a memset node in a captured graph is not reliable)
    hipLaunchKernelGGL(k_zero_ints, dim3((unsigned)((L.cap + 1 + 255) / 256)), dim3(256), 0, s, count,
                       (int64_t)L.cap + 1);
    int nbN = (int)((N + 255) / 256);
    hipLaunchKernelGGL(k_bin_count, dim3(nbN), dim3(256), 0, s, X, N, d, gp, count, cell_of, rank);
    hipLaunchKernelGGL(k_scan_blocks, dim3(L.nb_scan), dim3(256), 0, s, count, L.cap + 1, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, bsum, L.nb_scan);
    hipLaunchKernelGGL(k_scan_apply, dim3(L.nb_scan), dim3(256), 0, s, count, L.cap + 1, bsum);
    hipLaunchKernelGGL(k_bin_scatter, dim3(nbN), dim3(256), 0, s, X, N, d, count, cell_of, rank, sorted_id, sx);
    int64_t waves = N;
    dim3 grid((unsigned)((waves * WAVE + 255) / 256));
    if (n_max - 1 <= 64)
        hipLaunchKernelGGL(k_knn<1>, grid, dim3(256), 0, s, gp, count, sorted_id, sx, N, d, offsets, n_max, idx,
                           (double)INFINITY);
    else
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
