// CSR form of the operator matrix (Sec. 2.3.2): row i holds node i's stencil
// weights at the stencil columns, columns ascending, at most sum n_i nonzeros.
//
// One group of G lanes sorts one row: E elements per lane (G*E >= n_i),
// bitonic network on the column index carrying the stencil position, then the
// columns are written and every operator's weights gathered by that position.
// The pass is bandwidth-bound: it reads idx and w once and writes col and vals once.
#include "common.hpp"

namespace {

__global__ __launch_bounds__(256) void k_copy_rowptr(const int64_t* __restrict__ off, int64_t* __restrict__ rp,
                                                     int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) rp[i] = off[i];
}

template <int G, int E>
__global__ __launch_bounds__(256) void k_csr_rows(int64_t N, const int64_t* __restrict__ offsets,
                                                  const int32_t* __restrict__ idx, const double* __restrict__ w,
                                                  int n_ops, int64_t nnz, int n_max, int32_t* __restrict__ col,
                                                  double* __restrict__ vals) {
    constexpr int S = G * E;
    // the row's weights in stencil order, staged so that the sorted order can
    // be gathered without a second pass over global memory
    __shared__ double sw[256 / G][4][S];
    const int lane = lane_id();
    const int gl = lane & (G - 1);
    const int rib = threadIdx.x / G;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    if (row >= N) return;  // whole groups leave together (G divides 64)
    const int64_t off = offsets[row];
    const int64_t n64 = offsets[row + 1] - off;
    const int n = (n64 < 0 || n64 > n_max) ? 0 : (int)n64;
    int key[E], pos[E];
    double wv[4][E];
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int e = gl + G * s;
        pos[s] = e;
        key[s] = (e < n) ? idx[off + e] : 0x7FFFFFFF;
    }
    // issued before the sort so that the loads are in flight during it
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const int e = gl + G * s;
            wv[r][s] = (r < n_ops && e < n) ? w[r * nnz + off + e] : 0.0;
        }
#pragma unroll
    for (int k = 2; k <= S; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= G) {
                constexpr int dummy = 0;
                (void)dummy;
#pragma unroll
                for (int s = 0; s < E; ++s) {
                    const int s2 = s ^ (j / G);
                    if (s2 > s) {
                        const int e = gl + G * s;
                        const bool asc = (e & k) == 0;
                        const bool sw = asc ? (key[s] > key[s2] || (key[s] == key[s2] && pos[s] > pos[s2]))
                                            : (key[s] < key[s2] || (key[s] == key[s2] && pos[s] < pos[s2]));
                        if (sw) {
                            int tk = key[s], tp = pos[s];
                            key[s] = key[s2];
                            pos[s] = pos[s2];
                            key[s2] = tk;
                            pos[s2] = tp;
                        }
                    }
                }
            } else {
#pragma unroll
                for (int s = 0; s < E; ++s) {
                    const int e = gl + G * s;
                    const int pk = __shfl_xor(key[s], j);
                    const int pp = __shfl_xor(pos[s], j);
                    const bool asc = (e & k) == 0;
                    const bool want_min = ((e & j) == 0) == asc;
                    const bool pl = pk < key[s] || (pk == key[s] && pp < pos[s]);
                    const bool ml = key[s] < pk || (key[s] == pk && pos[s] < pp);
                    if (want_min ? pl : ml) {
                        key[s] = pk;
                        pos[s] = pp;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int s = 0; s < E; ++s) sw[rib][r][gl + G * s] = wv[r][s];
    wave_lds_sync();  // the group lies inside one wavefront
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int e = gl + G * s;
        if (e < n) {
            col[off + e] = key[s];
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (r < n_ops) vals[r * nnz + off + e] = sw[rib][r][pos[s]];
        }
    }
    (void)lane;
}

template <int G, int E>
void launch_rows(int64_t N, const int64_t* offsets, const int32_t* idx, const double* w, int n_ops, int64_t nnz,
                 int n_max, int32_t* col, double* vals, hipStream_t s) {
    const int64_t threads = N * G;
    hipLaunchKernelGGL((k_csr_rows<G, E>), dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, N, offsets, idx,
                       w, n_ops, nnz, n_max, col, vals);
}

}  // namespace

extern "C" rbf_status rbf_assemble_csr(rbf_ctx* ctx, int64_t N, const int64_t* offsets, const int32_t* idx,
                                       const double* w, int n_ops, int64_t nnz, int n_max, int64_t* row_ptr,
                                       int32_t* col, double* vals) {
    if (!ctx || !offsets || !idx || !row_ptr || !col || N < 1 || nnz < 1 || n_max < 1 || n_max > 256)
        return RBF_EINVAL;
    if (n_ops < 0 || n_ops > 4 || (n_ops > 0 && (!w || !vals))) return RBF_EINVAL;
    if (n_ops > 0 && w == vals) return RBF_EINVAL;
    RBF_HIP_CHECK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    hipLaunchKernelGGL(k_copy_rowptr, dim3((unsigned)((N + 1 + 255) / 256)), dim3(256), 0, s, offsets, row_ptr,
                       N + 1);
    if (n_max <= 16)
        launch_rows<16, 1>(N, offsets, idx, w, n_ops, nnz, n_max, col, vals, s);
    else if (n_max <= 32)
        launch_rows<16, 2>(N, offsets, idx, w, n_ops, nnz, n_max, col, vals, s);
    else if (n_max <= 64)
        launch_rows<32, 2>(N, offsets, idx, w, n_ops, nnz, n_max, col, vals, s);
    else if (n_max <= 128)
        launch_rows<64, 2>(N, offsets, idx, w, n_ops, nnz, n_max, col, vals, s);
    else
        launch_rows<64, 4>(N, offsets, idx, w, n_ops, nnz, n_max, col, vals, s);
    RBF_LAUNCH_CHECK();
    return RBF_OK;
}
