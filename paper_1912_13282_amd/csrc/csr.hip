// CSR form of the operator matrix (Sec. 2.3.2): row i holds node i's stencil
// weights at the stencil columns, columns ascending, at most sum n_i nonzeros.
//
// One group of G lanes sorts one row: E elements per lane (G*E >= n_i), a
// bitonic network (mirror form: every comparator keeps the minimum in its
// lower element) on keys that pack the column above the stencil position; lane
// exchanges inside a row of 16 lanes are DPP moves.  The columns are written
// and every operator's weights gathered by the position.  The pass reads idx
// and w once and writes col and vals once.
#include "common.hpp"

namespace {

__global__ __launch_bounds__(256) void k_copy_rowptr(const int64_t* __restrict__ off, int64_t* __restrict__ rp,
                                                     int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) rp[i] = off[i];
}

// Sort key of a row entry: its column above its stencil position (8 bits), so
// that equal columns keep the stencil order; 32 bits while every column is
// below 2^24, 64 bits otherwise.
template <typename K>
struct CsrKey;
template <>
struct CsrKey<uint32_t> {
    static __device__ __forceinline__ uint32_t pack(int c, int e) { return ((uint32_t)c << 8) | (uint32_t)e; }
    template <int M>
    static __device__ __forceinline__ uint32_t lane_xor(uint32_t v) { return lane_xor_u32<M>(v); }
    static __device__ __forceinline__ uint32_t mn(uint32_t a, uint32_t b) { return a < b ? a : b; }
    static __device__ __forceinline__ uint32_t mx(uint32_t a, uint32_t b) { return a < b ? b : a; }
    static constexpr uint32_t PAD = 0xFFFFFFFFu;
};
template <>
struct CsrKey<uint64_t> {
    static __device__ __forceinline__ uint64_t pack(int c, int e) { return ((uint64_t)(uint32_t)c << 8) | (uint32_t)e; }
    template <int M>
    static __device__ __forceinline__ uint64_t lane_xor(uint64_t v) {
        return (uint64_t)lane_xor_u32<M>((uint32_t)v) | ((uint64_t)lane_xor_u32<M>((uint32_t)(v >> 32)) << 32);
    }
    static __device__ __forceinline__ uint64_t mn(uint64_t a, uint64_t b) { return a < b ? a : b; }
    static __device__ __forceinline__ uint64_t mx(uint64_t a, uint64_t b) { return a < b ? b : a; }
    static constexpr uint64_t PAD = ~0ull;
};

// Compare-exchange of element e = gl + G s with e ^ J, the lower element keeping the minimum.
template <typename K, int G, int E, int J>
__device__ __forceinline__ void cmpx_xor(K (&key)[E], int gl) {
    using C = CsrKey<K>;
    if constexpr (J < G) {
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const K p = C::template lane_xor<J>(key[s]);
            key[s] = (gl & J) ? C::mx(key[s], p) : C::mn(key[s], p);
        }
    } else {
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const int s2 = s ^ (J / G);
            if (s2 > s) {
                const K lo = C::mn(key[s], key[s2]), hi = C::mx(key[s], key[s2]);
                key[s] = lo;
                key[s2] = hi;
            }
        }
    }
}

// First stage of the merge of blocks of KB elements: e pairs with e ^ (KB - 1)
// (the mirror inside the block), the lower element keeping the minimum.
template <typename K, int G, int E, int KB>
__device__ __forceinline__ void cmpx_mirror(K (&key)[E], int gl) {
    using C = CsrKey<K>;
    if constexpr (KB <= G) {
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const K p = C::template lane_xor<KB - 1>(key[s]);
            key[s] = (gl & (KB / 2)) ? C::mx(key[s], p) : C::mn(key[s], p);
        }
    } else {
        // partner of (lane gl, slot s): lane gl ^ (G - 1), slot s ^ (KB / G - 1)
        constexpr int SM = KB / G - 1, HB = KB / (2 * G);
        K p[E];
#pragma unroll
        for (int s = 0; s < E; ++s) p[s] = C::template lane_xor<G - 1>(key[s ^ SM]);
#pragma unroll
        for (int s = 0; s < E; ++s) key[s] = (s & HB) ? C::mx(key[s], p[s]) : C::mn(key[s], p[s]);
    }
}

template <typename K, int G, int E, int KB>
__device__ __forceinline__ void merge_stages(K (&key)[E], int gl) {
    cmpx_mirror<K, G, E, KB>(key, gl);
    if constexpr (KB / 4 >= 1) cmpx_xor<K, G, E, KB / 4>(key, gl);
    if constexpr (KB / 8 >= 1) cmpx_xor<K, G, E, KB / 8>(key, gl);
    if constexpr (KB / 16 >= 1) cmpx_xor<K, G, E, KB / 16>(key, gl);
    if constexpr (KB / 32 >= 1) cmpx_xor<K, G, E, KB / 32>(key, gl);
    if constexpr (KB / 64 >= 1) cmpx_xor<K, G, E, KB / 64>(key, gl);
    if constexpr (KB / 128 >= 1) cmpx_xor<K, G, E, KB / 128>(key, gl);
    if constexpr (KB / 256 >= 1) cmpx_xor<K, G, E, KB / 256>(key, gl);
}

// Ascending bitonic sort of the S = G E keys of a group of G lanes.
template <typename K, int G, int E, int KB = 2>
__device__ __forceinline__ void sort_keys(K (&key)[E], int gl) {
    if constexpr (KB <= G * E) {
        merge_stages<K, G, E, KB>(key, gl);
        sort_keys<K, G, E, 2 * KB>(key, gl);
    }
}

// One group of G lanes per row.  A row whose size lies outside [0, n_max], or
// that holds a column outside [0, N), gets col = -1 and NaN values over its
// range; a row whose range lies outside [0, nnz] is left unwritten.
template <int G, int E, typename K>
__global__ __launch_bounds__(256) void k_csr_rows(int64_t N, const int64_t* __restrict__ offsets,
                                                  const int32_t* __restrict__ idx, const double* __restrict__ w,
                                                  int n_ops, int64_t nnz, int n_max, int32_t* __restrict__ col,
                                                  double* __restrict__ vals) {
    constexpr int S = G * E;
    using C = CsrKey<K>;
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
    if (n64 < 0 || off < 0 || off + n64 > nnz) return;  // uniform per group
    const int n = (n64 > n_max) ? 0 : (int)n64;
    K key[E];
    bool bad = n64 > n_max;
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int e = gl + G * s;
        const int c = (e < n) ? idx[off + e] : 0;
        bad = bad || c < 0 || (int64_t)c >= N;
        key[s] = (e < n) ? C::pack(c, e) : C::PAD;
    }
    const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1) << (lane & ~(G - 1)));
    if (ballot64(bad) & gmask) {  // uniform per group
        for (int64_t e = gl; e < n64; e += G) {
            col[off + e] = -1;
            for (int r = 0; r < n_ops; ++r) vals[r * nnz + off + e] = __builtin_nan("");
        }
        return;
    }
    double wv[4][E];
    // issued before the sort so that the loads are in flight during it
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const int e = gl + G * s;
            wv[r][s] = (r < n_ops && e < n) ? w[r * nnz + off + e] : 0.0;
        }
    sort_keys<K, G, E>(key, gl);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int s = 0; s < E; ++s) sw[rib][r][gl + G * s] = wv[r][s];
    wave_lds_sync();  // the group lies inside one wavefront
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int e = gl + G * s;
        if (e < n) {
            const int p = (int)(key[s] & 0xFF);
            col[off + e] = (int32_t)(key[s] >> 8);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (r < n_ops) vals[r * nnz + off + e] = sw[rib][r][p];
        }
    }
}

template <int G, int E>
void launch_rows(int64_t N, const int64_t* offsets, const int32_t* idx, const double* w, int n_ops, int64_t nnz,
                 int n_max, int32_t* col, double* vals, hipStream_t s) {
    const int64_t threads = N * G;
    const dim3 grid((unsigned)((threads + 255) / 256));
    if (N < (int64_t)1 << 24)  // every valid column fits the 24 bits of the 32-bit key
        hipLaunchKernelGGL((k_csr_rows<G, E, uint32_t>), grid, dim3(256), 0, s, N, offsets, idx, w, n_ops, nnz, n_max,
                           col, vals);
    else
        hipLaunchKernelGGL((k_csr_rows<G, E, uint64_t>), grid, dim3(256), 0, s, N, offsets, idx, w, n_ops, nnz, n_max,
                           col, vals);
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
