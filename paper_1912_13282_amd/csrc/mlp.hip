// Learned surrogate of the 2D, 15-node Laplacian RBF-FD weights.
//
// Network 30 -> 128 -> 128 -> 128 -> 15 (erf-GELU), inputs the scaled stencil
// offsets (x_j - x_i)/s in stencil order and in a canonical frame (rotation
// and reflection, under which the Laplacian weights do not change), outputs
// the scaled weights w_j s^2.
// Matrix products run on the MFMA units in bfloat16 with float32 accumulation
// (v_mfma_f32_16x16x32_bf16); biases, activations' derivatives, the loss and
// Adam are float32.  Values are rounded to bfloat16 at exactly these points:
//   forward : the input x, every weight matrix, every hidden activation;
//   backward: the output gradient and every pre-activation gradient.
// Bias gradients use the unrounded float32 gradients.
//
// Layout trick.  A layer is computed transposed, Z^T = W H^T: the A operand is
// a 16-row tile of W, the B operand 16 samples of H^T.  The accumulator of an
// MFMA leaves lane (sample s, group g) holding output features 4g..4g+3 of its
// 16-row tile; two consecutive tiles then ARE the B operand of the next layer
// for a 32-wide k block, provided that block's k order is
//   k(g, j) = 32 kb + (j < 4 ? 4g + j : 16 + 4g + j - 4).
// The weights are stored ("packed") in that permuted order, so activations stay
// in registers from input to output.  Gradients of the weights contract over
// samples and need the transpose: they are staged through LDS.
//
// Inference adds, per stencil and in float64, the projection of the network
// output y onto the polynomial-reproduction constraints (second block row of
// eq. rbf-system-aug): w = y + Q (Q^T Q)^{-1} (l_q - Q^T y), the residual
// max|Q^T w - l_q| / max(1, max|l_q|), and acceptance against a tolerance;
// rejected stencils are solved by the plain float64 kernel.
#include "weights_kernels.hpp"

#include <math.h>

namespace rbf {
namespace mlp {

constexpr int IN = 30, H = 128, OUT = 15, NODES = 15;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + H * IN, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H;
constexpr int OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + H * H, OFF_W4 = OFF_B3 + H, OFF_B4 = OFF_W4 + OUT * H;
constexpr int NPARAM = OFF_B4 + OUT;
static_assert(NPARAM == RBF_MLP_NPARAM, "parameter count");
// packed operand tiles (64 lanes x 8 bfloat16 = 1 KiB each)
constexpr int TF1 = 0, TF2 = 8, TF3 = 40, TF4 = 72, TFWD = 76;  // forward: W tiles
constexpr int TB2 = 76, TB3 = 108, TB4 = 140, TALL = 148;       // backward: W^T tiles
static_assert(TALL * 1024 == RBF_MLP_PACKED_BYTES, "packed size");
constexpr int PSTRIDE = 38976;  // per-block partial gradients (+ loss at NPARAM), 64-float aligned
constexpr int SP = 72;          // LDS row stride (bfloat16) of the transposed staging arrays
constexpr int NCT = 2;          // inference: column tiles of 16 samples per wave
constexpr int SPB = 4 * 16 * NCT;  // inference: samples per block

typedef __bf16 bf16x8 __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef unsigned short u16x8 __attribute__((__vector_size__(8 * sizeof(unsigned short))));
typedef float f32x4 __attribute__((__vector_size__(4 * sizeof(float))));

// float -> bfloat16 bits, round to nearest, ties to even: the conversion
// instruction of gfx950 (two values per instruction; four integer operations
// per value by hand were an eighth of the surrogate's VALU work)
__device__ __forceinline__ unsigned short bf16_bits(float x) { return __builtin_bit_cast(unsigned short, (__bf16)x); }

// two values into one 32-bit word (lo in the low half), the unit the conversion
// writes: whole words keep the packed operands out of 16-bit inserts
typedef unsigned u32x4 __attribute__((__vector_size__(4 * sizeof(unsigned))));
__device__ __forceinline__ unsigned bf16x2_bits(float lo, float hi) {
    return (unsigned)bf16_bits(lo) | ((unsigned)bf16_bits(hi) << 16);
}

__device__ __forceinline__ bf16x8 pack8(const float v[8]) {
    u32x4 w;
#pragma unroll
    for (int j = 0; j < 4; ++j) w[j] = bf16x2_bits(v[2 * j], v[2 * j + 1]);
    return __builtin_bit_cast(bf16x8, w);
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 zero4() {
    f32x4 z = {0.f, 0.f, 0.f, 0.f};
    return z;
}

// erf-GELU g(z) = z Phi(z), Phi(z) = (1 + erf(z / sqrt 2)) / 2, g'(z) = Phi(z) + z phi(z).
// erf from Abramowitz & Stegun 7.1.26 (Hastings' rational approximation,
// |error| <= 1.5e-7): for u >= 0, 1 - erf(u) = t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) e^(-u^2),
// t = 1 / (1 + p u).  Phi comes straight from this tail form (no cancellation for
// negative z), and phi reuses the same exponential e^(-z^2/2).
struct PhiPair {
    float Phi, phi;
};
__device__ __forceinline__ PhiPair normal_cdf_pdf(float z) {
    const float u = fabsf(z) * 0.70710678118654752f;
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, u, 1.0f));
    const float poly =
        t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f), -0.284496736f), 0.254829592f);
    const float e = __builtin_amdgcn_exp2f(-u * u * 1.44269504088896341f);  // e^(-u^2) = e^(-z^2/2)
    const float tail = 0.5f * poly * e;                                     // 1 - Phi(|z|)
    PhiPair r;
    r.Phi = (z >= 0.0f) ? 1.0f - tail : tail;
    r.phi = 0.39894228040143268f * e;
    return r;
}
__device__ __forceinline__ float gelu(float z) { return z * normal_cdf_pdf(z).Phi; }
__device__ __forceinline__ float gelu_prime(float z) {
    const PhiPair p = normal_cdf_pdf(z);
    return p.Phi + z * p.phi;
}
__device__ __forceinline__ void gelu_both(float z, float& g, float& gp) {
    const PhiPair p = normal_cdf_pdf(z);
    g = z * p.Phi;
    gp = p.Phi + z * p.phi;
}

// feature index held in slot j of lane group g of k block kb (hidden layers)
__host__ __device__ constexpr int kperm(int kb, int g, int j) { return 32 * kb + (j < 4 ? 4 * g + j : 12 + 4 * g + j); }

// value of packed element e (tile e/512, lane (e%512)/8, slot e%8)
__device__ float packed_value(const float* __restrict__ p, int e) {
    const int tile = e >> 9, lane = (e >> 3) & 63, j = e & 7;
    const int g = lane >> 4, row = lane & 15;
    if (tile < TF2) {  // layer 1: W1[o][k], k = 8g + j (input order)
        const int o = 16 * tile + row, k = 8 * g + j;
        return k < IN ? p[OFF_W1 + o * IN + k] : 0.f;
    }
    if (tile < TF4) {  // layers 2, 3: W[o][kperm]
        const int L = tile < TF3 ? 2 : 3, t = tile - (L == 2 ? TF2 : TF3);
        const int o = 16 * (t >> 2) + row, k = kperm(t & 3, g, j);
        return p[(L == 2 ? OFF_W2 : OFF_W3) + o * H + k];
    }
    if (tile < TFWD) {  // layer 4: W4[o][kperm], o < 15
        const int o = row, k = kperm(tile - TF4, g, j);
        return o < OUT ? p[OFF_W4 + o * H + k] : 0.f;
    }
    if (tile < TB4) {  // transposed layers 2, 3: A[k][o] = W[o][k], o in kperm order
        const int L = tile < TB3 ? 2 : 3, t = tile - (L == 2 ? TB2 : TB3);
        const int k = 16 * (t >> 2) + row, o = kperm(t & 3, g, j);
        return p[(L == 2 ? OFF_W2 : OFF_W3) + o * H + k];
    }
    {  // transposed layer 4: one 32-wide o block, o = kperm(0, g, j) < 15
        const int k = 16 * (tile - TB4) + row, o = kperm(0, g, j);
        return o < OUT ? p[OFF_W4 + o * H + k] : 0.f;
    }
}

__global__ __launch_bounds__(256) void k_pack(const float* __restrict__ params, unsigned short* __restrict__ packed) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e < TALL * 512) packed[e] = bf16_bits(packed_value(params, e));
}

// One hidden layer for NCT column tiles of 16 samples: out = bf16(gelu(W in + b))
// in the next layer's B-operand order; optionally gelu'(z) in accumulator order.
template <int NCT, int KB, bool GRAD>
__device__ __forceinline__ void hidden_layer(const bf16x8* tiles, const float* __restrict__ bias,
                                             const bf16x8 (&in)[KB][NCT], bf16x8 (&out)[4][NCT],
                                             f32x4 (&gp)[8][NCT]) {
    const int lane = lane_id(), g = lane >> 4;
    u32x4 ow[4][NCT];
#pragma unroll
    for (int ot = 0; ot < 8; ++ot) {
        f32x4 acc[NCT];
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) acc[ct] = zero4();
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            const bf16x8 a = tiles[(ot * KB + kb) * 64 + lane];
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct) acc[ct] = mfma(a, in[kb][ct], acc[ct]);
        }
        float b[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) b[r] = bias[16 * ot + 4 * g + r];
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            float gz[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float z = acc[ct][r] + b[r];
                if constexpr (GRAD) {
                    float gpz;
                    gelu_both(z, gz[r], gpz);
                    gp[ot][ct][r] = gpz;
                } else {
                    gz[r] = gelu(z);
                }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) ow[ot >> 1][ct][(ot & 1) * 2 + h] = bf16x2_bits(gz[2 * h], gz[2 * h + 1]);
        }
        // keep each tile's operand loads next to their use (bounds register pressure)
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) out[kb][ct] = __builtin_bit_cast(bf16x8, ow[kb][ct]);
}

// Whole network for NCT column tiles; y[ct][r] = output 4g + r of sample 16 ct + (lane & 15)
template <int NCT, bool GRAD>
__device__ __forceinline__ void forward(const bf16x8* tiles, const float* __restrict__ params,
                                        const bf16x8 (&x)[1][NCT], bf16x8 (&h1)[4][NCT], bf16x8 (&h2)[4][NCT],
                                        bf16x8 (&h3)[4][NCT], f32x4 (&gp1)[8][NCT], f32x4 (&gp2)[8][NCT],
                                        f32x4 (&gp3)[8][NCT], f32x4 (&y)[NCT]) {
    const int lane = lane_id(), g = lane >> 4;
    hidden_layer<NCT, 1, GRAD>(tiles + TF1 * 64, params + OFF_B1, x, h1, gp1);
    hidden_layer<NCT, 4, GRAD>(tiles + TF2 * 64, params + OFF_B2, h1, h2, gp2);
    hidden_layer<NCT, 4, GRAD>(tiles + TF3 * 64, params + OFF_B3, h2, h3, gp3);
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) y[ct] = zero4();
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        const bf16x8 a = tiles[(TF4 + kb) * 64 + lane];
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) y[ct] = mfma(a, h3[kb][ct], y[ct]);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int o = 4 * g + r;
        const float b = o < OUT ? params[OFF_B4 + o] : 0.f;
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) y[ct][r] += b;
    }
}

// copy the forward tiles into LDS (whole block)
__device__ __forceinline__ void load_tiles(bf16x8* s, const bf16x8* __restrict__ packed) {
    for (int e = threadIdx.x; e < TFWD * 64; e += blockDim.x) s[e] = packed[e];
    __syncthreads();
}

// ------------------------------------------------------------ plain forward
// y[B][15] = net(x[B][30]); 16 NCT samples per wave, forward tiles in LDS.
__global__ __launch_bounds__(256, 1) void k_forward(const float* __restrict__ params,
                                                    const bf16x8* __restrict__ packed, const float* __restrict__ x,
                                                    int64_t B, float* __restrict__ y) {
    __shared__ bf16x8 sW[TFWD * 64];
    load_tiles(sW, packed);
    const int lane = lane_id(), g = lane >> 4, s = lane & 15, wv = threadIdx.x >> 6;
    const int64_t ntiles = (B + SPB - 1) / SPB;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t base = tile * SPB + wv * 16 * NCT;
        bf16x8 xb[1][NCT];
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            const int64_t b = base + 16 * ct + s;
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = 8 * g + j;
                v[j] = (b < B && k < IN) ? x[b * IN + k] : 0.f;
            }
            xb[0][ct] = pack8(v);
        }
        bf16x8 h1[4][NCT], h2[4][NCT], h3[4][NCT];
        f32x4 gp[8][NCT], yv[NCT];
        forward<NCT, false>(sW, params, xb, h1, h2, h3, gp, gp, gp, yv);
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            const int64_t b = base + 16 * ct + s;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (b < B && 4 * g + r < OUT) y[b * OUT + 4 * g + r] = yv[ct][r];
        }
    }
}

// ------------------------------------------------------------ gradients
__device__ __forceinline__ float sum16(float v) {
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    return v;
}

// bias gradient of one layer: per-wave sums over samples into red[wv][o], then
// (after the barrier) the block sum in wave order
template <int NOT>
__device__ __forceinline__ void stage_bias(float (*red)[H], const f32x4 (&dz)[NOT], int wv) {
    const int lane = lane_id(), g = lane >> 4, s = lane & 15;
#pragma unroll
    for (int ot = 0; ot < NOT; ++ot)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float t = sum16(dz[ot][r]);
            if (s == 0) red[wv][16 * ot + 4 * g + r] = t;
        }
}

// write the B-operand vectors v[kb] (features kperm, or 8g + j for the input)
// of this wave's 16 samples into the transposed staging array T[feature][sample]
template <int KB, bool INPUT>
__device__ __forceinline__ void stage_T(unsigned short* T, const bf16x8 (&v)[KB][1], int wv) {
    const int lane = lane_id(), g = lane >> 4, s = lane & 15;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        const u16x8 u = __builtin_bit_cast(u16x8, v[kb][0]);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int f = INPUT ? 8 * g + j : kperm(kb, g, j);
            T[f * SP + 16 * wv + s] = u[j];
        }
    }
}

// dW[o][k] = sum over the block's 64 samples of DZ[o][s] ACT[k][s], for
// o < NO (16-row tiles NOT), k < NI (16-col tiles NKT); the block's partial is
// written to part[woff + o * NI + k]
template <int NOT, int NKT>
__device__ __forceinline__ void weight_grad(const unsigned short* DZ, const unsigned short* ACT, float* part, int woff,
                                            int NO, int NI, int wv) {
    const int lane = lane_id(), g = lane >> 4, c = lane & 15;
    for (int t = wv; t < NOT * NKT; t += 4) {
        const int ot = t / NKT, kt = t % NKT;
        f32x4 acc = zero4();
#pragma unroll
        for (int sb = 0; sb < 2; ++sb) {
            const bf16x8 a = *(const bf16x8*)(DZ + (16 * ot + c) * SP + 32 * sb + 8 * g);
            const bf16x8 b = *(const bf16x8*)(ACT + (16 * kt + c) * SP + 32 * sb + 8 * g);
            acc = mfma(a, b, acc);
        }
        const int k = 16 * kt + c;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = 16 * ot + 4 * g + r;
            if (o < NO && k < NI) part[woff + o * NI + k] = acc[r];
        }
    }
}

// dh^T = W^T dz (A = packed W^T tiles, NOB o blocks), then dz' = dh * gelu'(z)
template <int NOB>
__device__ __forceinline__ void back_hidden(const bf16x8* __restrict__ tiles, const bf16x8 (&dzb)[NOB][1],
                                            const f32x4 (&gp)[8][1], f32x4 (&dz)[8], bf16x8 (&dzb_next)[4][1]) {
    const int lane = lane_id();
    u32x4 ow[4];
#pragma unroll
    for (int kt = 0; kt < 8; ++kt) {
        f32x4 acc = zero4();
#pragma unroll
        for (int ob = 0; ob < NOB; ++ob) acc = mfma(tiles[(kt * NOB + ob) * 64 + lane], dzb[ob][0], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) dz[kt][r] = acc[r] * gp[kt][0][r];
#pragma unroll
        for (int h = 0; h < 2; ++h) ow[kt >> 1][(kt & 1) * 2 + h] = bf16x2_bits(dz[kt][2 * h], dz[kt][2 * h + 1]);
    }
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) dzb_next[kb][0] = __builtin_bit_cast(bf16x8, ow[kb]);
}

// Partial gradients of one block of 64 samples (rows sel[b] of x and t, or b).
// loss = sum (y - t)^2 / (B 15); every gradient carries the factor 2 / (B 15).
__global__ __launch_bounds__(256, 1) void k_grad(const float* __restrict__ params, const bf16x8* __restrict__ packed,
                                                 const float* __restrict__ x, const float* __restrict__ tgt,
                                                 int64_t n_rows, const int64_t* __restrict__ sel, int64_t B,
                                                 float gscale, float* __restrict__ part_all) {
    __shared__ __attribute__((aligned(16))) unsigned short DZ[H * SP];
    __shared__ __attribute__((aligned(16))) unsigned short ACT[H * SP];
    __shared__ float red[4][H];
    const int lane = lane_id(), g = lane >> 4, s = lane & 15, wv = threadIdx.x >> 6;
    float* part = part_all + (int64_t)blockIdx.x * PSTRIDE;
    const int64_t b = (int64_t)blockIdx.x * 64 + wv * 16 + s;
    int64_t row = b < B ? (sel ? sel[b] : b) : -1;
    const bool valid = row >= 0 && row < n_rows;  // rows outside the arrays contribute nothing
    if (!valid) row = 0;

    bf16x8 xb[1][1];
    {
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * g + j;
            v[j] = (valid && k < IN) ? x[row * IN + k] : 0.f;
        }
        xb[0][0] = pack8(v);
    }
    bf16x8 h1[4][1], h2[4][1], h3[4][1];
    f32x4 gp1[8][1], gp2[8][1], gp3[8][1], y[1];
    forward<1, true>(packed, params, xb, h1, h2, h3, gp1, gp2, gp3, y);

    // output gradient
    float lossp = 0.f;
    f32x4 g4[1];
    {
        float v[8];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = 4 * g + r;
            float gv = 0.f;
            if (valid && o < OUT) {
                const float d = y[0][r] - tgt[row * OUT + o];
                lossp += d * d;
                gv = d * gscale;
            }
            g4[0][r] = gv;
            v[r] = gv;
            v[4 + r] = 0.f;
        }
        bf16x8 gb[1][1];
        gb[0][0] = pack8(v);

        // ---- layer 4
        stage_bias<1>(red, g4, wv);
        {
            // DZ rows o = 4g + r (< 16), ACT = h3
            const u16x8 u = __builtin_bit_cast(u16x8, gb[0][0]);
#pragma unroll
            for (int r = 0; r < 4; ++r) DZ[(4 * g + r) * SP + 16 * wv + s] = u[r];
        }
        stage_T<4, false>(ACT, h3, wv);
        // loss partial
        float l = lossp;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o);
        __syncthreads();
        if (threadIdx.x < OUT) part[OFF_B4 + threadIdx.x] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) +
                                                             red[2][threadIdx.x]) + red[3][threadIdx.x];
        weight_grad<1, 8>(DZ, ACT, part, OFF_W4, OUT, H, wv);
        __syncthreads();
        if (lane == 0) red[wv][0] = l;
        __syncthreads();
        if (threadIdx.x == 0) part[NPARAM] = ((red[0][0] + red[1][0]) + red[2][0]) + red[3][0];
        __syncthreads();

        // ---- layer 3
        f32x4 dz[8];
        bf16x8 dzb[4][1];
        back_hidden<1>(packed + TB4 * 64, gb, gp3, dz, dzb);
        stage_bias<8>(red, dz, wv);
        stage_T<4, false>(DZ, dzb, wv);
        stage_T<4, false>(ACT, h2, wv);
        __syncthreads();
        if (threadIdx.x < H) part[OFF_B3 + threadIdx.x] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) +
                                                           red[2][threadIdx.x]) + red[3][threadIdx.x];
        weight_grad<8, 8>(DZ, ACT, part, OFF_W3, H, H, wv);
        __syncthreads();

        // ---- layer 2
        bf16x8 dzb2[4][1];
        back_hidden<4>(packed + TB3 * 64, dzb, gp2, dz, dzb2);
        stage_bias<8>(red, dz, wv);
        stage_T<4, false>(DZ, dzb2, wv);
        stage_T<4, false>(ACT, h1, wv);
        __syncthreads();
        if (threadIdx.x < H) part[OFF_B2 + threadIdx.x] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) +
                                                           red[2][threadIdx.x]) + red[3][threadIdx.x];
        weight_grad<8, 8>(DZ, ACT, part, OFF_W2, H, H, wv);
        __syncthreads();

        // ---- layer 1
        bf16x8 dzb1[4][1];
        back_hidden<4>(packed + TB2 * 64, dzb2, gp1, dz, dzb1);
        stage_bias<8>(red, dz, wv);
        stage_T<4, false>(DZ, dzb1, wv);
        stage_T<1, true>(ACT, xb, wv);
        __syncthreads();
        if (threadIdx.x < H) part[OFF_B1 + threadIdx.x] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) +
                                                           red[2][threadIdx.x]) + red[3][threadIdx.x];
        weight_grad<8, 2>(DZ, ACT, part, OFF_W1, H, IN, wv);
    }
}

// grads[p] = sum over blocks (in block order) of the partials; loss likewise
__global__ __launch_bounds__(256) void k_reduce(const float* __restrict__ part, int nblk, float* __restrict__ grads,
                                                float* __restrict__ loss, float loss_scale) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p > NPARAM) return;
    float acc = 0.f;
    for (int k = 0; k < nblk; ++k) acc += part[(int64_t)k * PSTRIDE + p];
    if (p < NPARAM) grads[p] = acc;
    else if (loss) *loss = acc * loss_scale;
}

// Adam (bias-corrected moments; c1 = 1/(1-b1^t), c2 = 1/(1-b2^t))
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ gr,
                                              float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                              float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= NPARAM) return;
    const float gi = gr[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// ------------------------------------------------------------ input frame
// Canonical frame of a stencil (the Laplacian weights are invariant under
// rotations and reflections): rotate so that node 1, the nearest neighbour,
// lies on +x, then reflect y so that node 2 has y >= 0.  The same float64
// operations (no contraction) are used by the training data and by inference.
__device__ __forceinline__ double sq2(double x, double y) {
#pragma clang fp contract(off)
    return x * x + y * y;
}
__device__ __forceinline__ void canon_frame(double o1x, double o1y, double o2x, double o2y, double& cs, double& sn,
                                            double& fl) {
#pragma clang fp contract(off)
    const double r = sqrt(o1x * o1x + o1y * o1y);
    cs = r > 0.0 ? o1x / r : 1.0;
    sn = r > 0.0 ? o1y / r : 0.0;
    fl = (cs * o2y - sn * o2x) < 0.0 ? -1.0 : 1.0;
}
__device__ __forceinline__ void canon_apply(double ox, double oy, double cs, double sn, double fl, double sc, float& fx,
                                            float& fy) {
#pragma clang fp contract(off)
    fx = (float)((cs * ox + sn * oy) / sc);
    fy = (float)((fl * (cs * oy - sn * ox)) / sc);
}

// ------------------------------------------------------------ training data
// feat[i][2j..2j+1] = the offset X[idx_j] - X[i] in the canonical frame over s,
// s = max_j |X[idx_j] - X[i]|; tgt[i][j] = w_lap[off + j] s^2; scale[i] = s.
// Stencils that are not 2D 15-node stencils with valid indices get NaN rows.
__global__ __launch_bounds__(256) void k_dataset(const double* __restrict__ X, int64_t N,
                                                 const int64_t* __restrict__ offsets, const int32_t* __restrict__ idx,
                                                 int64_t nnz,
                                                 const double* __restrict__ wlap, float* __restrict__ feat,
                                                 float* __restrict__ tgt, double* __restrict__ scale) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const int64_t off = offsets[i];
    bool ok = offsets[i + 1] - off == NODES && off >= 0 && off + NODES <= nnz;
    double o[NODES][2];
    double r2 = 0.0;
    const int c = ok ? idx[off] : -1;
    ok = ok && c >= 0 && c < N;
    for (int j = 0; j < NODES; ++j) {
        const int id = ok ? idx[off + j] : -1;
        ok = ok && id >= 0 && id < N;
        o[j][0] = ok ? X[2 * (int64_t)id] - X[2 * (int64_t)c] : 0.0;
        o[j][1] = ok ? X[2 * (int64_t)id + 1] - X[2 * (int64_t)c + 1] : 0.0;
        r2 = fmax(r2, sq2(o[j][0], o[j][1]));
    }
    const double sc = sqrt(r2);
    double cs, sn, fl;
    canon_frame(o[1][0], o[1][1], o[2][0], o[2][1], cs, sn, fl);
    const float nan = __builtin_nanf("");
    for (int j = 0; j < NODES; ++j) {
        float fx, fy;
        canon_apply(o[j][0], o[j][1], cs, sn, fl, sc, fx, fy);
        feat[i * IN + 2 * j] = ok ? fx : nan;
        feat[i * IN + 2 * j + 1] = ok ? fy : nan;
        if (tgt) tgt[i * OUT + j] = (ok && wlap) ? (float)(wlap[off + j] * sc * sc) : nan;
    }
    if (scale) scale[i] = ok ? sc : __builtin_nan("");
}

// ------------------------------------------------------------ inference
// Per stencil: features -> network -> float64 projection -> residual test.
// Lane (s, g) of column tile ct works on stencil 16 ct + s and its nodes 4g..4g+3.
__device__ __forceinline__ double xor16_32_sum(double v) {
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}
__device__ __forceinline__ double xor16_32_max(double v) {
    v = fmax(v, __shfl_xor(v, 16));
    v = fmax(v, __shfl_xor(v, 32));
    return v;
}

__global__ __launch_bounds__(256, 2) void k_surrogate(const float* __restrict__ params,
                                                      const bf16x8* __restrict__ packed, const double* __restrict__ X,
                                                      int64_t N, const int64_t* __restrict__ offsets,
                                                      const int32_t* __restrict__ idx, int64_t nnz, double tol,
                                                      double ctol, double* __restrict__ w,
                                                      int8_t* __restrict__ status) {
    __shared__ bf16x8 sW[TFWD * 64];
    load_tiles(sW, packed);
    const int lane = lane_id(), g = lane >> 4, s = lane & 15, wv = threadIdx.x >> 6;
    const int64_t ntiles = (N + SPB - 1) / SPB;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t base = tile * SPB + wv * 16 * NCT;
        bf16x8 xb[1][NCT];
        bool okc[NCT];
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            const int64_t i = base + 16 * ct + s;
            bool ok = i < N;
            int64_t off = 0;
            if (ok) {
                off = offsets[i];
                ok = offsets[i + 1] - off == NODES && off >= 0 && off + NODES <= nnz;
            }
            const int c = ok ? idx[off] : 0;
            ok = ok && c >= 0 && c < N;
            double o[4][2];
            double r2 = 0.0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = 4 * g + r;
                o[r][0] = o[r][1] = 0.0;
                if (ok && j < NODES) {
                    const int id = idx[off + j];
                    if (id >= 0 && id < N) {
                        o[r][0] = X[2 * (int64_t)id] - X[2 * (int64_t)c];
                        o[r][1] = X[2 * (int64_t)id + 1] - X[2 * (int64_t)c + 1];
                    } else {
                        ok = false;
                    }
                }
                r2 = fmax(r2, sq2(o[r][0], o[r][1]));
            }
            // the four lanes of a stencil: g = 0..3 (lane xor 16, 32)
            r2 = fmax(r2, __shfl_xor(r2, 16));
            r2 = fmax(r2, __shfl_xor(r2, 32));
            int okl = ok ? 1 : 0;
            okl &= __shfl_xor(okl, 16);
            okl &= __shfl_xor(okl, 32);
            okc[ct] = okl != 0 && r2 > 0.0;
            const double sc = sqrt(r2);
            // nodes 1 and 2 sit in the g = 0 lane of this stencil
            const int src = lane & 15;
            const double o1x = __shfl(o[1][0], src), o1y = __shfl(o[1][1], src);
            const double o2x = __shfl(o[2][0], src), o2y = __shfl(o[2][1], src);
            double cs, sn, fl;
            canon_frame(o1x, o1y, o2x, o2y, cs, sn, fl);
            float v[8];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float fx, fy;
                canon_apply(o[r][0], o[r][1], cs, sn, fl, sc, fx, fy);
                v[2 * r] = okc[ct] ? fx : 0.f;
                v[2 * r + 1] = okc[ct] ? fy : 0.f;
            }
            xb[0][ct] = pack8(v);
        }
        bf16x8 h1[4][NCT], h2[4][NCT], h3[4][NCT];
        f32x4 gp[8][NCT], yv[NCT];
        forward<NCT, false>(sW, params, xb, h1, h2, h3, gp, gp, gp, yv);

        // projection onto Q^T w = l_q (basis 1, x, y, x^2, xy, y^2; l_q of the Laplacian)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            const int64_t i = base + 16 * ct + s;
            if (i >= N) continue;  // the four lanes of a stencil agree
            const int64_t off = offsets[i];
            if (!okc[ct]) {
                if (g == 0) status[i] = RBF_ST_SURROGATE_REJECTED;
                continue;
            }
            const int c = idx[off];
            double q[4][6], yy[4];
            double r2 = 0.0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = 4 * g + r;
                double ox = 0.0, oy = 0.0;
                if (j < NODES) {
                    const int id = idx[off + j];
                    ox = X[2 * (int64_t)id] - X[2 * (int64_t)c];
                    oy = X[2 * (int64_t)id + 1] - X[2 * (int64_t)c + 1];
                }
                r2 = fmax(r2, sq2(ox, oy));
                q[r][1] = ox;
                q[r][2] = oy;
                yy[r] = (j < NODES) ? (double)yv[ct][r] : 0.0;
            }
            r2 = fmax(r2, __shfl_xor(r2, 16));
            r2 = fmax(r2, __shfl_xor(r2, 32));
            const double sc = sqrt(r2), isc = 1.0 / sc;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const bool live = 4 * g + r < NODES;
                const double xh = q[r][1] * isc, yh = q[r][2] * isc;
                q[r][0] = live ? 1.0 : 0.0;
                q[r][1] = xh;
                q[r][2] = yh;
                q[r][3] = xh * xh;
                q[r][4] = xh * yh;
                q[r][5] = yh * yh;
            }
            // G = Q^T Q (upper triangle) and u = Q^T y
            double G[6][6], u[6];
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                double t = 0.0;
#pragma unroll
                for (int r = 0; r < 4; ++r) t += q[r][a] * yy[r];
                u[a] = xor16_32_sum(t);
#pragma unroll
                for (int bb = a; bb < 6; ++bb) {
                    double t2 = 0.0;
#pragma unroll
                    for (int r = 0; r < 4; ++r) t2 += q[r][a] * q[r][bb];
                    G[a][bb] = xor16_32_sum(t2);
                }
            }
            // Cholesky G = L L^T (L stored in the lower triangle of G, 1/L_kk kept)
            bool spd = true;
            double il[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                double dkk = G[k][k];
#pragma unroll
                for (int p = 0; p < k; ++p) dkk -= G[k][p] * G[k][p];
                spd = spd && dkk > 0.0;
                il[k] = 1.0 / sqrt(spd ? dkk : 1.0);
#pragma unroll
                for (int i2 = k + 1; i2 < 6; ++i2) {
                    double t = G[k][i2];
#pragma unroll
                    for (int p = 0; p < k; ++p) t -= G[i2][p] * G[k][p];
                    G[i2][k] = t * il[k];
                }
            }
            // rhs = l_q - Q^T y; solve L z = rhs, L^T cvec = z
            const double lq[6] = {0.0, 0.0, 0.0, 2.0, 0.0, 2.0};
            double cv[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                double t = lq[k] - u[k];
#pragma unroll
                for (int p = 0; p < k; ++p) t -= G[k][p] * cv[p];
                cv[k] = t * il[k];
            }
#pragma unroll
            for (int k = 5; k >= 0; --k) {
                double t = cv[k];
#pragma unroll
                for (int p = k + 1; p < 6; ++p) t -= G[p][k] * cv[p];
                cv[k] = t * il[k];
            }
            double wl[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double t = yy[r];
#pragma unroll
                for (int a = 0; a < 6; ++a) t += q[r][a] * cv[a];
                wl[r] = (4 * g + r < NODES) ? t : 0.0;
            }
            // residual of the reproduction conditions
            double rho = 0.0;
            bool finite = true;
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                double t = 0.0;
#pragma unroll
                for (int r = 0; r < 4; ++r) t += q[r][a] * wl[r];
                t = xor16_32_sum(t) - lq[a];
                finite = finite && isfinite(t);
                rho = fmax(rho, fabs(t));
            }
            rho /= 2.0;  // max(1, max |l_q|)
            // what the network controls: the projection's correction w - y relative to w
            // (the zero network needs a correction of the whole weights: ratio 1)
            double cmax = 0.0, wmax = 0.0;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (4 * g + r < NODES) {
                    cmax = fmax(cmax, fabs(wl[r] - yy[r]));
                    wmax = fmax(wmax, fabs(wl[r]));
                }
            cmax = xor16_32_max(cmax);
            wmax = xor16_32_max(wmax);
            const bool accept = spd && finite && rho <= tol && cmax <= ctol * wmax;
            if (accept) {
                const double is2 = isc * isc;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (4 * g + r < NODES) w[off + 4 * g + r] = wl[r] * is2;
            }
            if (g == 0) status[i] = accept ? RBF_ST_SURROGATE : RBF_ST_SURROGATE_REJECTED;
        }
    }
}

int grid_persistent(int device, int64_t tiles) {
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) cus = 256;
    const int64_t cap = 2LL * cus;
    return (int)(tiles < cap ? (tiles < 1 ? 1 : tiles) : cap);
}

}  // namespace mlp
}  // namespace rbf

using namespace rbf::mlp;

extern "C" rbf_status rbf_mlp_pack(rbf_ctx* ctx, const float* params, void* packed) {
    if (!ctx || !params || !packed) return RBF_EINVAL;
    RBF_HIP_CHECK(hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_pack, dim3((TALL * 512 + 255) / 256), dim3(256), 0, ctx->stream, params,
                       (unsigned short*)packed);
    RBF_LAUNCH_CHECK();
    return RBF_OK;
}

extern "C" rbf_status rbf_mlp_forward(rbf_ctx* ctx, const float* params, const void* packed, const float* x,
                                      int64_t B, float* y) {
    if (!ctx || !params || !packed || !x || !y || B < 1) return RBF_EINVAL;
    RBF_HIP_CHECK(hipSetDevice(ctx->device));
    const int grid = grid_persistent(ctx->device, (B + SPB - 1) / SPB);
    hipLaunchKernelGGL(k_forward, dim3(grid), dim3(256), 0, ctx->stream, params, (const bf16x8*)packed, x, B, y);
    RBF_LAUNCH_CHECK();
    return RBF_OK;
}

extern "C" rbf_status rbf_mlp_grad_workspace(int64_t B, size_t* bytes) {
    if (!bytes || B < 1) return RBF_EINVAL;
    *bytes = (size_t)((B + 63) / 64) * PSTRIDE * sizeof(float);
    return RBF_OK;
}

extern "C" rbf_status rbf_mlp_grad(rbf_ctx* ctx, const float* params, const void* packed, const float* x,
                                   const float* t, int64_t n_rows, const int64_t* sel, int64_t B, float* grads,
                                   float* loss, void* workspace, size_t ws_bytes) {
    if (!ctx || !params || !packed || !x || !t || !grads || B < 1 || n_rows < 1) return RBF_EINVAL;
    if (!sel && B > n_rows) return RBF_EINVAL;
    size_t need = 0;
    rbf_mlp_grad_workspace(B, &need);
    if (!workspace || ws_bytes < need) return RBF_EWORKSPACE;
    RBF_HIP_CHECK(hipSetDevice(ctx->device));
    const int64_t nblk = (B + 63) / 64;
    if (nblk > (1LL << 30)) return RBF_EINVAL;
    const float gscale = (float)(2.0 / ((double)B * OUT));
    hipLaunchKernelGGL(k_grad, dim3((unsigned)nblk), dim3(256), 0, ctx->stream, params, (const bf16x8*)packed, x, t,
                       n_rows, sel, B, gscale, (float*)workspace);
    hipLaunchKernelGGL(k_reduce, dim3((NPARAM + 1 + 255) / 256), dim3(256), 0, ctx->stream, (const float*)workspace,
                       (int)nblk, grads, loss, (float)(1.0 / ((double)B * OUT)));
    RBF_LAUNCH_CHECK();
    return RBF_OK;
}

extern "C" rbf_status rbf_mlp_adam(rbf_ctx* ctx, float* params, const float* grads, float* m, float* v, int step,
                                   float lr, float beta1, float beta2, float eps, void* packed) {
    if (!ctx || !params || !grads || !m || !v || step < 1) return RBF_EINVAL;
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f && lr >= 0.f)) return RBF_EINVAL;
    RBF_HIP_CHECK(hipSetDevice(ctx->device));
    const float c1 = (float)(1.0 / (1.0 - pow((double)beta1, step)));
    const float c2 = (float)(1.0 / (1.0 - pow((double)beta2, step)));
    hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, ctx->stream, params, grads, m, v, lr, beta1,
                       beta2, eps, c1, c2);
    if (packed)
        hipLaunchKernelGGL(k_pack, dim3((TALL * 512 + 255) / 256), dim3(256), 0, ctx->stream, params,
                           (unsigned short*)packed);
    RBF_LAUNCH_CHECK();
    return RBF_OK;
}

extern "C" rbf_status rbf_surrogate_dataset(rbf_ctx* ctx, const double* X, int64_t N, const int64_t* offsets,
                                            const int32_t* idx, int64_t nnz, const double* w_lap, float* feat,
                                            float* target, double* scale) {
    if (!ctx || !X || !offsets || !idx || !feat || N < 1 || nnz < 1) return RBF_EINVAL;
    RBF_HIP_CHECK(hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_dataset, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, ctx->stream, X, N, offsets, idx,
                       nnz, w_lap, feat, target, scale);
    RBF_LAUNCH_CHECK();
    return RBF_OK;
}

extern "C" rbf_status rbf_surrogate_load(rbf_ctx* ctx, const float* params) {
    if (!ctx || !params) return RBF_EINVAL;
    RBF_HIP_CHECK(hipSetDevice(ctx->device));
    const size_t bytes = rbf_align(NPARAM * sizeof(float)) + RBF_MLP_PACKED_BYTES;
    if (!ctx->mlp_params) {
        RBF_HIP_CHECK(hipMalloc(&ctx->mlp_params, bytes));
        ctx->mlp_bytes = bytes;
    }
    float* p = (float*)ctx->mlp_params;
    void* packed = (char*)ctx->mlp_params + rbf_align(NPARAM * sizeof(float));
    RBF_HIP_CHECK(hipMemcpyAsync(p, params, NPARAM * sizeof(float), hipMemcpyDeviceToDevice, ctx->stream));
    hipLaunchKernelGGL(k_pack, dim3((TALL * 512 + 255) / 256), dim3(256), 0, ctx->stream, p, (unsigned short*)packed);
    RBF_LAUNCH_CHECK();
    return RBF_OK;
}

extern "C" rbf_status rbf_surrogate_weights(rbf_ctx* ctx, const double* X, int64_t N, int d, const int64_t* offsets,
                                            const int32_t* idx, int64_t nnz, int n_max, const rbf_options* opt,
                                            double* w, int8_t* status) {
    if (!ctx || !X || !offsets || !idx || !w || !status || N < 1 || nnz < 1 || n_max < 1) return RBF_EINVAL;
    if (d != 2) return RBF_EDIM;
    if (n_max > N) return RBF_ETOOFEW;
    if (!ctx->mlp_params) return RBF_EINVAL;  // no network loaded
    rbf_options o;
    rbf_options_default(&o);
    if (opt) o = *opt;
    if (!(o.surrogate_tol >= 0.0) || !(o.surrogate_corr_tol >= 0.0)) return RBF_EINVAL;
    if (o.phs_power != 3 && o.phs_power != 5) return RBF_EINVAL;
    const rbf::ClassEntry* c = rbf::find_class(n_max + 6);
    if (!c) return RBF_EUNSUPPORTED;
    RBF_HIP_CHECK(hipSetDevice(ctx->device));
    const float* p = (const float*)ctx->mlp_params;
    const bf16x8* packed = (const bf16x8*)((const char*)ctx->mlp_params + rbf_align(NPARAM * sizeof(float)));
    const int grid = grid_persistent(ctx->device, (N + SPB - 1) / SPB);
    hipLaunchKernelGGL(k_surrogate, dim3(grid), dim3(256), 0, ctx->stream, p, packed, X, N, offsets, idx, nnz,
                       o.surrogate_tol, o.surrogate_corr_tol, w, status);
    RBF_LAUNCH_CHECK();
    // rejected stencils: the plain float64 solve
    rbf::StencilArgs a;
    a.X = X;
    a.N = N;
    a.d = 2;
    a.P = 2;
    a.offsets = offsets;
    a.idx = idx;
    a.nnz = nnz;
    a.n_max = n_max;
    a.op_mask = RBF_OP_LAP;
    a.phs_power = o.phs_power;
    a.scale_mode = o.scale_mode;
    a.repro_tol = o.repro_tol;
    a.w = w;
    a.status = status;
    if (c->fallback(a, N, RBF_ST_SURROGATE_REJECTED, ctx->stream) != hipSuccess) return RBF_EHIP;
    return RBF_OK;
}
