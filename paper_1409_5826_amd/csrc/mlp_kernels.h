// Learned step proposer: a 166 -> 128 -> 128 -> 1 ReLU perceptron run on the
// gfx950 matrix cores (v_mfma_f32_16x16x32_bf16: BF16 operands, FP32
// accumulation).  The network maps features of a zone's accepted state to o,
// the predicted log2 of the ratio of the next accepted step to the last one.
//
// Rounding points (the CPU reference rounds at the same places):
//   forward   xb = bf16(x), Wb = bf16(W), a1 = xb W1b + b1, h1b = bf16(relu(a1)),
//             a2 = h1b W2b + b2, h2b = bf16(relu(a2)), o = h2b W3b + b3
//   backward  g_o = 2 (o - y)/B, g_ob = bf16(g_o); dW3 = h2b^T g_ob; db3 = sum g_o;
//             g_a2 = g_ob W3b^T [a2 > 0], g_a2b = bf16(g_a2); dW2 = h1b^T g_a2b; db2 = sum g_a2;
//             g_a1 = (g_a2b W2b^T) [a1 > 0], g_a1b = bf16(g_a1); dW1 = xb^T g_a1b; db1 = sum g_a1
//   Adam on FP32 master weights.
//
// MFMA operand layout used here (16x16 output tile per wave, K = 32 per
// instruction): lane l feeds row (l % 16) of A and column (l % 16) of B with
// the 8 consecutive k values 8*(l/16) .. 8*(l/16)+7; it receives column
// (l % 16), rows 4*(l/16) .. 4*(l/16)+3 of the accumulator.  A and B use the
// same k assignment, so the product does not depend on how the hardware
// orders k inside the instruction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace asynet {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMlpIn = 166;
constexpr int kMlpInPad = 192;
constexpr int kMlpHid = 128;
// flat parameter layout: W1 [192][128], b1 [128], W2 [128][128], b2 [128], W3 [128], b3 [1]
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpInPad * kMlpHid;
constexpr int kOffW2 = kOffB1 + kMlpHid;
constexpr int kOffB2 = kOffW2 + kMlpHid * kMlpHid;
constexpr int kOffW3 = kOffB2 + kMlpHid;
constexpr int kOffB3 = kOffW3 + kMlpHid;
constexpr int kMlpParams = kOffB3 + 1;

// float -> bfloat16 bits, round to nearest, ties to even (NaN stays NaN)
__host__ __device__ inline uint16_t f32_to_bf16_bits(float f)
{
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u)
        return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__host__ __device__ inline float bf16_bits_to_f32(uint16_t b)
{
    const uint32_t u = (uint32_t)b << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

__device__ inline bf16x8 pack_bf16x8(const uint16_t v[8])
{
    uint4 w;
    w.x = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
    w.y = (uint32_t)v[2] | ((uint32_t)v[3] << 16);
    w.z = (uint32_t)v[4] | ((uint32_t)v[5] << 16);
    w.w = (uint32_t)v[6] | ((uint32_t)v[7] << 16);
    return __builtin_bit_cast(bf16x8, w);
}

// Epilogues of gemm_bf16_kernel
enum GemmEpilogue : int {
    kEpiStore = 0,    // C32 = acc (+ bias[n] when bias != nullptr)
    kEpiForward = 1,  // C32 = acc + bias[n]; Cb = bf16(relu(C32))
    kEpiReluGrad = 2, // v = acc * (pre[m][n] > 0); C32 = v; Cb = bf16(v)
};

// C[M][N] = op(A)[M][K] op(B)[K][N]; A, B are bfloat16 bits, C FP32 (and/or BF16).
// Element (m, k) of A is A[TA ? k*lda + m : m*lda + k]; (k, n) of B is B[TB ? n*ldb + k : k*ldb + n].
// M and N are multiples of 16, K a multiple of 32 (callers zero-pad); columns
// n >= n_store are not written.  One wave per 16x16 tile.
template <bool TA, bool TB>
__global__ void __launch_bounds__(256)
gemm_bf16_kernel(int M, int N, int K, const uint16_t *A, int lda, const uint16_t *B, int ldb,
                 float *C32, uint16_t *Cb, int ldc, const float *bias, const float *pre, int epi,
                 int n_store)
{
    const int lane = threadIdx.x % 64;
    const int tile = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    const int tiles_n = N / 16;
    if (tile >= (M / 16) * tiles_n)
        return;
    const int tm = tile / tiles_n, tn = tile % tiles_n;
    const int m = tm * 16 + lane % 16;
    const int n = tn * 16 + lane % 16;
    const int kg = (lane / 16) * 8;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < K; k0 += 32) {
        uint16_t a[8], b[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = k0 + kg + e;
            a[e] = TA ? A[(size_t)k * lda + m] : A[(size_t)m * lda + k];
            b[e] = TB ? B[(size_t)n * ldb + k] : B[(size_t)k * ldb + n];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pack_bf16x8(a), pack_bf16x8(b), acc, 0, 0, 0);
    }
    if (n >= n_store)
        return;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int mo = tm * 16 + (lane / 16) * 4 + e;
        float v = acc[e];
        const size_t at = (size_t)mo * ldc + n;
        if (epi == kEpiStore) {
            if (bias)
                v += bias[n];
            C32[at] = v;
        } else if (epi == kEpiForward) {
            v += bias[n];
            C32[at] = v;
            Cb[at] = f32_to_bf16_bits(v > 0.0f ? v : 0.0f);
        } else {
            v = pre[at] > 0.0f ? v : 0.0f;
            C32[at] = v;
            Cb[at] = f32_to_bf16_bits(v);
        }
    }
}

// Weight gradients C[M][N] = A^T[M][K] B[K][N] (A stored [K][M], B [K][N], bfloat16 bits,
// K = the batch, a multiple of 32): one 16x16 tile per workgroup of 4 waves.  Wave w multiplies
// the k-steps of 32 with index w, w + 4, w + 8, ... into its own accumulator; the four are added
// in wave order through LDS -- a fixed order, so the result is deterministic -- and stored.  The
// batch dimension is long and the tiles few (96 and 64), so splitting it is what fills the chip.
__global__ void __launch_bounds__(256)
gemm_bf16_wgrad_kernel(int M, int N, int K, const uint16_t *A, int lda, const uint16_t *B, int ldb,
                       float *C, int ldc)
{
    __shared__ float red[4][16][16];
    const int lane = threadIdx.x % 64;
    const int wave = threadIdx.x / 64;
    const int tiles_n = N / 16;
    const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
    const int m = tm * 16 + lane % 16;
    const int n = tn * 16 + lane % 16;
    const int kg = (lane / 16) * 8;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 32 * wave; k0 < K; k0 += 128) {
        uint16_t a[8], b[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = k0 + kg + e;
            a[e] = A[(size_t)k * lda + m];
            b[e] = B[(size_t)k * ldb + n];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pack_bf16x8(a), pack_bf16x8(b), acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
        red[wave][(lane / 16) * 4 + e][lane % 16] = acc[e];
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = (lane / 16) * 4 + e;
            const float v = ((red[0][r][lane % 16] + red[1][r][lane % 16]) + red[2][r][lane % 16]) +
                            red[3][r][lane % 16];
            C[(size_t)(tm * 16 + r) * ldc + n] = v;
        }
    }
}

// x [n][166] FP32 -> xb [n_pad][192] bf16 bits; padding columns and rows n..n_pad-1 are zero
__global__ void mlp_pack_input_kernel(int n, int n_pad, const float *x, uint16_t *xb)
{
    const size_t total = (size_t)n_pad * kMlpInPad;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t b = i / kMlpInPad;
        const int c = (int)(i % kMlpInPad);
        xb[i] = (c < kMlpIn && (int)b < n) ? f32_to_bf16_bits(x[b * kMlpIn + c]) : (uint16_t)0;
    }
}

// bf16 copies of the masters: W1b [192][128], W2b [128][128], W3b [128][16] (column 0 = W3)
__global__ void mlp_cast_weights_kernel(const float *p, uint16_t *W1b, uint16_t *W2b, uint16_t *W3b)
{
    const int total = kMlpInPad * kMlpHid + kMlpHid * kMlpHid + kMlpHid * 16;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        if (i < kMlpInPad * kMlpHid) {
            W1b[i] = f32_to_bf16_bits(p[kOffW1 + i]);
        } else if (i < kMlpInPad * kMlpHid + kMlpHid * kMlpHid) {
            const int j = i - kMlpInPad * kMlpHid;
            W2b[j] = f32_to_bf16_bits(p[kOffW2 + j]);
        } else {
            const int j = i - kMlpInPad * kMlpHid - kMlpHid * kMlpHid;
            W3b[j] = (j % 16 == 0) ? f32_to_bf16_bits(p[kOffW3 + j / 16]) : (uint16_t)0;
        }
    }
}

// o = column 0 of out [n][16]; g_o = 2 (o - y)/n; g_ob = bf16(g_o); loss = mean (o - y)^2.
// One workgroup of 1024 threads.
__global__ void __launch_bounds__(1024)
mlp_loss_kernel(int n, int n_pad, const float *out16, const float *y, float *o, float *g_o,
                uint16_t *g_ob, float *loss)
{
    __shared__ float part[1024];
    float s = 0.0f;
    for (int b = threadIdx.x; b < n_pad; b += blockDim.x) {
        if (b >= n) {  // padding rows carry no gradient
            if (y) {
                g_o[b] = 0.0f;
                g_ob[b] = 0;
            }
            continue;
        }
        const float ob = out16[(size_t)b * 16];
        if (o)
            o[b] = ob;
        if (y) {
            const float d = ob - y[b];
            s += d * d;
            const float g = 2.0f * d / (float)n;
            g_o[b] = g;
            g_ob[b] = f32_to_bf16_bits(g);
        }
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && y && loss)
        loss[0] = part[0] / (float)n;
}

// g_a2[b][j] = g_ob[b] W3b[j] [a2 > 0] (an outer product: exact in FP32), g_a2b = bf16(g_a2)
__global__ void mlp_out_grad_kernel(int n, const uint16_t *g_ob, const uint16_t *W3b, const float *a2,
                                    float *g_a2, uint16_t *g_a2b)
{
    const size_t total = (size_t)n * kMlpHid;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t b = i / kMlpHid;
        const int j = (int)(i % kMlpHid);
        float v = bf16_bits_to_f32(g_ob[b]) * bf16_bits_to_f32(W3b[j * 16]);
        v = a2[i] > 0.0f ? v : 0.0f;
        g_a2[i] = v;
        g_a2b[i] = f32_to_bf16_bits(v);
    }
}

// dW3[j] = sum_b h2b[b][j] g_ob[b] and the bias gradients (column sums), FP32.
// Column sums over the batch (the bias gradients, the output layer's weight gradient and b3's
// gradient) in two kernels.  Workgroup q of mlp_colsum_part_kernel (kColsumGroups x 128
// threads) takes the rows [q rows_per, (q + 1) rows_per): thread (g, j) sums rows r0 + g,
// r0 + g + kColsumGroups, ... of column j (coalesced across j), the group partials are added in
// group order, and the workgroup writes part[q][4][128] (b1, b2, W3 columns; b3 in [3][0]).
// mlp_colsum_final_kernel adds the workgroups' partials in workgroup order.  Every order is
// fixed, so the result is deterministic.
constexpr int kColsumGroups = 8;
constexpr int kColsumBlocks = 16;

__global__ void __launch_bounds__(kColsumGroups * kMlpHid)
mlp_colsum_part_kernel(int n, int rows_per, const float *g_a1, const float *g_a2, const float *g_o,
                       const uint16_t *h2b, const uint16_t *g_ob, float *part)
{
    __shared__ float grp[4][kColsumGroups][kMlpHid];
    const int j = threadIdx.x % kMlpHid;
    const int g = threadIdx.x / kMlpHid;
    const int r0 = blockIdx.x * rows_per;
    const int r1 = min(n, r0 + rows_per);
    float s1 = 0.0f, s2 = 0.0f, s3 = 0.0f, s4 = 0.0f;
    for (int b = r0 + g; b < r1; b += kColsumGroups) {
        const size_t at = (size_t)b * kMlpHid + j;
        const float go = bf16_bits_to_f32(g_ob[b]);
        s1 += g_a1[at];
        s2 += g_a2[at];
        s3 += bf16_bits_to_f32(h2b[at]) * go;
        if (j == 0)
            s4 += g_o[b];
    }
    grp[0][g][j] = s1;
    grp[1][g][j] = s2;
    grp[2][g][j] = s3;
    grp[3][g][j] = s4;
    __syncthreads();
    if (g == 0) {
        float t1 = 0.0f, t2 = 0.0f, t3 = 0.0f, t4 = 0.0f;
        for (int q = 0; q < kColsumGroups; ++q) {
            t1 += grp[0][q][j];
            t2 += grp[1][q][j];
            t3 += grp[2][q][j];
            t4 += grp[3][q][j];
        }
        float *out = part + (size_t)blockIdx.x * 4 * kMlpHid;
        out[j] = t1;
        out[kMlpHid + j] = t2;
        out[2 * kMlpHid + j] = t3;
        out[3 * kMlpHid + j] = t4;  // only column 0 carries b3's partial
    }
}

__global__ void __launch_bounds__(kMlpHid)
mlp_colsum_final_kernel(int blocks, const float *part, float *grad)
{
    const int j = threadIdx.x;
    float t1 = 0.0f, t2 = 0.0f, t3 = 0.0f, t4 = 0.0f;
    for (int q = 0; q < blocks; ++q) {
        const float *in = part + (size_t)q * 4 * kMlpHid;
        t1 += in[j];
        t2 += in[kMlpHid + j];
        t3 += in[2 * kMlpHid + j];
        t4 += in[3 * kMlpHid];
    }
    grad[kOffB1 + j] = t1;
    grad[kOffB2 + j] = t2;
    grad[kOffW3 + j] = t3;
    if (j == 0)
        grad[kOffB3] = t4;
}

// Adam on the FP32 masters; c1 = 1 - beta1^t, c2 = 1 - beta2^t.  The gradients of b1, b2, W3 and
// b3 come straight from the column-sum partials part[blocks][4][128], added in workgroup order as
// mlp_colsum_final_kernel adds them (the same values), and every updated weight is written to its
// BF16 copy as mlp_cast_weights_kernel writes it (W1b, W2b, column 0 of W3b), so a training step
// needs neither of those two kernels.
__global__ void mlp_adam_kernel(float *p, const float *g, const float *part, int blocks, float *m,
                                float *v, uint16_t *W1b, uint16_t *W2b, uint16_t *W3b, float lr,
                                float beta1, float beta2, float eps, float c1, float c2)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kMlpParams; i += gridDim.x * blockDim.x) {
        // which column sum holds this parameter's gradient (-1: g holds it)
        int sum = -1, j = 0;
        if (i >= kOffB1 && i < kOffB1 + kMlpHid) {
            sum = 0;
            j = i - kOffB1;
        } else if (i >= kOffB2 && i < kOffB2 + kMlpHid) {
            sum = 1;
            j = i - kOffB2;
        } else if (i >= kOffW3 && i < kOffW3 + kMlpHid) {
            sum = 2;
            j = i - kOffW3;
        } else if (i == kOffB3) {
            sum = 3;
        }
        float gi;
        if (sum >= 0) {
            gi = 0.0f;
            for (int q = 0; q < blocks; ++q)
                gi += part[(size_t)q * 4 * kMlpHid + sum * kMlpHid + j];
        } else {
            gi = g[i];
        }
        const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
        const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pn = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        p[i] = pn;
        if (i < kOffB1)
            W1b[i - kOffW1] = f32_to_bf16_bits(pn);
        else if (i >= kOffW2 && i < kOffB2)
            W2b[i - kOffW2] = f32_to_bf16_bits(pn);
        else if (sum == 2)
            W3b[j * 16] = f32_to_bf16_bits(pn);
    }
}

// ---- inference inside the integrator ---------------------------------------------------------

// Weights for in-kernel inference, pre-arranged so that every lane reads the 8
// bf16 values of its MFMA B-fragment with one 16-byte load:
//   w1s[((tn * 6 + kk) * 64 + lane) * 8 + e] = W1[32 kk + 8 (lane/16) + e][16 tn + lane % 16]
//   w2s[((tn * 4 + kk) * 64 + lane) * 8 + e] = W2[32 kk + 8 (lane/16) + e][16 tn + lane % 16]
//   w3s[(kk * 64 + lane) * 8 + e]            = W3[32 kk + 8 (lane/16) + e] for lane % 16 == 0, else 0
struct MlpDevice {
    const uint16_t *w1s;
    const uint16_t *w2s;
    const uint16_t *w3s;
    const float *b1;
    const float *b2;
    float b3;
};

// The W waves of a workgroup evaluate the network for one feature vector x
// (kMlpInPad floats in LDS, zero padded) together.  Wave w computes the
// 16-column output tiles w, w + W, ... of each hidden layer and keeps the
// weights of its next tile in flight while it multiplies the current one; the
// hidden activations go to LDS (h1, h2: kMlpHid floats each) between the
// layers, and wave 0 computes the output and leaves it in *o_slot (LDS).
// sync() is a barrier of the W waves.  Only row 0 of each 16-row A tile
// carries data.  Every tile sums its k-fragments in the same order whichever
// wave computes it, so the result does not depend on W.  Returns o in every
// lane of every wave.
template <int W, typename Sync>
__device__ inline float mlp_infer_group(const MlpDevice &w, const float *x, float *h1, float *h2,
                                        float *o_slot, int lane, int wave, Sync sync)
{
    static_assert(8 % W == 0, "the 8 output tiles split evenly over the waves");
    constexpr int TPW = 8 / W;
    const bool row0 = (lane % 16) == 0;
    const int kg = (lane / 16) * 8;
    auto frag = [&](const float *src, int kk) {
        uint16_t a[8];
#pragma unroll
        for (int e = 0; e < 8; ++e)
            a[e] = row0 ? f32_to_bf16_bits(src[32 * kk + kg + e]) : (uint16_t)0;
        return pack_bf16x8(a);
    };
    // weights and biases through buffer resources: the lane's offset is one register and a
    // fragment's offset a scalar (the wave index is uniform), so no 64-bit address per load
    // is computed, kept or spilled, and a tile's loads issue together
    auto rsrc = [](const void *p, int bytes) {
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, bytes, 0x00020000);
    };
    const __amdgpu_buffer_rsrc_t rw1 = rsrc(w.w1s, 8 * 6 * 64 * 16);
    const __amdgpu_buffer_rsrc_t rw2 = rsrc(w.w2s, 8 * 4 * 64 * 16);
    const __amdgpu_buffer_rsrc_t rw3 = rsrc(w.w3s, 4 * 64 * 16);
    const __amdgpu_buffer_rsrc_t rb1 = rsrc(w.b1, kMlpHid * 4);
    const __amdgpu_buffer_rsrc_t rb2 = rsrc(w.b2, kMlpHid * 4);
    auto ld = [&](__amdgpu_buffer_rsrc_t r, int tile_frag) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, lane * 16, tile_frag * 1024, 0);
        return uint4{v[0], v[1], v[2], v[3]};
    };
    // bias of column 16 tn + lane (lanes 0..15)
    auto bias = [&](__amdgpu_buffer_rsrc_t r, int tn) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, lane * 4, tn * 64, 0));
    };
    // layer 1
    {
        bf16x8 af[6];
#pragma unroll
        for (int kk = 0; kk < 6; ++kk)
            af[kk] = frag(x, kk);
        uint4 nb[6];
#pragma unroll
        for (int kk = 0; kk < 6; ++kk)
            nb[kk] = ld(rw1, wave * 6 + kk);
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            const int tn = wave + t * W;
            uint4 cb[6];
#pragma unroll
            for (int kk = 0; kk < 6; ++kk)
                cb[kk] = nb[kk];
            if (t + 1 < TPW) {
#pragma unroll
                for (int kk = 0; kk < 6; ++kk)
                    nb[kk] = ld(rw1, (tn + W) * 6 + kk);
            }
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kk = 0; kk < 6; ++kk)
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[kk], __builtin_bit_cast(bf16x8, cb[kk]),
                                                              acc, 0, 0, 0);
            // row 0 of the tile sits in lanes 0..15, element 0
            if (lane < 16) {
                const float v = acc[0] + bias(rb1, tn);
                h1[16 * tn + lane] = bf16_bits_to_f32(f32_to_bf16_bits(v > 0.0f ? v : 0.0f));
            }
        }
    }
    sync();
    // layer 2
    {
        bf16x8 af[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
            af[kk] = frag(h1, kk);
        uint4 nb[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
            nb[kk] = ld(rw2, wave * 4 + kk);
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            const int tn = wave + t * W;
            uint4 cb[4];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                cb[kk] = nb[kk];
            if (t + 1 < TPW) {
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    nb[kk] = ld(rw2, (tn + W) * 4 + kk);
            }
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[kk], __builtin_bit_cast(bf16x8, cb[kk]),
                                                              acc, 0, 0, 0);
            if (lane < 16) {
                const float v = acc[0] + bias(rb2, tn);
                h2[16 * tn + lane] = bf16_bits_to_f32(f32_to_bf16_bits(v > 0.0f ? v : 0.0f));
            }
        }
    }
    sync();
    // layer 3
    if (wave == 0) {
        uint4 b3w[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
            b3w[kk] = ld(rw3, kk);
        f32x4 acc3 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
            acc3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag(h2, kk), __builtin_bit_cast(bf16x8, b3w[kk]),
                                                           acc3, 0, 0, 0);
        if (lane == 0)
            *o_slot = acc3[0] + w.b3;
    }
    sync();
    return *o_slot;
}

// Barrier of one wave: LDS operations of a wave complete in order; this only
// keeps the compiler from moving LDS accesses across it.
struct WaveSync {
    __device__ void operator()() const
    {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
};

// Arrange the bf16 weights for mlp_infer_group (see MlpDevice).
__global__ void mlp_swizzle_kernel(const float *p, uint16_t *w1s, uint16_t *w2s, uint16_t *w3s)
{
    const int n1 = 8 * 6 * 64 * 8, n2 = 8 * 4 * 64 * 8, n3 = 4 * 64 * 8;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n1 + n2 + n3; i += gridDim.x * blockDim.x) {
        if (i < n1) {
            const int e = i % 8, lane = (i / 8) % 64, kk = (i / 512) % 6, tn = i / (512 * 6);
            const int k = 32 * kk + 8 * (lane / 16) + e, n = 16 * tn + lane % 16;
            w1s[i] = f32_to_bf16_bits(p[kOffW1 + k * kMlpHid + n]);
        } else if (i < n1 + n2) {
            const int j = i - n1;
            const int e = j % 8, lane = (j / 8) % 64, kk = (j / 512) % 4, tn = j / (512 * 4);
            const int k = 32 * kk + 8 * (lane / 16) + e, n = 16 * tn + lane % 16;
            w2s[j] = f32_to_bf16_bits(p[kOffW2 + k * kMlpHid + n]);
        } else {
            const int j = i - n1 - n2;
            const int e = j % 8, lane = (j / 8) % 64, kk = j / 512;
            const int k = 32 * kk + 8 * (lane / 16) + e;
            w3s[j] = (lane % 16 == 0) ? f32_to_bf16_bits(p[kOffW3 + k]) : (uint16_t)0;
        }
    }
}

// Standalone batched inference with the in-kernel routine (one wave per sample);
// used to check the integrator's inference against the training forward pass.
__global__ void __launch_bounds__(64)
mlp_infer_batch_kernel(int n, const float *x, MlpDevice w, float *o)
{
    __shared__ float xs[kMlpInPad];
    __shared__ float h1[kMlpHid];
    __shared__ float h2[kMlpHid];
    __shared__ float os;
    const int lane = threadIdx.x;
    for (int b = blockIdx.x; b < n; b += gridDim.x) {
        for (int c = lane; c < kMlpInPad; c += 64)
            xs[c] = c < kMlpIn ? x[(size_t)b * kMlpIn + c] : 0.0f;
        WaveSync{}();
        const float ob = mlp_infer_group<1>(w, xs, h1, h2, &os, lane, 0, WaveSync{});
        if (lane == 0)
            o[b] = ob;
        WaveSync{}();
    }
}

}  // namespace asynet
