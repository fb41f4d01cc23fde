// Kernels of the learned candidate ordering: a small MLP encoder whose
// embedding distances predict DK distances.  The encoder never prunes; it
// only orders candidates so that the running k-th best threshold falls
// early (the scan's results do not depend on the order).
//
// Numerics: layer inputs and weights are rounded to bfloat16 (nearest, ties
// to even) where the products read them, products accumulate in fp32 on the
// matrix cores (v_mfma_f32_32x32x16_bf16), biases and activations stay fp32.
// Backward products round their operands the same way.
#pragma once
#include "device.hpp"

namespace tsk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// fp32 -> bfloat16, round to nearest even on the bit pattern (finite inputs)
__device__ __forceinline__ uint16_t bf16_bits(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ __bf16 to_bf16(float f)
{
    return __builtin_bit_cast(__bf16, bf16_bits(f));
}

// Resampling to P points by linear interpolation at t_k = k (L-1) / (P-1):
// one thread per (series, point); out[s][k*D + dim].  The fraction is the
// exact ratio (k (L-1) mod (P-1)) / (P-1), rounded once.
template <int D>
__global__ void k_resample(const float *__restrict__ vals, const int64_t *__restrict__ off,
                           int64_t n, int P, float *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * P)
        return;
    const int64_t s = t / P;
    const int k = (int)(t % P);
    const int64_t o = off[s];
    const int L = (int)(off[s + 1] - o);
    const int64_t num = (int64_t)k * (L - 1);
    const int i0 = (int)(num / (P - 1));
    const float f = (float)(num - (int64_t)i0 * (P - 1)) / (float)(P - 1);
    const int i1 = min(i0 + 1, L - 1);
#pragma unroll
    for (int e = 0; e < D; ++e) {
        const float a = vals[(o + i0) * D + e], b = vals[(o + i1) * D + e];
        out[s * P * D + k * D + e] = a + f * (b - a);
    }
}

// Row gather: out[r] = in[idx[r]] for rows of `width` floats.
static __global__ void k_gather_rows(const float *__restrict__ in, const int32_t *__restrict__ idx,
                                     int64_t rows, int width, float *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * width)
        return;
    const int64_t r = t / width;
    const int c = (int)(t % width);
    out[t] = in[(int64_t)idx[r] * width + c];
}

// C[M x N] = A[M x K] * B[K x N] on bfloat16 operands with fp32 accumulation.
// Element (m, k) of A is A[m*sam + k*sak], (k, n) of B is B[k*sbk + n*sbn]
// (fp32 in memory, rounded when loaded), so transposed operands need no
// copies.  Epilogue per element: + bias[n], ReLU, zero where mask[m][n] <= 0
// (the backward pass through a ReLU), in that order; C row-major (ldc).
// One wave per 32 x 32 tile, four tiles (2 x 2) per block of 256.
struct GemmArgs {
    const float *A;
    int64_t sam, sak;
    const float *B;
    int64_t sbk, sbn;
    float *C;
    int64_t ldc;
    int M, N, K;
    const float *bias; // [N] or null
    int relu;
    const float *mask; // [M][ldm] or null
    int64_t ldm;
};

__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g);

// Loss of a batch of pairs: rows [0, n) of E are the first members, rows
// [n, 2n) the second.  pred = ||e_a - e_b||, loss = mean (pred - y)^2;
// dE holds the loss gradient of every row; loss_out accumulates the sum of
// squared errors / n.  One wave per pair.
__global__ __launch_bounds__(64) void k_pair_loss(const float *__restrict__ E, int width,
                                                  const float *__restrict__ y, int64_t n,
                                                  float *__restrict__ dE, float *loss_out);

// Column sums: out[c] = sum over rows of G[r][c] (bias gradients).
__global__ void k_colsum(const float *__restrict__ G, int64_t rows, int cols,
                         float *__restrict__ out);

// Adam on the fp32 master parameters; c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t).
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2);

// Squared embedding distance of every (query, candidate):
// S[q][c] = sum_e (Eq[q][e] - Ec[c][e])^2, one thread per candidate, the
// group's query embeddings in LDS.
__global__ __launch_bounds__(256) void k_embed_score(const float *__restrict__ Eq, int nq,
                                                     const float *__restrict__ Ec, int64_t N,
                                                     int width, float *__restrict__ S);

// Candidate order of each query by ascending score: a counting sort on the
// top bits of the (non-negative) fp32 score, 2^-5 relative bucket width
// (bucket-mates in arbitrary order: any permutation keeps the scan exact).
// One block of 1024 per query, ORDER_BUCKETS counters in dynamic LDS.
constexpr int ORDER_BUCKETS = 8192;
constexpr int ORDER_SHIFT = 18;
__global__ __launch_bounds__(1024) void k_bucket_order(const float *__restrict__ S, int64_t N,
                                                       int32_t *__restrict__ order);

} // namespace tsk
