// The learned candidate ordering: encoder kernels (bf16 matrix-core
// products, loss, Adam, scores, bucket order) and the tsk_model C-ABI.
// Not part of the paper's method: the encoder only reorders candidates,
// so the scan's results never depend on it.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstring>
#include <vector>

#include "kernels_mlp.hpp"
#include "model.hpp"
#include "runtime.hpp"
#include "tsknn.h"

namespace tsk {

// ------------------------------------------------------------------ kernels
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g)
{
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int m0 = (blockIdx.y * 2 + (w >> 1)) * 32;
    const int n0 = (blockIdx.x * 2 + (w & 1)) * 32;
    if (m0 >= g.M || n0 >= g.N)
        return; // the whole wave: its tile is outside C
    // operand layout of v_mfma_f32_32x32x16_bf16: lane l supplies row l%32
    // of A and column l%32 of B at k = 8 (l/32) .. 8 (l/32) + 7
    const int r = lane & 31;
    const int kh = (lane >> 5) * 8;
    const int am = m0 + r, bn = n0 + r;
    const bool arow = am < g.M, bcol = bn < g.N;
    const float *Ap = g.A + (arow ? (int64_t)am * g.sam : 0);
    const float *Bp = g.B + (bcol ? (int64_t)bn * g.sbn : 0);
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i)
        acc[i] = 0.0f;
    for (int k0 = 0; k0 < g.K; k0 += 16) {
        bf16x8 a, b;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = k0 + kh + i;
            const bool kin = k < g.K;
            const float av = (arow && kin) ? Ap[(int64_t)k * g.sak] : 0.0f;
            const float bv = (bcol && kin) ? Bp[(int64_t)k * g.sbk] : 0.0f;
            a[i] = to_bf16(av);
            b[i] = to_bf16(bv);
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    // result layout: element i of lane l is row 8 (i/4) + 4 (l/32) + i%4,
    // column l%32 of the tile
    const int col = n0 + (lane & 31);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int row = m0 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
        if (row < g.M && col < g.N) {
            float v = acc[i];
            if (g.bias)
                v += g.bias[col];
            if (g.relu)
                v = fmaxf(v, 0.0f);
            if (g.mask && !(g.mask[(int64_t)row * g.ldm + col] > 0.0f))
                v = 0.0f;
            g.C[(int64_t)row * g.ldc + col] = v;
        }
    }
}

__global__ __launch_bounds__(64) void k_pair_loss(const float *__restrict__ E, int width,
                                                  const float *__restrict__ y, int64_t n,
                                                  float *__restrict__ dE, float *loss_out)
{
    const int64_t p = blockIdx.x;
    const int lane = threadIdx.x;
    const float *ea = E + p * width, *eb = E + (p + n) * width;
    float ss = 0.0f;
    for (int e = lane; e < width; e += 64) {
        const float d = ea[e] - eb[e];
        ss = __builtin_fmaf(d, d, ss);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        ss += __shfl_xor(ss, o, 64);
    const float pred = sqrtf(ss);
    const float err = pred - y[p];
    const float gs = 2.0f * err / (float)n;
    const float f = pred > 0.0f ? gs / pred : 0.0f;
    for (int e = lane; e < width; e += 64) {
        const float d = ea[e] - eb[e];
        dE[p * width + e] = f * d;
        dE[(p + n) * width + e] = -(f * d);
    }
    if (lane == 0)
        atomicAdd(loss_out, err * err / (float)n);
}

__global__ void k_colsum(const float *__restrict__ G, int64_t rows, int cols,
                         float *__restrict__ out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols)
        return;
    float s = 0.0f;
    for (int64_t r = 0; r < rows; ++r)
        s += G[r * cols + c];
    out[c] = s;
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * (gi * gi);
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

static __global__ void k_zero_f32(float *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0.0f;
}

constexpr int SCORE_QG = 8;

__global__ __launch_bounds__(256) void k_embed_score(const float *__restrict__ Eq, int nq,
                                                     const float *__restrict__ Ec, int64_t N,
                                                     int width, float *__restrict__ S)
{
    __shared__ float qe[SCORE_QG * 256];
    const int q0 = blockIdx.y * SCORE_QG;
    const int nqg = min(SCORE_QG, nq - q0);
    for (int i = threadIdx.x; i < nqg * width; i += blockDim.x)
        qe[i] = Eq[(int64_t)q0 * width + i];
    __syncthreads();
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N)
        return;
    float acc[SCORE_QG];
#pragma unroll
    for (int g = 0; g < SCORE_QG; ++g)
        acc[g] = 0.0f;
    const float *ec = Ec + c * width;
    for (int e = 0; e < width; ++e) {
        const float x = ec[e];
#pragma unroll
        for (int g = 0; g < SCORE_QG; ++g) {
            const float d = qe[(g < nqg ? g : 0) * width + e] - x;
            acc[g] = __builtin_fmaf(d, d, acc[g]);
        }
    }
#pragma unroll
    for (int g = 0; g < SCORE_QG; ++g)
        if (g < nqg)
            S[(int64_t)(q0 + g) * N + c] = acc[g];
}

__global__ __launch_bounds__(1024) void k_bucket_order(const float *__restrict__ S, int64_t N,
                                                       int32_t *__restrict__ order)
{
    extern __shared__ int32_t hist[]; // ORDER_BUCKETS counters, then cursors
    __shared__ int32_t wsum[16];
    const int64_t q = blockIdx.x;
    const float *s = S + q * N;
    const int tid = threadIdx.x;
    for (int b = tid; b < ORDER_BUCKETS; b += 1024)
        hist[b] = 0;
    __syncthreads();
    for (int64_t c = tid; c < N; c += 1024) {
        const uint32_t key = min(__float_as_uint(s[c]) >> ORDER_SHIFT, (uint32_t)ORDER_BUCKETS - 1);
        atomicAdd(&hist[key], 1);
    }
    __syncthreads();
    // exclusive scan: 8 consecutive buckets per thread, then the threads
    constexpr int PER = ORDER_BUCKETS / 1024;
    int loc[PER];
    int tot = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        loc[i] = tot;
        tot += hist[tid * PER + i];
    }
    const int lane = tid & 63, wv = tid >> 6;
    int inc = tot; // inclusive scan of the thread totals inside the wave
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(inc, o, 64);
        if (lane >= o)
            inc += t;
    }
    if (lane == 63)
        wsum[wv] = inc;
    __syncthreads();
    int base = 0;
    for (int w = 0; w < wv; ++w)
        base += wsum[w];
    const int excl = base + inc - tot;
    __syncthreads(); // every thread has read its buckets' counts
#pragma unroll
    for (int i = 0; i < PER; ++i)
        hist[tid * PER + i] = excl + loc[i];
    __syncthreads();
    for (int64_t c = tid; c < N; c += 1024) {
        const uint32_t key = min(__float_as_uint(s[c]) >> ORDER_SHIFT, (uint32_t)ORDER_BUCKETS - 1);
        const int pos = atomicAdd(&hist[key], 1);
        order[q * N + pos] = (int32_t)c;
    }
}

// ------------------------------------------------------------------ launches
namespace {

int grid1(int64_t n, int block) { return (int)((n + block - 1) / block); }

void gemm(const GemmArgs &g, hipStream_t s)
{
    dim3 grid((unsigned)((g.N + 63) / 64), (unsigned)((g.M + 63) / 64));
    hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, s, g);
}

GemmArgs gemm_args(const float *A, int64_t sam, int64_t sak, const float *B, int64_t sbk,
                   int64_t sbn, float *C, int64_t ldc, int M, int N, int K)
{
    GemmArgs g;
    g.A = A;
    g.sam = sam;
    g.sak = sak;
    g.B = B;
    g.sbk = sbk;
    g.sbn = sbn;
    g.C = C;
    g.ldc = ldc;
    g.M = M;
    g.N = N;
    g.K = K;
    g.bias = nullptr;
    g.relu = 0;
    g.mask = nullptr;
    g.ldm = 0;
    return g;
}

void resample(int D, const float *vals, const int64_t *off, int64_t n, int P, float *out,
              hipStream_t s)
{
    const dim3 grid(grid1(n * P, 256)), block(256);
    switch (D) {
    case 1: hipLaunchKernelGGL(k_resample<1>, grid, block, 0, s, vals, off, n, P, out); break;
    case 2: hipLaunchKernelGGL(k_resample<2>, grid, block, 0, s, vals, off, n, P, out); break;
    case 3: hipLaunchKernelGGL(k_resample<3>, grid, block, 0, s, vals, off, n, P, out); break;
    case 4: hipLaunchKernelGGL(k_resample<4>, grid, block, 0, s, vals, off, n, P, out); break;
    case 5: hipLaunchKernelGGL(k_resample<5>, grid, block, 0, s, vals, off, n, P, out); break;
    case 6: hipLaunchKernelGGL(k_resample<6>, grid, block, 0, s, vals, off, n, P, out); break;
    case 7: hipLaunchKernelGGL(k_resample<7>, grid, block, 0, s, vals, off, n, P, out); break;
    case 8: hipLaunchKernelGGL(k_resample<8>, grid, block, 0, s, vals, off, n, P, out); break;
    default: break;
    }
}

// Forward pass of `rows` input rows: a1, a2 = post-ReLU hidden layers, e =
// embeddings.
void forward(tsk_model *mdl, const float *x, int64_t rows, float *a1, float *a2, float *e,
             hipStream_t s)
{
    const float *P = mdl->params.p;
    const int H = mdl->hidden, I = mdl->d_in, O = mdl->embed;
    GemmArgs g = gemm_args(x, I, 1, P + mdl->off[0], 1, I, a1, H, (int)rows, H, I);
    g.bias = P + mdl->off[1];
    g.relu = 1;
    gemm(g, s);
    g = gemm_args(a1, H, 1, P + mdl->off[2], 1, H, a2, H, (int)rows, H, H);
    g.bias = P + mdl->off[3];
    g.relu = 1;
    gemm(g, s);
    g = gemm_args(a2, H, 1, P + mdl->off[4], 1, H, e, O, (int)rows, O, H);
    g.bias = P + mdl->off[5];
    gemm(g, s);
}

// Backward pass for upstream gradient de [rows][embed]: parameter gradients
// into mdl->grads.
void backward(tsk_model *mdl, const float *x, int64_t rows, const float *a1, const float *a2,
              const float *de, hipStream_t s)
{
    const float *P = mdl->params.p;
    float *G = mdl->grads.p;
    const int H = mdl->hidden, I = mdl->d_in, O = mdl->embed;
    const int R = (int)rows;
    float *g2 = mdl->g2.p, *g1 = mdl->g1.p;
    // layer 3: dW3 = de^T a2, db3 = colsum(de), g2 = (de W3) * [a2 > 0]
    gemm(gemm_args(de, 1, O, a2, H, 1, G + mdl->off[4], H, O, H, R), s);
    hipLaunchKernelGGL(k_colsum, dim3(grid1(O, 256)), dim3(256), 0, s, de, rows, O, G + mdl->off[5]);
    GemmArgs g = gemm_args(de, O, 1, P + mdl->off[4], H, 1, g2, H, R, H, O);
    g.mask = a2;
    g.ldm = H;
    gemm(g, s);
    // layer 2
    gemm(gemm_args(g2, 1, H, a1, H, 1, G + mdl->off[2], H, H, H, R), s);
    hipLaunchKernelGGL(k_colsum, dim3(grid1(H, 256)), dim3(256), 0, s, g2, rows, H, G + mdl->off[3]);
    g = gemm_args(g2, H, 1, P + mdl->off[2], H, 1, g1, H, R, H, H);
    g.mask = a1;
    g.ldm = H;
    gemm(g, s);
    // layer 1
    gemm(gemm_args(g1, 1, H, x, I, 1, G + mdl->off[0], I, H, I, R), s);
    hipLaunchKernelGGL(k_colsum, dim3(grid1(H, 256)), dim3(256), 0, s, g1, rows, H, G + mdl->off[1]);
}

int ensure_batch(tsk_model *mdl, int64_t rows)
{
    TSK_TRY(mdl->x.ensure((size_t)rows * mdl->d_in));
    TSK_TRY(mdl->a1.ensure((size_t)rows * mdl->hidden));
    TSK_TRY(mdl->a2.ensure((size_t)rows * mdl->hidden));
    TSK_TRY(mdl->e.ensure((size_t)rows * mdl->embed));
    TSK_TRY(mdl->de.ensure((size_t)rows * mdl->embed));
    TSK_TRY(mdl->g2.ensure((size_t)rows * mdl->hidden));
    TSK_TRY(mdl->g1.ensure((size_t)rows * mdl->hidden));
    return TSK_OK;
}


uint64_t splitmix64(uint64_t &x)
{
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

std::atomic<uint64_t> g_model_uid{0};

void set_offsets(tsk_model *m)
{
    const int64_t H = m->hidden, I = m->d_in, O = m->embed;
    const int64_t sz[6] = {H * I, H, H * H, H, O * H, O};
    m->off[0] = 0;
    for (int i = 0; i < 6; ++i)
        m->off[i + 1] = m->off[i] + sz[i];
    m->n_params = m->off[6];
}

int check_model(const tsk_model *m)
{
    if (!m)
        return set_err(TSK_ERR_INVALID_ARG, "model is NULL");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != m->device)
        return set_err(TSK_ERR_INVALID_ARG, "current device %d differs from the model's %d", dev,
                       m->device);
    return TSK_OK;
}

int check_offsets(const int64_t *off, int64_t n)
{
    if (!off)
        return set_err(TSK_ERR_INVALID_ARG, "offsets are NULL");
    if (n < 1 || n > INT32_MAX)
        return set_err(TSK_ERR_INVALID_ARG, "series count %lld out of range", (long long)n);
    if (off[0] != 0)
        return set_err(TSK_ERR_INVALID_ARG, "offsets[0] must be 0");
    for (int64_t i = 0; i < n; ++i)
        if (off[i + 1] - off[i] < 1 || off[i + 1] - off[i] > TSK_MAX_LEN)
            return set_err(TSK_ERR_INVALID_ARG, "series %lld has length %lld", (long long)i,
                           (long long)(off[i + 1] - off[i]));
    return TSK_OK;
}

int create_model(const tsk_mlp_shape &sh, tsk_model **out)
{
    int dev = 0, ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return set_err(TSK_ERR_DEVICE, "no HIP device available");
    }
    HIP_TRY(hipGetDevice(&dev));
    tsk_model *m = new (std::nothrow) tsk_model();
    if (!m)
        return set_err(TSK_ERR_OOM, "host allocation failed");
    m->device = dev;
    m->dim = sh.dim;
    m->points = sh.points;
    m->hidden = sh.hidden;
    m->embed = sh.embed;
    m->d_in = sh.points * sh.dim;
    m->uid = ++g_model_uid;
    set_offsets(m);
    int rc = TSK_OK;
    if ((rc = m->params.ensure(m->n_params)) != TSK_OK || (rc = m->grads.ensure(m->n_params)) ||
        (rc = m->m.ensure(m->n_params)) || (rc = m->v.ensure(m->n_params)) ||
        (rc = m->loss.ensure(1))) {
        delete m;
        return rc;
    }
    if (hipMemset(m->m.p, 0, m->n_params * sizeof(float)) != hipSuccess ||
        hipMemset(m->v.p, 0, m->n_params * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        delete m;
        return set_err(TSK_ERR_DEVICE, "clearing the optimiser state failed");
    }
    *out = m;
    return TSK_OK;
}

int resolve_shape(const tsk_mlp_shape *in, tsk_mlp_shape *sh)
{
    if (!in)
        return set_err(TSK_ERR_INVALID_ARG, "shape is NULL");
    if (in->size != (int64_t)sizeof(tsk_mlp_shape))
        return set_err(TSK_ERR_INVALID_ARG, "shape->size mismatch");
    *sh = *in;
    if (sh->points == 0)
        sh->points = 32;
    if (sh->hidden == 0)
        sh->hidden = 256;
    if (sh->embed == 0)
        sh->embed = 64;
    if (sh->dim < 1 || sh->dim > TSK_MLP_MAX_DIM)
        return set_err(TSK_ERR_UNSUPPORTED, "dim %d outside [1, %d]", sh->dim, TSK_MLP_MAX_DIM);
    if (sh->points < 2 || sh->points > 256)
        return set_err(TSK_ERR_UNSUPPORTED, "points %d outside [2, 256]", sh->points);
    if (sh->hidden < 32 || sh->hidden > 1024 || sh->hidden % 32)
        return set_err(TSK_ERR_UNSUPPORTED, "hidden %d not a multiple of 32 in [32, 1024]",
                       sh->hidden);
    if (sh->embed < 32 || sh->embed > 256 || sh->embed % 32)
        return set_err(TSK_ERR_UNSUPPORTED, "embed %d not a multiple of 32 in [32, 256]",
                       sh->embed);
    return TSK_OK;
}

// Uploads host offsets of n series to the model's scratch.
int upload_offsets(tsk_model *m, const int64_t *off, int64_t n, hipStream_t s)
{
    TSK_TRY(m->off_dev.ensure(n + 1));
    HIP_TRY(hipMemcpyAsync(m->off_dev.p, off, (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    return TSK_OK;
}

// One training step on rows already gathered into mdl->x (2 b rows) with
// targets y [b]: forward, loss (added to *loss_slot), backward.
void grad_step(tsk_model *m, int64_t b, const float *y, float *loss_slot, hipStream_t s)
{
    const int64_t rows = 2 * b;
    forward(m, m->x.p, rows, m->a1.p, m->a2.p, m->e.p, s);
    hipLaunchKernelGGL(k_pair_loss, dim3((unsigned)b), dim3(64), 0, s, m->e.p, m->embed, y, b,
                       m->de.p, loss_slot);
    backward(m, m->x.p, rows, m->a1.p, m->a2.p, m->de.p, s);
}

void gather_pairs(tsk_model *m, const int32_t *ia, const int32_t *ib, int64_t b, hipStream_t s)
{
    const int I = m->d_in;
    hipLaunchKernelGGL(k_gather_rows, dim3(grid1(b * I, 256)), dim3(256), 0, s, m->pool.p, ia, b,
                       I, m->x.p);
    hipLaunchKernelGGL(k_gather_rows, dim3(grid1(b * I, 256)), dim3(256), 0, s, m->pool.p, ib, b,
                       I, m->x.p + b * I);
}

int check_pairs(const int32_t *a, const int32_t *b, const float *y, int64_t np, int64_t n)
{
    if (!a || !b || !y)
        return set_err(TSK_ERR_INVALID_ARG, "pair arrays are NULL");
    if (np < 1 || np > INT32_MAX)
        return set_err(TSK_ERR_INVALID_ARG, "n_pairs %lld out of range", (long long)np);
    for (int64_t i = 0; i < np; ++i) {
        if (a[i] < 0 || a[i] >= n || b[i] < 0 || b[i] >= n)
            return set_err(TSK_ERR_INVALID_ARG, "pair %lld refers to a series outside [0, %lld)",
                           (long long)i, (long long)n);
        if (!std::isfinite(y[i]))
            return set_err(TSK_ERR_INVALID_ARG, "target %lld is not finite", (long long)i);
    }
    return TSK_OK;
}

// Resampled inputs of the whole series set into mdl->pool.
int prepare_pool(tsk_model *m, const float *vals, const int64_t *off, int64_t n, hipStream_t s)
{
    TSK_TRY(upload_offsets(m, off, n, s));
    TSK_TRY(m->pool.ensure((size_t)n * m->d_in));
    resample(m->dim, vals, m->off_dev.p, n, m->points, m->pool.p, s);
    return TSK_OK;
}

} // namespace

int model_reserve_rows(tsk_model *m, int64_t rows) { return ensure_batch(m, rows); }

int model_embed_dev(tsk_model *m, const float *vals, const int64_t *off_dev, int64_t n, float *out,
                    hipStream_t s)
{
    const int64_t chunk = std::min<int64_t>(n, EMBED_CHUNK);
    TSK_TRY(ensure_batch(m, chunk));
    for (int64_t r0 = 0; r0 < n; r0 += chunk) {
        const int64_t rows = std::min<int64_t>(chunk, n - r0);
        resample(m->dim, vals, off_dev + r0, rows, m->points, m->x.p, s);
        forward(m, m->x.p, rows, m->a1.p, m->a2.p, out + r0 * m->embed, s);
    }
    HIP_TRY(hipGetLastError());
    return TSK_OK;
}

void launch_embed_score(const float *Eq, int nq, const float *Ec, int64_t N, int width, float *S,
                        hipStream_t s)
{
    dim3 grid((unsigned)((N + 255) / 256), (unsigned)((nq + SCORE_QG - 1) / SCORE_QG));
    hipLaunchKernelGGL(k_embed_score, grid, dim3(256), 0, s, Eq, nq, Ec, N, width, S);
}

void launch_bucket_order(const float *S, int nq, int64_t N, int32_t *order, hipStream_t s)
{
    hipLaunchKernelGGL(k_bucket_order, dim3(nq), dim3(1024), ORDER_BUCKETS * sizeof(int32_t), s, S,
                       N, order);
}

} // namespace tsk

using namespace tsk;

// ------------------------------------------------------------------ C-ABI
extern "C" int tsk_model_create(const tsk_mlp_shape *shape, uint64_t seed, tsk_model **out)
{
    g_err.clear();
    if (!out)
        return set_err(TSK_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    tsk_mlp_shape sh;
    TSK_TRY(resolve_shape(shape, &sh));
    tsk_model *m = nullptr;
    TSK_TRY(create_model(sh, &m));
    // He-uniform weights from a splitmix64 stream, zero biases
    std::vector<float> h(m->n_params, 0.0f);
    uint64_t st = seed;
    const int64_t fan[3] = {m->d_in, m->hidden, m->hidden};
    for (int l = 0; l < 3; ++l) {
        const double lim = std::sqrt(6.0 / (double)fan[l]);
        for (int64_t i = m->off[2 * l]; i < m->off[2 * l + 1]; ++i) {
            const double u = (double)(splitmix64(st) >> 11) * 0x1.0p-53;
            h[i] = (float)((2.0 * u - 1.0) * lim);
        }
    }
    if (hipMemcpy(m->params.p, h.data(), m->n_params * sizeof(float), hipMemcpyHostToDevice) !=
        hipSuccess) {
        (void)hipGetLastError();
        delete m;
        return set_err(TSK_ERR_DEVICE, "uploading the initial parameters failed");
    }
    *out = m;
    return TSK_OK;
}

extern "C" int tsk_model_free(tsk_model *m)
{
    if (!m)
        return TSK_OK;
    (void)hipDeviceSynchronize();
    delete m;
    return TSK_OK;
}

extern "C" int tsk_model_info(const tsk_model *m, tsk_mlp_shape *shape, int64_t *n_params)
{
    g_err.clear();
    if (!m)
        return set_err(TSK_ERR_INVALID_ARG, "model is NULL");
    if (shape) {
        shape->size = sizeof(tsk_mlp_shape);
        shape->dim = m->dim;
        shape->points = m->points;
        shape->hidden = m->hidden;
        shape->embed = m->embed;
    }
    if (n_params)
        *n_params = m->n_params;
    return TSK_OK;
}

extern "C" int tsk_model_get_params(const tsk_model *cm, float *out_host, int64_t n)
{
    g_err.clear();
    TSK_TRY(check_model(cm));
    if (!out_host || n != cm->n_params)
        return set_err(TSK_ERR_INVALID_ARG, "need a host buffer of %lld floats",
                       (long long)cm->n_params);
    tsk_model *m = const_cast<tsk_model *>(cm);
    std::lock_guard<std::mutex> lock(m->mu);
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(out_host, m->params.p, n * sizeof(float), hipMemcpyDeviceToHost));
    return TSK_OK;
}

extern "C" int tsk_model_set_params(tsk_model *m, const float *in_host, int64_t n)
{
    g_err.clear();
    TSK_TRY(check_model(m));
    if (!in_host || n != m->n_params)
        return set_err(TSK_ERR_INVALID_ARG, "need %lld floats", (long long)m->n_params);
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(in_host[i]))
            return set_err(TSK_ERR_INVALID_ARG, "parameter %lld is not finite", (long long)i);
    std::lock_guard<std::mutex> lock(m->mu);
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(m->params.p, in_host, n * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(m->m.p, 0, n * sizeof(float)));
    HIP_TRY(hipMemset(m->v.p, 0, n * sizeof(float)));
    m->step = 0;
    ++m->version;
    return TSK_OK;
}

extern "C" int tsk_model_embed(tsk_model *m, const float *values_dev, const int64_t *offsets_host,
                               int64_t n_series, float *out_dev, void *hip_stream)
{
    g_err.clear();
    TSK_TRY(check_model(m));
    if (!values_dev || !out_dev)
        return set_err(TSK_ERR_INVALID_ARG, "NULL device pointer");
    TSK_TRY(check_offsets(offsets_host, n_series));
    TSK_TRY(check_dev_ptr(values_dev, m->device, "values_dev"));
    TSK_TRY(check_dev_ptr(out_dev, m->device, "out_dev"));
    std::lock_guard<std::mutex> lock(m->mu);
    hipStream_t s = (hipStream_t)hip_stream;
    TSK_TRY(upload_offsets(m, offsets_host, n_series, s));
    TSK_TRY(model_embed_dev(m, values_dev, m->off_dev.p, n_series, out_dev, s));
    // the offsets buffer is reused by the next call: finish with it
    HIP_TRY(hipStreamSynchronize(s));
    return TSK_OK;
}

extern "C" int tsk_model_batch_grad(tsk_model *m, const float *values_dev,
                                    const int64_t *offsets_host, int64_t n_series,
                                    const int32_t *a_host, const int32_t *b_host,
                                    const float *target_host, int64_t n_pairs,
                                    float *out_loss_host, float *out_grad_host, void *hip_stream)
{
    g_err.clear();
    TSK_TRY(check_model(m));
    if (!values_dev)
        return set_err(TSK_ERR_INVALID_ARG, "values_dev is NULL");
    TSK_TRY(check_offsets(offsets_host, n_series));
    TSK_TRY(check_pairs(a_host, b_host, target_host, n_pairs, n_series));
    TSK_TRY(check_dev_ptr(values_dev, m->device, "values_dev"));
    if (n_pairs > 65536)
        return set_err(TSK_ERR_UNSUPPORTED, "at most 65536 pairs per batch");
    std::lock_guard<std::mutex> lock(m->mu);
    hipStream_t s = (hipStream_t)hip_stream;
    TSK_TRY(prepare_pool(m, values_dev, offsets_host, n_series, s));
    TSK_TRY(ensure_batch(m, 2 * n_pairs));
    TSK_TRY(m->ia.ensure(n_pairs));
    TSK_TRY(m->ib.ensure(n_pairs));
    TSK_TRY(m->y.ensure(n_pairs));
    HIP_TRY(hipMemcpyAsync(m->ia.p, a_host, n_pairs * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(m->ib.p, b_host, n_pairs * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(m->y.p, target_host, n_pairs * sizeof(float), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, s, m->loss.p, (int64_t)1);
    gather_pairs(m, m->ia.p, m->ib.p, n_pairs, s);
    grad_step(m, n_pairs, m->y.p, m->loss.p, s);
    HIP_TRY(hipGetLastError());
    float loss = 0.0f;
    HIP_TRY(hipMemcpyAsync(&loss, m->loss.p, sizeof(float), hipMemcpyDeviceToHost, s));
    if (out_grad_host)
        HIP_TRY(hipMemcpyAsync(out_grad_host, m->grads.p, m->n_params * sizeof(float),
                               hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (out_loss_host)
        *out_loss_host = loss;
    return TSK_OK;
}

extern "C" int tsk_model_train(tsk_model *m, const float *values_dev, const int64_t *offsets_host,
                               int64_t n_series, const int32_t *a_host, const int32_t *b_host,
                               const float *target_host, int64_t n_pairs,
                               const tsk_train_opts *opts, float *out_epoch_loss_host,
                               void *hip_stream)
{
    g_err.clear();
    TSK_TRY(check_model(m));
    if (!values_dev)
        return set_err(TSK_ERR_INVALID_ARG, "values_dev is NULL");
    if (!opts || opts->size != (int64_t)sizeof(tsk_train_opts))
        return set_err(TSK_ERR_INVALID_ARG, "opts missing or opts->size mismatch");
    if (opts->epochs < 1 || opts->batch < 1 || opts->batch > 65536 || !(opts->lr > 0.0f))
        return set_err(TSK_ERR_INVALID_ARG, "epochs >= 1, batch in [1, 65536], lr > 0");
    TSK_TRY(check_offsets(offsets_host, n_series));
    TSK_TRY(check_pairs(a_host, b_host, target_host, n_pairs, n_series));
    TSK_TRY(check_dev_ptr(values_dev, m->device, "values_dev"));
    const float b1 = opts->beta1 > 0.0f ? opts->beta1 : 0.9f;
    const float b2 = opts->beta2 > 0.0f ? opts->beta2 : 0.999f;
    const float eps = opts->eps > 0.0f ? opts->eps : 1e-8f;
    std::lock_guard<std::mutex> lock(m->mu);
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t B = std::min<int64_t>(opts->batch, n_pairs);
    const int64_t steps = (n_pairs + B - 1) / B;
    TSK_TRY(prepare_pool(m, values_dev, offsets_host, n_series, s));
    TSK_TRY(ensure_batch(m, 2 * B));
    TSK_TRY(m->ia.ensure(n_pairs));
    TSK_TRY(m->ib.ensure(n_pairs));
    TSK_TRY(m->y.ensure(n_pairs));
    TSK_TRY(m->loss.ensure((size_t)steps * opts->epochs));
    hipLaunchKernelGGL(k_zero_f32, dim3(grid1(steps * opts->epochs, 256)), dim3(256), 0, s,
                       m->loss.p, steps * (int64_t)opts->epochs);
    std::vector<int32_t> perm(n_pairs), ha(n_pairs), hb(n_pairs);
    std::vector<float> hy(n_pairs);
    uint64_t st = opts->seed;
    for (int ep = 0; ep < opts->epochs; ++ep) {
        for (int64_t i = 0; i < n_pairs; ++i)
            perm[i] = (int32_t)i;
        for (int64_t i = n_pairs - 1; i > 0; --i) { // Fisher-Yates
            const int64_t j = (int64_t)(splitmix64(st) % (uint64_t)(i + 1));
            std::swap(perm[i], perm[j]);
        }
        for (int64_t i = 0; i < n_pairs; ++i) {
            ha[i] = a_host[perm[i]];
            hb[i] = b_host[perm[i]];
            hy[i] = target_host[perm[i]];
        }
        // the previous epoch's steps still read these buffers
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(hipMemcpyAsync(m->ia.p, ha.data(), n_pairs * sizeof(int32_t),
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(m->ib.p, hb.data(), n_pairs * sizeof(int32_t),
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(m->y.p, hy.data(), n_pairs * sizeof(float), hipMemcpyHostToDevice,
                               s));
        for (int64_t k = 0; k < steps; ++k) {
            const int64_t p0 = k * B;
            const int64_t b = std::min<int64_t>(B, n_pairs - p0);
            gather_pairs(m, m->ia.p + p0, m->ib.p + p0, b, s);
            grad_step(m, b, m->y.p + p0, m->loss.p + (int64_t)ep * steps + k, s);
            ++m->step;
            const double c1 = 1.0 / (1.0 - std::pow((double)b1, (double)m->step));
            const double c2 = 1.0 / (1.0 - std::pow((double)b2, (double)m->step));
            hipLaunchKernelGGL(k_adam, dim3(grid1(m->n_params, 256)), dim3(256), 0, s, m->params.p,
                               m->grads.p, m->m.p, m->v.p, m->n_params, opts->lr, b1, b2, eps,
                               (float)c1, (float)c2);
        }
        HIP_TRY(hipGetLastError());
    }
    ++m->version;
    std::vector<float> losses((size_t)steps * opts->epochs);
    HIP_TRY(hipMemcpyAsync(losses.data(), m->loss.p, losses.size() * sizeof(float),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (out_epoch_loss_host)
        for (int ep = 0; ep < opts->epochs; ++ep) {
            double sum = 0.0;
            for (int64_t k = 0; k < steps; ++k)
                sum += losses[(size_t)ep * steps + k];
            out_epoch_loss_host[ep] = (float)(sum / (double)steps);
        }
    return TSK_OK;
}

static const char MODEL_MAGIC[8] = {'T', 'S', 'K', 'M', 'L', 'P', '0', '1'};

extern "C" int tsk_model_save(const tsk_model *m, const char *path)
{
    g_err.clear();
    if (!m || !path)
        return set_err(TSK_ERR_INVALID_ARG, "model and path must be non-NULL");
    std::vector<float> h(m->n_params);
    TSK_TRY(tsk_model_get_params(m, h.data(), m->n_params));
    FILE *f = fopen(path, "wb");
    if (!f)
        return set_err(TSK_ERR_IO, "cannot open %s for writing", path);
    const int32_t hdr[4] = {m->dim, m->points, m->hidden, m->embed};
    const int64_t n = m->n_params;
    bool ok = fwrite(MODEL_MAGIC, 1, 8, f) == 8 && fwrite(hdr, sizeof(hdr), 1, f) == 1 &&
              fwrite(&n, sizeof(n), 1, f) == 1 &&
              fwrite(h.data(), sizeof(float), (size_t)n, f) == (size_t)n;
    ok = (fclose(f) == 0) && ok;
    if (!ok)
        return set_err(TSK_ERR_IO, "short write to %s", path);
    return TSK_OK;
}

extern "C" int tsk_model_load(const char *path, tsk_model **out)
{
    g_err.clear();
    if (!path || !out)
        return set_err(TSK_ERR_INVALID_ARG, "path and out must be non-NULL");
    *out = nullptr;
    FILE *f = fopen(path, "rb");
    if (!f)
        return set_err(TSK_ERR_IO, "cannot open %s", path);
    char magic[8];
    int32_t hdr[4];
    int64_t n = 0;
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, MODEL_MAGIC, 8) == 0 &&
              fread(hdr, sizeof(hdr), 1, f) == 1 && fread(&n, sizeof(n), 1, f) == 1;
    if (!ok) {
        fclose(f);
        return set_err(TSK_ERR_IO, "%s is not an encoder file", path);
    }
    tsk_mlp_shape sh;
    sh.size = sizeof(sh);
    sh.dim = hdr[0];
    sh.points = hdr[1];
    sh.hidden = hdr[2];
    sh.embed = hdr[3];
    tsk_mlp_shape chk;
    int rc = resolve_shape(&sh, &chk);
    if (rc != TSK_OK) {
        fclose(f);
        return set_err(TSK_ERR_IO, "%s: bad shape (%s)", path, g_err.c_str());
    }
    tsk_model *m = nullptr;
    rc = create_model(chk, &m);
    if (rc != TSK_OK) {
        fclose(f);
        return rc;
    }
    std::vector<float> h(m->n_params);
    ok = n == m->n_params && fread(h.data(), sizeof(float), (size_t)n, f) == (size_t)n;
    fclose(f);
    if (!ok) {
        delete m;
        return set_err(TSK_ERR_IO, "%s: parameter count or data mismatch", path);
    }
    rc = tsk_model_set_params(m, h.data(), n);
    if (rc != TSK_OK) {
        delete m;
        return rc;
    }
    *out = m;
    return TSK_OK;
}
