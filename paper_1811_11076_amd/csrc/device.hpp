// Device helpers shared by the tsknn kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define TSK_INF_BITS 0x7F800000u
#define TSK_KEY_EMPTY 0xFFFFFFFFFFFFFFFFull

__device__ __forceinline__ float tsk_inf() { return __builtin_huge_valf(); }

__device__ __forceinline__ float bits_f(uint32_t u) { return __uint_as_float(u); }
__device__ __forceinline__ uint32_t f_bits(float f) { return __float_as_uint(f); }

// Squared Euclidean point cost (Sec. 3, d(s,t) = ||s - t||_2, squared as DTW
// uses it in Sec. 2.1).  Fixed fp32 order: e_k = fl(s_k - t_k);
// acc = e_0 * e_0; acc = fma(e_k, e_k, acc) for k = 1..D-1.  The library is
// compiled with -ffp-contract=off so no other fusion happens.
template <int D>
__device__ __forceinline__ float point_cost(const float (&s)[D], const float (&t)[D])
{
    float e = s[0] - t[0];
    float acc = e * e;
#pragma unroll
    for (int k = 1; k < D; ++k) {
        e = s[k] - t[k];
        acc = __builtin_fmaf(e, e, acc);
    }
    return acc;
}

template <int D>
__device__ __forceinline__ void load_point(const float *__restrict__ p, float (&v)[D])
{
#pragma unroll
    for (int k = 0; k < D; ++k)
        v[k] = p[k];
}

// Correctly rounded fp32 square root.  The hardware/library square root is
// taken as a first guess r, then corrected with Tuckerman's rounding test: the
// midpoints between r and its fp32 neighbours have at most 25 significant
// bits, so their squares are exact in fp64 and comparing x with them decides
// whether r, or a neighbour, is the nearest fp32 value to sqrt(x).  (x cannot
// equal a midpoint's square: that square needs more than 24 bits.)
__device__ __forceinline__ float sqrt_rn_f32(float x)
{
    if (!(x > 0.0f) || x == __builtin_huge_valf())
        return x == 0.0f ? x : (x > 0.0f ? x : __builtin_nanf(""));
    float r = __builtin_sqrtf(x);
    const double xd = (double)x;
#pragma unroll
    for (int it = 0; it < 3; ++it) {
        // r > 0 and finite: the fp32 neighbours are one bit pattern apart
        const float lo = __uint_as_float(__float_as_uint(r) - 1u);
        const float hi = __uint_as_float(__float_as_uint(r) + 1u);
        const double mlo = 0.5 * ((double)r + (double)lo);
        const double mhi = 0.5 * ((double)r + (double)hi);
        if (xd < mlo * mlo)
            r = lo;
        else if (xd > mhi * mhi)
            r = hi;
        else
            break;
    }
    return r;
}

// Wave-uniform copy of lane 0's value (readfirstlane keeps the result in
// SGPRs, so loops and addresses that depend on it stay uniform).
__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ float min3f(float a, float b, float c)
{
    return fminf(fminf(a, b), c);
}

__device__ __forceinline__ int64_t floor_div64(int64_t a, int64_t b)
{
    // b > 0
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0))
        --q;
    return q;
}

__device__ __forceinline__ int64_t ceil_div64(int64_t a, int64_t b) { return -floor_div64(-a, b); }

// Sakoe-Chiba band for a pair of lengths (m rows = query, n columns =
// candidate).  Cell (i, j) is inside iff |i B - j A| K <= R with A = m-1,
// B = n-1, K = max(m,n)-1, R = w A B; every cell when w < 0 or m == 1 or
// n == 1.  For m == n this is |i - j| <= w (Sec. 2.2).
struct Band {
    int64_t A, B, K, R;
    int all;
};

// Half-width for a pair: mode 0 none (-1), 1 absolute r, 2 floor(frac * L).
__device__ __forceinline__ int band_w(int mode, int r, float frac, int m, int n)
{
    if (mode == 1)
        return r;
    if (mode == 2) {
        int L = m > n ? m : n;
        return (int)floor((double)frac * (double)L);
    }
    return -1;
}

__device__ __forceinline__ Band make_band(int m, int n, int w)
{
    Band b;
    b.all = (w < 0 || m == 1 || n == 1);
    b.A = m - 1;
    b.B = n - 1;
    b.K = (m > n ? m : n) - 1;
    b.R = (int64_t)(w < 0 ? 0 : w) * b.A * b.B;
    return b;
}

__device__ __forceinline__ bool band_ok(const Band &b, int i, int j)
{
    if (b.all)
        return true;
    int64_t a = (int64_t)i * b.B - (int64_t)j * b.A;
    a = a < 0 ? -a : a;
    return a * b.K <= b.R;
}

// Columns of row i inside the band, clipped to [0, n-1]; empty -> lo > hi.
__device__ __forceinline__ void band_cols(const Band &b, int i, int n, int &lo, int &hi)
{
    if (b.all) {
        lo = 0;
        hi = n - 1;
        return;
    }
    int64_t den = b.A * b.K;
    int64_t c = (int64_t)i * b.B * b.K;
    int64_t l = ceil_div64(c - b.R, den), h = floor_div64(c + b.R, den);
    lo = (int)(l < 0 ? 0 : l);
    hi = (int)(h > n - 1 ? n - 1 : h);
}

// Rows of column j inside the band, clipped to [0, m-1]; empty -> lo > hi.
__device__ __forceinline__ void band_rows(const Band &b, int j, int m, int &lo, int &hi)
{
    if (b.all) {
        lo = 0;
        hi = m - 1;
        return;
    }
    int64_t den = b.B * b.K;
    int64_t c = (int64_t)j * b.A * b.K;
    int64_t l = ceil_div64(c - b.R, den), h = floor_div64(c + b.R, den);
    lo = (int)(l < 0 ? 0 : l);
    hi = (int)(h > m - 1 ? m - 1 : h);
}

// k smallest 64-bit keys of one query, kept sorted in k slots initialised to
// TSK_KEY_EMPTY.  Lock-free: a key walks down the slots; at each slot an
// atomic min keeps the smaller value there and the larger one walks on.
// Every key that ever reached slot s lost to a distinct smaller key held by
// each slot before s, so at every moment slot k-1 holds a key that has at
// least k-1 distinct smaller keys inserted: an upper bound on the k-th
// smallest key over everything inserted so far.  Keys are
// (float bits of a non-negative value << 32) | candidate id, so the order is
// (value, id) and distinct candidates never collide.
__device__ __forceinline__ void topk_insert(unsigned long long *slots, int k, unsigned long long key)
{
    for (int s = 0; s < k; ++s) {
        unsigned long long old = atomicMin(slots + s, key);
        if (old > key)
            key = old;
        if (key == TSK_KEY_EMPTY)
            break;
    }
}

__device__ __forceinline__ uint32_t load_relaxed_u32(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long load_relaxed_u64(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Lowers the running threshold of a query to the key value held by slot k-1
// (a valid upper bound on the k-th smallest distance, see topk_insert).
__device__ __forceinline__ void tau_from_slots(const unsigned long long *slots, int k, uint32_t *tau)
{
    unsigned long long last = load_relaxed_u64(slots + (k - 1));
    if (last != TSK_KEY_EMPTY)
        atomicMin(tau, (uint32_t)(last >> 32));
}

__device__ __forceinline__ unsigned long long make_key(float v, uint32_t id)
{
    return ((unsigned long long)f_bits(v) << 32) | (unsigned long long)id;
}
