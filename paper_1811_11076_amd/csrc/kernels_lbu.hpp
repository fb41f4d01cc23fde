// LB_Box for databases whose series differ in length (eq. (1) with the
// query's envelope, Sec. 2.3-3).  The band window of candidate point j,
// rows [lo_j, hi_j] of the query, depends on the pair of lengths (m, n), so
// no single envelope per query serves every candidate.  Instead:
//
//  * the index keeps its series sorted by (length, id) and cut into tiles of
//    at most 64 series of ONE length, each packed SoA [pos][dim][64];
//  * every query gets a sparse table: level l, entry i holds the per-dimension
//    [min, max] of query points i .. i + 2^l - 1 (clipped at the end);
//  * one wave takes one tile against a group of queries: the window of point
//    j is the same for all its lanes; the two table entries of level
//    floor(log2(hi_j - lo_j + 1)) that cover [lo_j, hi_j] exactly give its
//    [min, max].
//
// The envelope is exact, so the bound equals the plain definition term by
// term; terms are summed over j in order in fp32, as in the equal-length
// kernel.
#pragma once
#include "kernels.hpp"
#include "kernels_fast.hpp"

namespace tsk {

struct BucketArgs {
    const int32_t *perm;  // position (length-sorted) -> series id
    const int32_t *tpos;  // tile -> first position
    const int32_t *tcnt;  // tile -> number of series (1..64)
    const int32_t *tlen;  // tile -> the common length of its series
    const int64_t *toff;  // tile -> offset of its SoA block (floats)
    const float *soa;     // [tile][pos][dim][64]
    int64_t n_tiles;
};

// floor(log2(m)) + 1 levels of m entries of 2*DP floats
__host__ __device__ inline int64_t qtable_floats(int m, int DP)
{
    int lv = 0;
    while ((2 << lv) <= m)
        ++lv;
    return (int64_t)(lv + 1) * m * 2 * DP;
}

// One block per query.  Level 0 is the query itself; level l combines the
// two halves of level l-1 (entries whose span would pass the end repeat the
// last point, which leaves their [min, max] unchanged).
template <int D>
__global__ __launch_bounds__(256) void k_qtable(const float *__restrict__ qv,
                                                const int64_t *__restrict__ qoff,
                                                const int64_t *__restrict__ tab_off,
                                                float *__restrict__ tab)
{
    constexpr int DP = PadDim<D>::value;
    const int q = blockIdx.x;
    const int64_t o0 = qoff[q];
    const int m = (int)(qoff[q + 1] - o0);
    float *T = tab + tab_off[q];
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        float *e = T + (int64_t)i * 2 * DP;
#pragma unroll
        for (int k = 0; k < DP; ++k) {
            const float v = k < D ? qv[(o0 + i) * D + k] : 0.0f;
            e[k] = v;
            e[DP + k] = v;
        }
    }
    for (int l = 1; (2 << (l - 1)) <= m; ++l) {
        __syncthreads(); // level l-1 complete and visible to the block
        const float *P = T + (int64_t)(l - 1) * m * 2 * DP;
        float *C = T + (int64_t)l * m * 2 * DP;
        const int h = 1 << (l - 1);
        for (int i = threadIdx.x; i < m; i += blockDim.x) {
            const int i2 = min(i + h, m - 1);
            const float *a = P + (int64_t)i * 2 * DP, *b = P + (int64_t)i2 * 2 * DP;
            float *c = C + (int64_t)i * 2 * DP;
#pragma unroll
            for (int k = 0; k < DP; ++k) {
                c[k] = fminf(a[k], b[k]);
                c[DP + k] = fmaxf(a[DP + k], b[DP + k]);
            }
        }
    }
}

// One wave (block of 64) per (tile, group of QG queries).  Per chunk of 64
// candidate points, lane l builds the envelope of point j0 + l for every
// query of the group (two table entries each, combined) into LDS; the
// chunk's terms then read it back with wave-uniform addresses.  lbv is
// written in length-sorted position order: lbv[q][position], +inf where the
// bound exceeds the running threshold.  DEBUG writes the raw bound to
// dbg_lb[q][id] instead.
template <int D, int QG, bool DEBUG>
__global__ __launch_bounds__(64) void k_bound_lbu(BoundArgs a, BucketArgs bk,
                                                  const float *__restrict__ tab,
                                                  const int64_t *__restrict__ tab_off)
{
    constexpr int DP = PadDim<D>::value;
    __shared__ float env_s[QG][64][2 * D]; // [query][point of chunk][lo D, hi D]
    const int lane = threadIdx.x;
    const int64_t t = blockIdx.x;
    const int q0 = blockIdx.y * QG;
    const int nqg = min(QG, a.nq - q0);
    const int cnt = bk.tcnt[t];
    const int n = bk.tlen[t];
    const int64_t pos = (int64_t)bk.tpos[t] + lane;
    const bool valid = lane < cnt;
    // lanes past cnt read the tile's zero padding (the block has 64 lanes)
    const float *tb = bk.soa + bk.toff[t] + lane;
    int mq[QG];
    Band bq[QG];
    const float *T[QG];
#pragma unroll
    for (int g = 0; g < QG; ++g) {
        // groups past the last query repeat query q0; their sums are dropped
        const int q = q0 + (g < nqg ? g : 0);
        mq[g] = (int)(a.qoff[q + 1] - a.qoff[q]);
        bq[g] = pair_band(a.ba, mq[g], n);
        T[g] = tab + tab_off[q];
    }
    float acc[QG];
#pragma unroll
    for (int g = 0; g < QG; ++g)
        acc[g] = 0.0f;
    for (int j0 = 0; j0 < n; j0 += 64) {
        const int jl = min(j0 + lane, n - 1);
        __syncthreads(); // the previous chunk's reads are done
#pragma unroll
        for (int g = 0; g < QG; ++g) {
            int lo, hi;
            band_rows(bq[g], jl, mq[g], lo, hi);
            float *e = env_s[g][lane];
            if (lo > hi) {
                // no query row may align with this point: the term is +inf
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    e[k] = tsk_inf();
                    e[D + k] = -tsk_inf();
                }
            } else {
                // [lo, hi] = union of two power-of-two spans of one level
                const int lv = 31 - __clz(hi - lo + 1);
                const float *e1 = T[g] + ((int64_t)lv * mq[g] + lo) * 2 * DP;
                const float *e2 = T[g] + ((int64_t)lv * mq[g] + hi - (1 << lv) + 1) * 2 * DP;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    e[k] = fminf(e1[k], e2[k]);
                    e[D + k] = fmaxf(e1[DP + k], e2[DP + k]);
                }
            }
        }
        __syncthreads();
        const int jn = min(64, n - j0);
        for (int jj = 0; jj < jn; ++jj) {
            float x[D];
#pragma unroll
            for (int k = 0; k < D; ++k)
                x[k] = tb[((int64_t)(j0 + jj) * D + k) * 64];
#pragma unroll
            for (int g = 0; g < QG; ++g) {
                const float *e = env_s[g][jj];
                float term = 0.0f;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const float d = fmaxf(fmaxf(e[k] - x[k], x[k] - e[D + k]), 0.0f);
                    term = (k == 0) ? d * d : __builtin_fmaf(d, d, term);
                }
                acc[g] = term + acc[g];
            }
        }
    }
    if (DEBUG) {
        if (valid) {
            const int id = bk.perm[pos];
#pragma unroll
            for (int g = 0; g < QG; ++g)
                if (g < nqg)
                    a.dbg_lb[(int64_t)(q0 + g) * a.N + id] = acc[g];
        }
        return;
    }
    unsigned long long pruned = 0, pairs = 0;
    if (valid) {
        // the group's thresholds first: independent loads, one latency
        float tq[QG];
#pragma unroll
        for (int g = 0; g < QG; ++g)
            tq[g] = g < nqg ? bits_f(load_relaxed_u32(a.tau + q0 + g)) : 0.0f;
#pragma unroll
        for (int g = 0; g < QG; ++g) {
            if (g < nqg) {
                const int q = q0 + g;
                const bool keep = acc[g] <= tq[g];
                a.lbv[(int64_t)q * a.N + pos] = keep ? acc[g] : tsk_inf();
                pruned += keep ? 0 : 1;
                ++pairs;
            }
        }
    }
    wave_count(a.ctr, C_BOUND_PRUNED, pruned);
    wave_count(a.ctr, C_PAIRS, pairs);
    wave_count(a.ctr, C_BOUND_STEPS, valid ? (unsigned long long)n * nqg : 0ull);
}

// SoA packing of the length buckets: block t fills tile t.
template <int D>
__global__ void k_pack_bucket(const float *__restrict__ aos, const int64_t *__restrict__ off,
                              BucketArgs bk, float *__restrict__ soa)
{
    const int64_t t = blockIdx.x;
    const int n = bk.tlen[t], cnt = bk.tcnt[t];
    const int64_t p0 = bk.tpos[t];
    const int64_t total = (int64_t)n * D * 64;
    float *dst = soa + bk.toff[t];
    for (int64_t idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int lane = (int)(idx & 63);
        const int dim = (int)((idx >> 6) % D);
        const int64_t p = (idx >> 6) / D;
        float v = 0.0f;
        if (lane < cnt)
            v = aos[(off[bk.perm[p0 + lane]] + p) * D + dim];
        dst[idx] = v;
    }
}

} // namespace tsk
