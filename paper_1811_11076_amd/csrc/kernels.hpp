// tsknn device kernels for gfx950 (wave64).
#pragma once

#include "device.hpp"

namespace tsk {

enum { DIST_DTW = 0, DIST_DK = 1 };

// Counter slots (device u64), mirrored by tsk_stats.
enum {
    C_PAIRS = 0,
    C_SEED_PAIRS,
    C_BOUND_PRUNED,
    C_DP_STARTED,
    C_DP_COMPLETED,
    C_DP_ABANDONED,
    C_DP_CELLS,
    C_BOUND_STEPS,
    C_FALLBACK,
    C_LATE_PRUNED,
    C_VALID_CELLS,
    C_VALID_GEN, // valid cells of the general DP (also counted in C_VALID_CELLS)
    C_SEED_STEPS, // greedy moves of the threshold-seeding walks
    C_NUM
};
constexpr int CTR_STRIPES = 64;
constexpr int CTR_WORDS = C_NUM * CTR_STRIPES; // device words of the counters

// Host: the counters from their striped device words.
inline void ctr_sum(const unsigned long long *words, unsigned long long *out)
{
    for (int i = 0; i < C_NUM; ++i) {
        unsigned long long t = 0;
        for (int j = 0; j < CTR_STRIPES; ++j)
            t += words[i * CTR_STRIPES + j];
        out[i] = t;
    }
}

// Dimensions the kernels are built for: 1..8, and 12, 16, 24, 32, to which
// larger dimensionalities are padded with zero coordinates (a zero
// coordinate on both sides adds fl(0*0 + acc) = acc to a point cost and 0 to
// a box term, so every cost and bound keeps its bits).
__host__ __device__ constexpr int kernel_dim(int d)
{
    return d <= 8 ? d : (d <= 12 ? 12 : (d <= 16 ? 16 : (d <= 24 ? 24 : 32)));
}
// Floats per staged point: 4 up to 4 dimensions, 8 up to 8, else the
// dimension itself (a multiple of 4 above 8).
__host__ __device__ constexpr int pad_dim(int D) { return D <= 4 ? 4 : (D <= 8 ? 8 : D); }

// Point rows [rows][d] -> [rows][kd] with zero coordinates d..kd-1.
static __global__ void k_pad_dims(const float *__restrict__ src, int64_t rows, int d, int kd,
                                  float *__restrict__ dst)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = rows * kd;
    for (int64_t i = t; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / kd;
        const int k = (int)(i % kd);
        dst[i] = k < d ? src[r * d + k] : 0.0f;
    }
}

struct BandArgs {
    int mode, r;
    float frac;
};

__device__ __forceinline__ Band pair_band(const BandArgs &ba, int m, int n)
{
    return make_band(m, n, band_w(ba.mode, ba.r, ba.frac, m, n));
}

// Wave-wide sum of a per-lane counter, added once per wave.
// Statistics counters (ctr[C_...]): a null base turns counting off (calls
// that ask for neither stats nor a profile), sparing every wave its atomics
// on the few shared counter words.
// Each counter is CTR_STRIPES words (ctr[idx * CTR_STRIPES + stripe]) that
// the host sums: a kernel of millions of waves would otherwise serialise on
// one word's atomics.  A wave adds to the stripe of its block.
__device__ __forceinline__ unsigned long long *ctr_word(unsigned long long *ctr, int idx)
{
    const unsigned b = blockIdx.x + 7u * blockIdx.y + 13u * blockIdx.z + (threadIdx.x >> 6);
    return ctr + idx * CTR_STRIPES + (b & (CTR_STRIPES - 1));
}

__device__ __forceinline__ void wave_count(unsigned long long *ctr, int idx, unsigned long long v)
{
    if (ctr == nullptr)
        return;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0 && v)
        atomicAdd(ctr_word(ctr, idx), v);
}

__device__ __forceinline__ void ctr_add(unsigned long long *ctr, int idx, unsigned long long v)
{
    if (ctr != nullptr)
        atomicAdd(ctr_word(ctr, idx), v);
}

// Sum over the wave's 64 lanes (xor butterfly: both lanes of every pair add
// the same two values, so every lane ends with the same bits).
__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ float wave_min(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}

// ------------------------------------------------------------------ fills
// Plain fill kernels (no hipMemsetAsync, so the sequence stays capturable).
static __global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// rows of 0 .. N-1: a survivor list holding every candidate of each query
static __global__ void k_iota_rows(int32_t *p, int64_t rows, int64_t N)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < rows * N; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)(i % N);
}

static __global__ void k_fill_u64(unsigned long long *p, unsigned long long v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static __global__ void k_add_u64(unsigned long long *dst, const unsigned long long *src, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        dst[i] += src[i];
}

// ------------------------------------------------------------------ index pack
// AoS [sum len][D] -> 64-series struct-of-arrays tiles: tile t holds series
// 64t..64t+63 as [pos][dim][lane] with pos < the tile's longest length, so a
// wave whose lane l handles series 64t+l reads 256 contiguous bytes per
// (pos, dim).  Slots past a series' end hold 0 and are never read.
template <int D>
__global__ void k_pack_soa(const float *__restrict__ aos, const int64_t *__restrict__ off,
                           const int32_t *__restrict__ len, int64_t N,
                           const int64_t *__restrict__ tile_off, const int32_t *__restrict__ tile_len,
                           float *__restrict__ soa)
{
    const int64_t t = blockIdx.x;
    const int64_t cnt = (int64_t)tile_len[t] * D * 64;
    float *dst = soa + tile_off[t];
    for (int64_t idx = threadIdx.x; idx < cnt; idx += blockDim.x) {
        const int lane = (int)(idx & 63);
        const int dim = (int)((idx >> 6) % D);
        const int64_t pos = (idx >> 6) / D;
        const int64_t s = t * 64 + lane;
        float v = 0.0f;
        if (s < N && pos < len[s])
            v = aos[(off[s] + pos) * D + dim];
        dst[idx] = v;
    }
}

// ------------------------------------------------------------------ query envelope
// Envelope of the query for candidates of length n (Sec. 2.3 / Sec. 3 boxes,
// with the query in the role of the enveloped series): for every candidate
// point j, the per-dimension [min, max] of the query points i that the band
// lets align with j.  Brute-force window; an empty window gives
// [+inf, -inf].  env: [q][j][2][D].
template <int D>
__global__ void k_env(const float *__restrict__ qv, const int64_t *__restrict__ qoff, int nq, int n,
                      BandArgs ba, float *__restrict__ env)
{
    const int q = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq || j >= n)
        return;
    const int m = (int)(qoff[q + 1] - qoff[q]);
    const float *Q = qv + qoff[q] * D;
    const Band b = pair_band(ba, m, n);
    int lo, hi;
    band_rows(b, j, m, lo, hi);
    float mn[D], mx[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        mn[k] = tsk_inf();
        mx[k] = -tsk_inf();
    }
    for (int i = lo; i <= hi; ++i) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const float v = Q[i * D + k];
            mn[k] = fminf(mn[k], v);
            mx[k] = fmaxf(mx[k], v);
        }
    }
    float *e = env + ((int64_t)q * n + j) * 2 * D;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        e[k] = mn[k];
        e[D + k] = mx[k];
    }
}

// Squared distance of x to the box [lo, hi] (Sec. 3: sum over dimensions of
// the squared interval distances), same fp32 order as the point cost; an
// empty box gives +inf.
template <int D>
__device__ __forceinline__ float box_term(const float (&x)[D], const float *lo, const float *hi)
{
    float acc = 0.0f;
    bool empty = false;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        empty |= lo[k] > hi[k];
        float e = 0.0f;
        if (x[k] < lo[k])
            e = lo[k] - x[k];
        else if (x[k] > hi[k])
            e = x[k] - hi[k];
        acc = (k == 0) ? e * e : __builtin_fmaf(e, e, acc);
    }
    return empty ? tsk_inf() : acc;
}

// ------------------------------------------------------------------ greedy walk
// Alg. 1 (Sec. 4.1): from (0,0) step to the cheapest of (i+1,j), (i+1,j+1),
// (i,j+1) (ties to the first listed; off-matrix or out-of-band moves +inf)
// until (m-1, n-1).  DIST_DK keeps the running maximum (the greedy DK upper
// bound, squared domain); DIST_DTW sums along the path in path order (an
// upper bound of the fp32 DTW, used to seed its threshold).  Returns as soon
// as the value exceeds eps; eps is lowered from *tau (nullable) every 8
// moves.  *completed says whether the walk reached the corner.
template <int D, int DIST>
__device__ float greedy_walk(const float *__restrict__ q, int m, const float *__restrict__ c, int n,
                             const Band &band, float eps, const uint32_t *tau, int &steps_out,
                             bool &completed)
{
    float qi[D], qi1[D], cj[D], cj1[D];
    load_point<D>(q, qi);
    load_point<D>(c, cj);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        qi1[k] = 0.0f;
        cj1[k] = 0.0f;
    }
    float g = point_cost<D>(qi, cj);
    int i = 0, j = 0, steps = 0;
    completed = false;
    if (g > eps) {
        steps_out = 0;
        return g;
    }
    if (m > 1)
        load_point<D>(q + D, qi1);
    if (n > 1)
        load_point<D>(c + D, cj1);
    while (i < m - 1 || j < n - 1) {
        const bool di = i + 1 < m, dj = j + 1 < n;
        float c_dn = tsk_inf(), c_dg = tsk_inf(), c_rt = tsk_inf();
        if (di && band_ok(band, i + 1, j))
            c_dn = point_cost<D>(qi1, cj);
        if (di && dj && band_ok(band, i + 1, j + 1))
            c_dg = point_cost<D>(qi1, cj1);
        if (dj && band_ok(band, i, j + 1))
            c_rt = point_cost<D>(qi, cj1);
        int mv;
        float cst;
        if (c_dn <= c_dg && c_dn <= c_rt) {
            mv = 0;
            cst = c_dn;
        } else if (c_dg <= c_rt) {
            mv = 1;
            cst = c_dg;
        } else {
            mv = 2;
            cst = c_rt;
        }
        ++steps;
        if (cst == tsk_inf()) {
            g = tsk_inf();
            steps_out = steps;
            return g;
        }
        g = DIST == DIST_DK ? fmaxf(g, cst) : cst + g;
        if (mv != 2) {
            ++i;
#pragma unroll
            for (int k = 0; k < D; ++k)
                qi[k] = qi1[k];
            if (i + 1 < m)
                load_point<D>(q + (int64_t)(i + 1) * D, qi1);
        }
        if (mv != 0) {
            ++j;
#pragma unroll
            for (int k = 0; k < D; ++k)
                cj[k] = cj1[k];
            if (j + 1 < n)
                load_point<D>(c + (int64_t)(j + 1) * D, cj1);
        }
        if (tau && (steps & 7) == 0)
            eps = fminf(eps, bits_f(load_relaxed_u32(tau)));
        if (g > eps) {
            steps_out = steps;
            return g;
        }
    }
    steps_out = steps;
    completed = true;
    return g;
}

// ------------------------------------------------------------------ seed pass
// Threshold seed (Sec. 4.3, first loop, generalised to k): the greedy bound
// of the first S candidates of each query (in the query's candidate order)
// is computed in full; the k-th smallest of them bounds the k-th smallest
// distance from above and becomes the query's starting threshold.
template <int D, int DIST>
__global__ void k_seed(const float *__restrict__ qv, const int64_t *__restrict__ qoff, int nq,
                       const float *__restrict__ aos, const int64_t *__restrict__ off,
                       const int32_t *__restrict__ len, int64_t N, const int32_t *__restrict__ order,
                       int S, int k, BandArgs ba, unsigned long long *seedslots, uint32_t *tau,
                       unsigned long long *ctr)
{
    const int q = blockIdx.y;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long steps_cnt = 0, pairs = 0;
    if (q < nq && p < S) {
        const int c = order ? order[(int64_t)q * N + p] : p;
        const int m = (int)(qoff[q + 1] - qoff[q]);
        const int n = len[c];
        const Band b = pair_band(ba, m, n);
        int steps;
        bool done;
        const float g = greedy_walk<D, DIST>(qv + qoff[q] * D, m, aos + off[c] * D, n, b, tsk_inf(),
                                             nullptr, steps, done);
        if (done && g != tsk_inf()) {
            topk_insert(seedslots + (int64_t)q * k, k, make_key(g, (uint32_t)c));
            tau_from_slots(seedslots + (int64_t)q * k, k, tau + q);
        }
        steps_cnt = steps;
        pairs = 1;
    }
    wave_count(ctr, C_SEED_STEPS, steps_cnt);
    wave_count(ctr, C_SEED_PAIRS, pairs);
}

// ------------------------------------------------------------------ bound pass
// One lane per candidate (64-series SoA tiles, coalesced), a group of
// queries per block.
//   DTW: LB_Box with the query's envelope around each candidate point (eq. (1)
//        with the two series' roles exchanged), fp32, summed over the
//        candidate's points in order; stops once the partial sum exceeds the
//        threshold (terms are >= 0).
//   DK:  every path starts at (0,0) and ends at (m-1,n-1), so
//        max(c(0,0), c(m-1,n-1)) <= squared DK; pairs passing it run the
//        greedy walk of Alg. 1 with early return at the running threshold,
//        and a completed walk lowers that threshold (Sec. 4.3).
// lbv[q][c] receives the bound if the pair survives (<= threshold), else
// +inf.  DEBUG mode: no threshold, writes lb / greedy value / moves instead.
struct BoundArgs {
    const float *qv;
    const int64_t *qoff;
    int nq;
    int qgroup;
    const float *soa;
    const int64_t *tile_off;
    const float *aos;
    const int64_t *off;
    const int32_t *len;
    int64_t N;
    int k;
    BandArgs ba;
    const float *env; // [nq][env_n][2][D] or null
    int env_n;
    // k_bound_lb_surv (DTW): after this many candidate points (a multiple
    // of 64), a pair whose partial sum extrapolated to all points stays
    // below tau keeps the partial sum as its bound; 0 = every point
    int lb_prefix;
    uint32_t *tau;
    unsigned long long *ubslots;
    float *lbv;
    unsigned long long *ctr;
    // debug outputs (DEBUG mode)
    float *dbg_lb;
    float *dbg_ub;
    int32_t *dbg_steps;
};

template <int D, int DIST, bool DEBUG>
__global__ __launch_bounds__(256) void k_bounds(BoundArgs a)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int q0 = blockIdx.y * a.qgroup;
    const int q1 = min(a.nq, q0 + a.qgroup);
    const bool valid = c < a.N;
    const int64_t tile = c >> 6;
    const int lane = (int)(c & 63);
    const int n = valid ? a.len[c] : 1;
    const float *tb = valid ? a.soa + a.tile_off[tile] + lane : a.soa;
    unsigned long long pruned = 0, steps_cnt = 0, pairs = 0;

    float c0[D], cl[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        c0[k] = valid ? tb[(0 * D + k) * 64] : 0.0f;
        cl[k] = valid ? tb[((int64_t)(n - 1) * D + k) * 64] : 0.0f;
    }

    for (int q = q0; q < q1; ++q) {
        if (!valid)
            continue;
        ++pairs;
        const int m = (int)(a.qoff[q + 1] - a.qoff[q]);
        const float *Q = a.qv + a.qoff[q] * D;
        const Band b = pair_band(a.ba, m, n);
        float tq = DEBUG ? tsk_inf() : bits_f(load_relaxed_u32(a.tau + q));
        float lb;
        if (DIST == DIST_DK) {
            float qa[D], qz[D];
            load_point<D>(Q, qa);
            load_point<D>(Q + (int64_t)(m - 1) * D, qz);
            lb = fmaxf(point_cost<D>(qa, c0), point_cost<D>(qz, cl));
            if (DEBUG || lb <= tq) {
                int steps;
                bool done;
                const float g = greedy_walk<D, DIST_DK>(Q, m, a.aos + a.off[c] * D, n, b, tq,
                                                        DEBUG ? nullptr : a.tau + q, steps, done);
                steps_cnt += steps;
                if (DEBUG) {
                    if (a.dbg_ub)
                        a.dbg_ub[(int64_t)q * a.N + c] = g;
                    if (a.dbg_steps)
                        a.dbg_steps[(int64_t)q * a.N + c] = steps;
                } else if (a.ubslots && done && g != tsk_inf() &&
                           g <= bits_f(load_relaxed_u32(a.tau + q))) {
                    // (no ubslots: a range query, whose threshold is fixed)
                    topk_insert(a.ubslots + (int64_t)q * a.k, a.k, make_key(g, (uint32_t)c));
                    tau_from_slots(a.ubslots + (int64_t)q * a.k, a.k, a.tau + q);
                }
            }
        } else {
            // LB_Box, candidate points against the query envelope.
            float acc = 0.0f;
            if (a.env && n == a.env_n) {
                const float *E = a.env + (int64_t)q * a.env_n * 2 * D;
                for (int j = 0; j < n; ++j) {
                    float x[D];
#pragma unroll
                    for (int k = 0; k < D; ++k)
                        x[k] = tb[((int64_t)j * D + k) * 64];
                    acc = box_term<D>(x, E + (int64_t)j * 2 * D, E + (int64_t)j * 2 * D + D) + acc;
                    if (!DEBUG && acc > tq)
                        break;
                }
            } else {
                for (int j = 0; j < n; ++j) {
                    float x[D], lo[D], hi[D];
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        x[k] = tb[((int64_t)j * D + k) * 64];
                        lo[k] = tsk_inf();
                        hi[k] = -tsk_inf();
                    }
                    int ilo, ihi;
                    band_rows(b, j, m, ilo, ihi);
                    for (int i = ilo; i <= ihi; ++i) {
#pragma unroll
                        for (int k = 0; k < D; ++k) {
                            const float v = Q[(int64_t)i * D + k];
                            lo[k] = fminf(lo[k], v);
                            hi[k] = fmaxf(hi[k], v);
                        }
                    }
                    acc = box_term<D>(x, lo, hi) + acc;
                    if (!DEBUG && acc > tq)
                        break;
                }
            }
            steps_cnt += n;
            lb = acc;
            if (DEBUG) {
                int steps;
                bool done;
                const float g = greedy_walk<D, DIST_DTW>(Q, m, a.aos + a.off[c] * D, n, b, tsk_inf(),
                                                         nullptr, steps, done);
                if (a.dbg_ub)
                    a.dbg_ub[(int64_t)q * a.N + c] = g;
                if (a.dbg_steps)
                    a.dbg_steps[(int64_t)q * a.N + c] = steps;
            }
        }
        if (DEBUG) {
            if (a.dbg_lb)
                a.dbg_lb[(int64_t)q * a.N + c] = lb;
        } else {
            tq = bits_f(load_relaxed_u32(a.tau + q));
            const bool keep = lb <= tq;
            a.lbv[(int64_t)q * a.N + c] = keep ? lb : tsk_inf();
            pruned += keep ? 0 : 1;
        }
    }
    if (!DEBUG) {
        wave_count(a.ctr, C_BOUND_PRUNED, pruned);
        wave_count(a.ctr, C_PAIRS, pairs);
    }
    wave_count(a.ctr, C_BOUND_STEPS, steps_cnt);
}

// ------------------------------------------------------------------ compaction
// Survivors of one query, in the query's candidate order, re-checked against
// the current threshold: surv[q][0..cnt).  One block of 1024 per query; each
// pass takes 4096 positions, 4 consecutive ones per thread (so the survivors
// of a thread precede those of the next), ranks them by a block-wide prefix
// sum of the per-thread counts and writes them in order.
// Candidate order: order[q][p] if given, else perm[p] (length-sorted
// positions) if given, else p.  lbv is indexed by candidate id, except after
// the length-bucket bound pass, which writes it by position (then perm maps
// positions to ids and inv ids to positions).
constexpr int COMPACT_PER = 4;
static __global__ __launch_bounds__(1024) void k_compact(const float *__restrict__ lbv, int64_t N,
                                                  const int32_t *__restrict__ order,
                                                  const int32_t *__restrict__ perm,
                                                  const int32_t *__restrict__ inv,
                                                  const uint32_t *__restrict__ tau,
                                                  int32_t *__restrict__ surv, int32_t *__restrict__ cnt,
                                                  int32_t *__restrict__ max_cnt,
                                                  unsigned long long *ctr)
{
    const int q = blockIdx.x;
    __shared__ int wave_tot[2][16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const float tq = bits_f(tau[q]);
    const float *L = lbv + (int64_t)q * N;
    int32_t *out = surv + (int64_t)q * N;
    int base = 0;
    unsigned long long late = 0;
    int buf = 0;
    for (int64_t p0 = 0; p0 < N; p0 += 1024 * COMPACT_PER, buf ^= 1) {
        const int64_t pb = p0 + (int64_t)threadIdx.x * COMPACT_PER;
        int cs[COMPACT_PER];
        bool keep[COMPACT_PER];
        int mine = 0;
#pragma unroll
        for (int u = 0; u < COMPACT_PER; ++u) {
            const int64_t p = pb + u;
            cs[u] = -1;
            keep[u] = false;
            if (p < N) {
                int64_t li;
                int c;
                if (order) {
                    c = order[(int64_t)q * N + p];
                    li = inv ? inv[c] : c;
                } else {
                    c = perm ? perm[p] : (int)p;
                    li = p;
                }
                const float lb = L[li];
                cs[u] = c;
                keep[u] = lb <= tq;
                late += (lb != tsk_inf() && !keep[u]) ? 1 : 0;
                mine += keep[u] ? 1 : 0;
            }
        }
        // inclusive prefix sum of the counts over the wave, then over waves
        int inc = mine;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(inc, o, 64);
            if (lane >= o)
                inc += t;
        }
        if (lane == 63)
            wave_tot[buf][wv] = inc;
        __syncthreads(); // (the other buffer is free: read before this barrier)
        int off = base + inc - mine, all = 0;
        for (int w = 0; w < 16; ++w) {
            const int t = wave_tot[buf][w];
            off += w < wv ? t : 0;
            all += t;
        }
#pragma unroll
        for (int u = 0; u < COMPACT_PER; ++u)
            if (keep[u])
                out[off++] = cs[u];
        base += all;
    }
    wave_count(ctr, C_BOUND_PRUNED, late);
    if (threadIdx.x == 0) {
        cnt[q] = base;
        atomicMax(max_cnt, base);
    }
}

// Survivors of one query ordered by ascending bound instead of candidate
// order (a counting sort on bits 18.. of the non-negative fp32 bound, 8192
// buckets of 2^-5 relative width; bucket-mates in arbitrary order): the
// pairs most likely to be neighbours run first, so the threshold falls
// early, and pairs of similar bound share a wave.  Same survivors as
// k_compact (tau is fixed while it runs: no DP of this chunk has started).
// cap < N keeps only the first cap survivors of that order (the cap
// smallest bounds, up to the order inside the last bucket they reach).
// With cnt_in the candidates are a survivor list (order, its counts cnt_in;
// the output surv must be another buffer), re-ranked by their bounds.
// One block of 1024 per query; SURV_BUCKETS counters in dynamic LDS.
constexpr int SURV_BUCKETS = 8192;
constexpr int SURV_SHIFT = 18;
static __global__ __launch_bounds__(1024) void k_compact_sorted(
    const float *__restrict__ lbv, int64_t N, const int32_t *__restrict__ order,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ inv,
    const uint32_t *__restrict__ tau, int32_t *__restrict__ surv, int32_t *__restrict__ cnt,
    int32_t *__restrict__ max_cnt, unsigned long long *ctr, int64_t cap,
    const int32_t *__restrict__ cnt_in)
{
    extern __shared__ int32_t hist[];
    __shared__ int32_t wsum[16];
    const int q = blockIdx.x;
    const int tid = threadIdx.x;
    const float tq = bits_f(tau[q]);
    for (int b = tid; b < SURV_BUCKETS; b += 1024)
        hist[b] = 0;
    __syncthreads();
    unsigned long long late = 0;
    auto cand = [&](int64_t p, int &c, float &lb) {
        int64_t li;
        if (order) {
            c = order[(int64_t)q * N + p];
            li = inv ? inv[c] : c;
        } else {
            c = perm ? perm[p] : (int)p;
            li = p;
        }
        lb = lbv[(int64_t)q * N + li];
    };
    // cnt_in: re-rank a survivor list (order[q][0 .. cnt_in[q])) instead of
    // every candidate
    const int64_t P = cnt_in ? (int64_t)cnt_in[q] : N;
    for (int64_t p = tid; p < P; p += 1024) {
        int c;
        float lb;
        cand(p, c, lb);
        if (lb <= tq)
            atomicAdd(&hist[min(__float_as_uint(lb) >> SURV_SHIFT, (uint32_t)SURV_BUCKETS - 1)], 1);
        else if (lb != tsk_inf())
            ++late;
    }
    __syncthreads();
    constexpr int PER = SURV_BUCKETS / 1024;
    int loc[PER];
    int tot = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        loc[i] = tot;
        tot += hist[tid * PER + i];
    }
    const int lane = tid & 63, wv = tid >> 6;
    int inc = tot;
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
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i)
        hist[tid * PER + i] = excl + loc[i];
    __syncthreads();
    for (int64_t p = tid; p < P; p += 1024) {
        int c;
        float lb;
        cand(p, c, lb);
        if (lb <= tq) {
            const int pos =
                atomicAdd(&hist[min(__float_as_uint(lb) >> SURV_SHIFT, (uint32_t)SURV_BUCKETS - 1)], 1);
            if (pos < cap)
                surv[(int64_t)q * N + pos] = c;
        }
    }
    wave_count(ctr, C_BOUND_PRUNED, late);
    if (tid == 0) {
        int all = 0;
        for (int w = 0; w < 16; ++w)
            all += wsum[w];
        all = (int)min((int64_t)all, cap);
        cnt[q] = all;
        atomicMax(max_cnt, all);
    }
}

// ------------------------------------------------------------------ compaction, many blocks per query
// The same survivors as k_compact / k_compact_sorted in the plain candidate
// order (lbv indexed by id, position = id), for long candidate lists: each
// wave owns a segment of SEG_LEN consecutive positions of one query, so a
// chunk of queries spreads over nq * ceil(N / SEG_LEN) waves instead of nq
// blocks (one block per query leaves most CUs idle and each block bound by
// the latency of its sequential loads).  tau is fixed while they run.
constexpr int SEG_LEN = 4096;   // positions per wave
constexpr int SEG_WAVES = 4;    // waves per block

// The lbv values of positions p .. p+3 of a row (+inf past the end, which
// every caller masks out by position: a threshold of +inf keeps +inf).
__device__ __forceinline__ void load_lbv4(const float *__restrict__ L, int64_t p, int64_t end,
                                          bool vec, float (&v)[4])
{
    if (vec && p + 3 < end) {
        const float4 x = *reinterpret_cast<const float4 *>(L + p);
        v[0] = x.x;
        v[1] = x.y;
        v[2] = x.z;
        v[3] = x.w;
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            v[i] = p + i < end ? L[p + i] : tsk_inf();
    }
}

// The candidates at positions p .. p+3 of a query's order (O: its row of
// the order array, or null for the plain order) and their bounds.
__device__ __forceinline__ void load_cand4(const float *__restrict__ L, const int32_t *__restrict__ O,
                                           int64_t p, int64_t end, bool vec, float (&v)[4],
                                           int32_t (&id)[4])
{
    if (O == nullptr) {
        load_lbv4(L, p, end, vec, v);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            id[i] = (int32_t)(p + i);
        return;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        id[i] = p + i < end ? O[p + i] : 0;
        v[i] = p + i < end ? L[id[i]] : tsk_inf();
    }
}

// Pass 1: each wave counts the survivors (lb <= tau) of its segment into
// segcnt[q][seg]; SORTED also counts them by bound bucket into hist[q][b]
// (global atomics: survivors are few).  Pairs above tau are counted pruned.
template <bool SORTED>
__global__ __launch_bounds__(64 * SEG_WAVES) void k_seg_count(
    const float *__restrict__ lbv, int64_t N, const int32_t *__restrict__ order,
    const uint32_t *__restrict__ tau, int32_t *__restrict__ segcnt, int32_t *__restrict__ hist,
    unsigned long long *ctr)
{
    const int q = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int64_t nseg = (N + SEG_LEN - 1) / SEG_LEN;
    const int64_t seg = (int64_t)blockIdx.x * SEG_WAVES + (threadIdx.x >> 6);
    if (seg >= nseg)
        return;
    const float tq = bits_f(tau[q]);
    const float *L = lbv + (int64_t)q * N;
    const bool vec = ((uint64_t)L & 15u) == 0;
    const int64_t p0 = seg * SEG_LEN, p1 = min(N, p0 + SEG_LEN);
    const int32_t *O = order ? order + (int64_t)q * N : nullptr;
    int mine = 0;
    unsigned long long late = 0;
    for (int64_t p = p0 + lane * 4; p < p1; p += 256) {
        float v[4];
        int32_t id[4];
        load_cand4(L, O, p, p1, vec, v, id);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (p + i >= p1)
                continue;
            if (v[i] <= tq) {
                ++mine;
                if (SORTED)
                    atomicAdd(&hist[(int64_t)q * SURV_BUCKETS +
                                    min(__float_as_uint(v[i]) >> SURV_SHIFT, (uint32_t)SURV_BUCKETS - 1)],
                              1);
            } else if (v[i] != tsk_inf()) {
                ++late;
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        mine += __shfl_xor(mine, o, 64);
    if (lane == 0)
        segcnt[(int64_t)q * nseg + seg] = mine;
    wave_count(ctr, C_BOUND_PRUNED, late);
}

// Sum of segcnt[q][0 .. seg) over the wave (every lane gets it).
__device__ __forceinline__ int seg_prefix(const int32_t *__restrict__ segcnt, int64_t nseg, int q,
                                          int64_t seg, int lane)
{
    int s = 0;
    for (int64_t i = lane; i < seg; i += 64)
        s += segcnt[(int64_t)q * nseg + i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        s += __shfl_xor(s, o, 64);
    return s;
}

// Pass 2, candidate order: each wave writes its segment's survivors at the
// offset of the segments before it, in position order (4 consecutive
// positions per lane, ranked by a wave prefix sum); the query's last
// segment writes its count.
static __global__ __launch_bounds__(64 * SEG_WAVES) void k_seg_scatter(
    const float *__restrict__ lbv, int64_t N, const int32_t *__restrict__ order,
    const uint32_t *__restrict__ tau, const int32_t *__restrict__ segcnt,
    int32_t *__restrict__ surv, int32_t *__restrict__ cnt, int32_t *__restrict__ max_cnt)
{
    const int q = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int64_t nseg = (N + SEG_LEN - 1) / SEG_LEN;
    const int64_t seg = (int64_t)blockIdx.x * SEG_WAVES + (threadIdx.x >> 6);
    if (seg >= nseg)
        return;
    const float tq = bits_f(tau[q]);
    const float *L = lbv + (int64_t)q * N;
    const bool vec = ((uint64_t)L & 15u) == 0;
    int32_t *out = surv + (int64_t)q * N;
    const int64_t p0 = seg * SEG_LEN, p1 = min(N, p0 + SEG_LEN);
    int base = seg_prefix(segcnt, nseg, q, seg, lane);
    if (seg == nseg - 1 && lane == 0) {
        const int all = base + segcnt[(int64_t)q * nseg + seg];
        cnt[q] = all;
        atomicMax(max_cnt, all);
    }
    if (segcnt[(int64_t)q * nseg + seg] == 0)
        return;
    const int32_t *O = order ? order + (int64_t)q * N : nullptr;
    for (int64_t p = p0 + lane * 4; p - lane * 4 < p1; p += 256) {
        float v[4];
        int32_t id[4];
        load_cand4(L, O, p, p1, vec, v, id);
        bool keep[4];
        int mine = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            keep[i] = p + i < p1 && v[i] <= tq;
            mine += keep[i] ? 1 : 0;
        }
        int inc = mine;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(inc, o, 64);
            if (lane >= o)
                inc += t;
        }
        int at = base + inc - mine;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (keep[i])
                out[at++] = id[i];
        base += __shfl(inc, 63, 64);
    }
}

// Sorted pass 2: exclusive prefix of each query's bucket counts, in place
// (one block of 1024 per query, 8 buckets per thread); count = min(total,
// cap).
static __global__ __launch_bounds__(1024) void k_seg_bucket_scan(int32_t *__restrict__ hist,
                                                                 int64_t cap, int32_t *__restrict__ cnt,
                                                                 int32_t *__restrict__ max_cnt)
{
    __shared__ int32_t wsum[16];
    const int q = blockIdx.x;
    const int tid = threadIdx.x;
    int32_t *h = hist + (int64_t)q * SURV_BUCKETS;
    constexpr int PER = SURV_BUCKETS / 1024;
    int loc[PER];
    int tot = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        loc[i] = tot;
        tot += h[tid * PER + i];
    }
    const int lane = tid & 63, wv = tid >> 6;
    int inc = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(inc, o, 64);
        if (lane >= o)
            inc += t;
    }
    if (lane == 63)
        wsum[wv] = inc;
    __syncthreads();
    int base = 0, all = 0;
    for (int w = 0; w < 16; ++w) {
        base += w < wv ? wsum[w] : 0;
        all += wsum[w];
    }
    const int excl = base + inc - tot;
#pragma unroll
    for (int i = 0; i < PER; ++i)
        h[tid * PER + i] = excl + loc[i];
    if (tid == 0) {
        all = (int)min((int64_t)all, cap);
        cnt[q] = all;
        atomicMax(max_cnt, all);
    }
}

// Sorted pass 3: each survivor takes the next slot of its bound bucket
// (bucket-mates in arbitrary order, as in k_compact_sorted); slots from cap
// on are dropped.
static __global__ __launch_bounds__(64 * SEG_WAVES) void k_seg_bucket_scatter(
    const float *__restrict__ lbv, int64_t N, const uint32_t *__restrict__ tau,
    const int32_t *__restrict__ segcnt, int32_t *__restrict__ hist, int64_t cap,
    int32_t *__restrict__ surv)
{
    const int q = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int64_t nseg = (N + SEG_LEN - 1) / SEG_LEN;
    const int64_t seg = (int64_t)blockIdx.x * SEG_WAVES + (threadIdx.x >> 6);
    if (seg >= nseg || segcnt[(int64_t)q * nseg + seg] == 0)
        return;
    const float tq = bits_f(tau[q]);
    const float *L = lbv + (int64_t)q * N;
    const bool vec = ((uint64_t)L & 15u) == 0;
    const int64_t p0 = seg * SEG_LEN, p1 = min(N, p0 + SEG_LEN);
    for (int64_t p = p0 + lane * 4; p < p1; p += 256) {
        float v[4];
        load_lbv4(L, p, p1, vec, v);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (p + i < p1 && v[i] <= tq) {
                const int pos = atomicAdd(
                    &hist[(int64_t)q * SURV_BUCKETS +
                          min(__float_as_uint(v[i]) >> SURV_SHIFT, (uint32_t)SURV_BUCKETS - 1)],
                    1);
                if (pos < cap)
                    surv[(int64_t)q * N + pos] = (int32_t)(p + i);
            }
        }
    }
}

// ------------------------------------------------------------------ seed set from segment minima
// The threshold seed's candidate set for long lists: the 2*cap segments of
// a query's candidates (plain order) each give the candidate of smallest
// bound (ties to the lower id), and the cap smallest of those minima form
// the seed set, in ascending bound.  Any seed set leaves the results exact
// (the seed only sets a starting threshold that the k nearest never
// exceed); this one costs one read of the bounds instead of a counting sort
// of every candidate.  k_seg_min: a wave per segment.
constexpr int SEEDSEG_MAX = 1024; // 2 * cap at most

static __global__ __launch_bounds__(256) void k_seg_min(const float *__restrict__ lbv, int64_t N,
                                                        int nseg, unsigned long long *__restrict__ keys)
{
    const int q = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int sg = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (sg >= nseg)
        return;
    const int64_t len = (N + nseg - 1) / nseg;
    const int64_t p0 = (int64_t)sg * len, p1 = min(N, p0 + len);
    const float *L = lbv + (int64_t)q * N;
    unsigned long long best = ~0ull;
    for (int64_t p = p0 + lane; p < p1; p += 64) {
        const unsigned long long k =
            ((unsigned long long)__float_as_uint(L[p]) << 32) | (unsigned long long)(uint32_t)p;
        best = k < best ? k : best;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long other = __shfl_xor(best, o, 64);
        best = other < best ? other : best;
    }
    if (lane == 0)
        keys[(int64_t)q * SEEDSEG_MAX + sg] = best;
}

// One block of 1024 per query: bitonic sort of the nseg segment minima
// (padded to a power of two with the largest key), the cap smallest ids
// to surv[q][0 .. cap).
static __global__ __launch_bounds__(1024) void k_seg_pick(const unsigned long long *__restrict__ keys,
                                                          int nseg, int cap, int64_t N,
                                                          int32_t *__restrict__ surv,
                                                          int32_t *__restrict__ cnt,
                                                          int32_t *__restrict__ max_cnt)
{
    __shared__ unsigned long long k[SEEDSEG_MAX];
    const int q = blockIdx.x;
    const int tid = threadIdx.x;
    int P = 1;
    while (P < nseg)
        P <<= 1;
    for (int i = tid; i < P; i += 1024)
        k[i] = i < nseg ? keys[(int64_t)q * SEEDSEG_MAX + i] : ~0ull;
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < P; i += 1024) {
                const int jx = i ^ stride;
                if (jx > i) {
                    const bool up = (i & size) == 0;
                    const unsigned long long a = k[i], b = k[jx];
                    if ((a > b) == up) {
                        k[i] = b;
                        k[jx] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    const int take = min(cap, nseg);
    for (int i = tid; i < take; i += 1024)
        surv[(int64_t)q * N + i] = (int32_t)(uint32_t)(k[i] & 0xffffffffull);
    if (tid == 0) {
        cnt[q] = take;
        atomicMax(max_cnt, take);
    }
}

// ------------------------------------------------------------------ range query output
// Hits of one query in ascending id order: cnt pass (one block per query),
// then fill at the query's offset; DK keys leave as correctly rounded sqrt.
static __global__ __launch_bounds__(256) void k_range_count(const float *__restrict__ hits,
                                                            int64_t N, int64_t *__restrict__ cnt)
{
    const int q = blockIdx.x;
    __shared__ int64_t part[4];
    int64_t c = 0;
    for (int64_t p = threadIdx.x; p < N; p += 256)
        c += hits[(int64_t)q * N + p] != tsk_inf() ? 1 : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0)
        cnt[q] = part[0] + part[1] + part[2] + part[3];
}

template <int DIST>
__global__ __launch_bounds__(256) void k_range_fill(const float *__restrict__ hits, int64_t N,
                                                    const int64_t *__restrict__ qoffs,
                                                    int64_t *__restrict__ ids,
                                                    float *__restrict__ dist)
{
    const int q = blockIdx.x;
    __shared__ int wave_tot[4];
    __shared__ int64_t base_s;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (threadIdx.x == 0)
        base_s = qoffs[q];
    __syncthreads();
    for (int64_t p0 = 0; p0 < N; p0 += 256) {
        const int64_t p = p0 + threadIdx.x;
        const float v = p < N ? hits[(int64_t)q * N + p] : tsk_inf();
        const bool hit = v != tsk_inf();
        const unsigned long long bal = __ballot(hit);
        const int rank = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0)
            wave_tot[wv] = __popcll(bal);
        __syncthreads();
        int64_t off = base_s;
        for (int w = 0; w < wv; ++w)
            off += wave_tot[w];
        if (hit) {
            ids[off + rank] = p;
            dist[off + rank] = DIST == DIST_DK ? sqrt_rn_f32(v) : v;
        }
        __syncthreads();
        if (threadIdx.x == 0)
            base_s += wave_tot[0] + wave_tot[1] + wave_tot[2] + wave_tot[3];
        __syncthreads();
    }
}

// ------------------------------------------------------------------ general DP
// One wave per pair: the quadratic DP of Sec. 2.1 (DTW: cost + min of the
// three predecessors; DK: max(cost, min)), with D(-1,-1) = 0 and every other
// outside cell +inf, restricted to the band.  Rows are processed in strips
// of 64 R (R consecutive rows per lane: 4 amortises the per-step work over
// more cells, 1 and 2 waste fewer out-of-band cells on narrow bands); inside a
// strip lane l works on column s - l at step s (a skewed wavefront),
// receiving the row below from lane l-1 of the previous step; the strip's
// top row is handed to the next strip through a per-wave buffer.
// Cells above tau are dead (the sparse-DK semantics of Alg. 3; for DTW the
// same holds because values only grow along a path): they keep their value,
// which can only feed values above tau, and liveness tests compare with tau.
// A strip hands up only columns up to its last live one.  With
// sigma(i, j) = j + floor(i / R) a path moves sigma by 0, 1 or 2 per move,
// so it cannot skip two consecutive steps of a strip: when two consecutive
// steps are all dead and no live input from the strip below is still
// pending, the rest of the strip is dead, and if it handed no live value up
// the whole pair is > tau (abandoned).  Returns the value, or +inf if > tau.
template <int D, int DIST, int R>
__device__ float dp_wave_pair(const float *__restrict__ qp, int m, const float *__restrict__ cp, int n,
                              const Band &band_in, const uint32_t *tau_ptr, float *__restrict__ tbuf,
                              unsigned long long &cells, unsigned long long &valid)
{
    // Both distances are symmetric in the two series (the point cost is,
    // bit for bit: fl(s - t) = -fl(t - s); so is the band), and every cell
    // keeps its value when the matrix is transposed: the longer series runs
    // down the strips, so a strip's 64R rows are filled and a slanted band
    // crosses fewer of its columns.
    Band band = band_in;
    if (m < n) {
        const float *t = qp;
        qp = cp;
        cp = t;
        const int tm = m;
        m = n;
        n = tm;
        const int64_t ta = band.A;
        band.A = band.B;
        band.B = ta;
    }
    const int lane = threadIdx.x & 63;
    const float tau = tau_ptr ? bits_f(load_relaxed_u32(tau_ptr)) : tsk_inf();
    float result = tsk_inf();
    int in_max = -1;  // largest column with a live value in the strip input
    int js_prev = 0;  // first column of the previous strip
    float *tb_in = tbuf, *tb_out = tbuf + n;
    constexpr int H = 64 * R; // strip height
    for (int base = 0; base < m; base += H) {
        if (base > 0 && in_max < 0)
            break;
        const bool last_strip = base + H >= m;
        float qr[R][D];
        // row r's band columns: j is inside iff (unsigned)(j - jlo) <= span;
        // rows past the query or with an empty band never are
        int jlo[R];
        unsigned span[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = base + R * lane + r;
            int lo = 1 << 30, hi = -1;
            if (i < m) {
                load_point<D>(qp + (int64_t)i * D, qr[r]);
                band_cols(band, i, n, lo, hi);
            } else {
#pragma unroll
                for (int k = 0; k < D; ++k)
                    qr[r][k] = 0.0f;
            }
            const bool empty = lo > hi;
            jlo[r] = empty ? (1 << 30) : lo;
            span[r] = empty ? 0u : (unsigned)(hi - lo);
        }
        int js, je, tmp;
        band_cols(band, base, n, js, tmp);
        band_cols(band, min(base + H - 1, m - 1), n, tmp, je);
        if (js > je)
            break;
        int out_max = -1;
        float Dp[R];
#pragma unroll
        for (int r = 0; r < R; ++r)
            Dp[r] = tsk_inf();
        // lane 0's first cell (base, js) has the lower-left predecessor
        // (base-1, js-1), which a band can leave inside and finite; the
        // previous strip wrote it iff js-1 is within its columns
        float recv_prev = tsk_inf(), my_top = tsk_inf();
        if (lane == 0 && base > 0 && js - 1 >= js_prev && js - 1 <= in_max)
            recv_prev = tb_in[js - 1];
        // cell (0,0): its lower-left predecessor is the virtual D(-1,-1) = 0
        if (lane == 0 && base == 0)
            recv_prev = 0.0f;
        bool alive_prev = true;
        const int nsteps = je - js + 64;
        // software pipeline: the candidate point (and lane 0's strip input)
        // of step s is loaded two steps ahead, so a step never waits on
        // memory latency (single pairs run with few waves per SIMD)
        auto cand = [&](int jj, float (&out)[D]) {
            const int jc = min(max(jj, 0), n - 1);
            load_point<D>(cp + (int64_t)jc * D, out);
        };
        auto strip_in = [&](int jj) -> float {
            return (lane == 0 && base > 0 && jj >= 0 && jj <= in_max) ? tb_in[jj] : tsk_inf();
        };
        float c0[D], c1[D];
        cand(js - lane, c0);
        cand(js - lane + 1, c1);
        float t0 = strip_in(js), t1 = strip_in(js + 1);
        for (int s = 0; s < nsteps; ++s) {
            const int j = js + s - lane;
            float recv = __shfl_up(my_top, 1, 64);
            if (lane == 0)
                recv = t0;
            const bool jv = j >= 0 && j < n;
            float cv[D];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                cv[k] = c0[k]; // a clamped point where j is outside: masked below
                c0[k] = c1[k];
            }
            cand(j + 2, c1);
            t0 = t1;
            t1 = strip_in(js + s + 2);
            float down = recv, diag = recv_prev;
            float vmin = tsk_inf();
            float Dc[R];
            // Out-of-band cells get an infinite cost.  Cells above tau keep
            // their (exact) value: every extension of them stays above tau,
            // so liveness is tested against tau instead of killing them.
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const bool ok = (unsigned)(j - jlo[r]) <= span[r];
                const float pred = min3f(diag, down, Dp[r]);
                float cst = point_cost<D>(qr[r], cv);
                cst = ok ? cst : tsk_inf();
                const float v = DIST == DIST_DK ? fmaxf(cst, pred) : cst + pred;
                valid += __popcll(__ballot(ok));
                diag = Dp[r];
                down = v;
                Dc[r] = v;
                vmin = fminf(vmin, v);
            }
            const bool any = vmin <= tau;
#pragma unroll
            for (int r = 0; r < R; ++r)
                Dp[r] = Dc[r];
            recv_prev = recv;
            my_top = Dc[R - 1];
            if (!last_strip && lane == 63 && jv) {
                tb_out[j] = Dc[R - 1];
                if (Dc[R - 1] <= tau)
                    out_max = j;
            }
            if (last_strip && j == n - 1) {
                const int rr = m - 1 - base - R * lane;
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (rr == r)
                        result = Dc[r];
            }
            cells += R;
            const bool alive_now = __ballot(any) != 0ull;
            if (!alive_now && !alive_prev && js + s > in_max)
                break;
            alive_prev = alive_now;
        }
        in_max = __shfl(out_max, 63, 64);
        js_prev = js;
        float *t = tb_in;
        tb_in = tb_out;
        tb_out = t;
        __threadfence_block();
        if (last_strip)
            break;
    }
    result = wave_min(result);
    return result <= tau ? result : tsk_inf();
}

struct DpArgs {
    const float *qv;
    const int64_t *qoff;
    int nq;
    const float *aos;
    const int64_t *off;
    const int32_t *len;
    int64_t N;
    int k;
    BandArgs ba;
    uint32_t *tau;
    const float *lbv;
    const int32_t *lb_inv; // lbv index of a candidate id (null: the id itself)
    const int32_t *surv;
    const int32_t *surv_cnt;
    const int32_t *max_cnt;
    unsigned long long *resslots;
    unsigned long long *work;
    float *tbuf;
    int tb_stride;
    unsigned long long *ctr;
    float *out_all;     // ALLPAIRS: [nq][N]
    const int2 *fb;     // FALLBACK: (query, candidate) list
    const unsigned long long *fb_count;
    int rows_per_lane;  // R of the strips: 1, 2 or 4
    float *range_out;   // range query: [nq][N] keys of hits, else null (top-k)
};

enum { DPW_SURV = 0, DPW_ALLPAIRS = 1, DPW_FALLBACK = 2 };

// MODE: DPW_SURV walks the compacted survivors (query-interleaved ranks),
// DPW_ALLPAIRS every pair with no threshold (tsk_pair_distances),
// DPW_FALLBACK the pairs the lane-per-pair kernels handed over.
template <int D, int DIST, int MODE, int R>
__global__ __launch_bounds__(256) void k_dp_wave(DpArgs a)
{
    constexpr bool ALLPAIRS = MODE == DPW_ALLPAIRS;
    const int lane = threadIdx.x & 63;
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    float *tb = a.tbuf + gw * a.tb_stride;
    unsigned long long cells = 0, valid = 0, started = 0, completed = 0, abandoned = 0, late = 0;
    const int64_t total = ALLPAIRS ? (int64_t)a.nq * a.N
                          : MODE == DPW_FALLBACK ? (int64_t)(*a.fb_count)
                                                 : (int64_t)a.nq * (int64_t)(*a.max_cnt);
    if (total == 0)
        return; // nothing handed over: no contended counter traffic
    for (;;) {
        unsigned long long t = 0;
        if (lane == 0)
            t = atomicAdd(a.work, 1ull);
        t = uniform_u64(t);
        if (t >= (unsigned long long)total)
            break;
        int q, c;
        if (ALLPAIRS) {
            q = (int)(t / a.N);
            c = (int)(t % a.N);
        } else if (MODE == DPW_FALLBACK) {
            const int2 item = a.fb[t];
            q = item.x;
            c = item.y;
            if (a.lbv[(int64_t)q * a.N + (a.lb_inv ? a.lb_inv[c] : c)] > bits_f(load_relaxed_u32(a.tau + q))) {
                ++late;
                continue;
            }
        } else {
            q = (int)(t % a.nq);
            const int r = (int)(t / a.nq);
            if (r >= a.surv_cnt[q])
                continue;
            c = a.surv[(int64_t)q * a.N + r];
            if (a.lbv[(int64_t)q * a.N + (a.lb_inv ? a.lb_inv[c] : c)] > bits_f(load_relaxed_u32(a.tau + q))) {
                ++late;
                continue;
            }
        }
        const int m = (int)(a.qoff[q + 1] - a.qoff[q]);
        const int n = a.len[c];
        const Band b = pair_band(a.ba, m, n);
        const float res = dp_wave_pair<D, DIST, R>(a.qv + a.qoff[q] * D, m, a.aos + a.off[c] * D, n, b,
                                                ALLPAIRS ? nullptr : a.tau + q, tb, cells, valid);
        if (ALLPAIRS) {
            if (lane == 0)
                a.out_all[t] = res;
        } else {
            ++started; // (the fast kernels do not count the pairs they hand over)
            if (res != tsk_inf()) {
                ++completed;
                if (lane == 0 && res <= bits_f(load_relaxed_u32(a.tau + q))) {
                    if (a.range_out) {
                        a.range_out[(int64_t)q * a.N + c] = res;
                    } else {
                        topk_insert(a.resslots + (int64_t)q * a.k, a.k,
                                    make_key(res, (uint32_t)c));
                        tau_from_slots(a.resslots + (int64_t)q * a.k, a.k, a.tau + q);
                    }
                }
            } else {
                ++abandoned;
            }
        }
    }
    if (lane == 0) {
        if (cells)
            ctr_add(a.ctr, C_DP_CELLS, cells * 64ull);
        if (valid) {
            ctr_add(a.ctr, C_VALID_CELLS, valid);
            ctr_add(a.ctr, C_VALID_GEN, valid);
        }
        if (!ALLPAIRS) {
            if (started)
                ctr_add(a.ctr, C_DP_STARTED, started);
            if (completed)
                ctr_add(a.ctr, C_DP_COMPLETED, completed);
            if (abandoned)
                ctr_add(a.ctr, C_DP_ABANDONED, abandoned);
            if (late)
                ctr_add(a.ctr, C_BOUND_PRUNED, late);
        }
    }
}

// ------------------------------------------------------------------ finalize
// Slots -> (id, distance) rows, ascending; DK distances are the correctly
// rounded square root of the squared key; empty ranks -> (-1, +inf).
template <int DIST>
__global__ void k_finalize(const unsigned long long *__restrict__ resslots, int nq, int k,
                           int64_t *__restrict__ out_ids, float *__restrict__ out_dist)
{
    const int q = blockIdx.x;
    const int r = threadIdx.x;
    if (q >= nq || r >= k)
        return;
    const unsigned long long key = resslots[(int64_t)q * k + r];
    int64_t id = -1;
    float dist = tsk_inf();
    if (key != TSK_KEY_EMPTY) {
        id = (int64_t)(uint32_t)(key & 0xFFFFFFFFull);
        const float v = bits_f((uint32_t)(key >> 32));
        dist = DIST == DIST_DK ? sqrt_rn_f32(v) : v;
    }
    out_ids[(int64_t)q * k + r] = id;
    out_dist[(int64_t)q * k + r] = dist;
}

} // namespace tsk
