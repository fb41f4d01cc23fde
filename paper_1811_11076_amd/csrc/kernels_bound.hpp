// Bound-pass kernels tuned for gfx950: LB_Box for DTW and the greedy bound
// of Alg. 1 for DK, one lane per candidate.
#pragma once

#include "kernels_fast.hpp"

namespace tsk {

// floats of LDS per lane for the greedy walk's candidate ring, and the
// distance between two lanes' rings: odd, so that the 64 lanes' rings start
// in different LDS banks (a stride of 128 floats puts every lane's slot s in
// one bank and serialises each ring access 64 ways)
constexpr int WALK_RING_FLOATS = 128;
constexpr int WALK_RING_STRIDE = WALK_RING_FLOATS + 1;

// Greedy walk of Alg. 1 (Sec. 4.1), same moves, tie order and value as
// greedy_walk().  Latency layout for gfx950: the query comes from LDS (row
// stride DP floats); the candidate goes through a lane-private LDS ring of
// RN = 4B points (slot = point mod RN; B = 8 points per block for DP = 4, 4
// for DP = 8, 2 for DP = 12 and 16, 1 for DP = 24 and 32, so a ring is at
// most 128 floats).  Every B moves, on the
// same moves for every lane still walking (lanes advance j at their own
// pace, and a refill taken by some lanes only would wait on loads that
// others had just issued into the same registers), each lane writes the B
// points it loaded at the previous refill, [jb' + 3B, jb' + 4B) for its
// block jb' then, and requests [jb + 3B, jb + 4B) for its current block
// jb = B floor(j / B); a lane that has not changed block rewrites the same
// points.  After a refill the ring holds the 4B points from jb' on, and a
// walk of B moves from j < jb' + 2B reads points below jb' + 3B: every
// point read is staged, and the slots written hold points behind the walk.
// Global loads are thus waited on B moves after they were issued.  The
// points at j, j+1, j+2 (and i, i+1, i+2) sit in registers, the third one
// read from LDS one move before use.  The running threshold is re-read at
// each refill and used at the next.
template <int D, int DIST, bool BANDED>
__device__ float greedy_walk_ring(const float *qs, int m, const float *__restrict__ c, int n,
                                  float *ring, const Band &band, float eps, const uint32_t *tau,
                                  int &steps_out, bool &completed)
{
    constexpr int DP = PadDim<D>::value;
    constexpr int B = WALK_RING_FLOATS / (4 * DP); // points per block
    constexpr int RN = 4 * B;                       // ring points
    static_assert((B & (B - 1)) == 0 && B >= 1, "block of points: a power of two");
    float q0[D], q1[D], q2[D];
    float r0[D], r1[D], r2[D];
    float pf[B][D];
#pragma unroll
    for (int e = 0; e < D; ++e) {
        q0[e] = qs[e];
        q1[e] = qs[min(1, m - 1) * DP + e];
        q2[e] = qs[min(2, m - 1) * DP + e];
    }
    // ring <- points 0 .. RN-1, registers <- points 3B .. 4B-1 (the pending
    // refill of block 0; indices clamped)
#pragma unroll
    for (int t = 0; t < RN; ++t)
#pragma unroll
        for (int e = 0; e < D; ++e)
            ring[t * DP + e] = c[(int64_t)min(t, n - 1) * D + e];
    int pjb = 0; // block whose points 3B .. 4B-1 are pending in pf
#pragma unroll
    for (int t = 0; t < B; ++t)
#pragma unroll
        for (int e = 0; e < D; ++e)
            pf[t][e] = c[(int64_t)min(3 * B + t, n - 1) * D + e];
#pragma unroll
    for (int e = 0; e < D; ++e) {
        r0[e] = ring[0 * DP + e];
        r1[e] = ring[1 * DP + e];
        r2[e] = ring[2 * DP + e];
    }
    float g = point_cost<D>(q0, r0);
    int i = 0, j = 0, steps = 0;
    completed = false;
    if (g > eps) {
        steps_out = 0;
        return g;
    }
    uint32_t tau_next = tau ? load_relaxed_u32(tau) : TSK_INF_BITS;
    // The lanes move in lockstep: a lane whose walk has ended (corner
    // reached: status 1, an infinite move: 2, value above eps: 3) keeps
    // executing the moves without changing its state, and the loop ends
    // when no lane walks.  mv counts the wave's moves (the refill cadence);
    // steps counts the lane's own.
    int status = 0;
    for (int mv = 1;; ++mv) {
        if (status == 0 && !(i < m - 1 || j < n - 1))
            status = 1;
        if (__ballot(status == 0) == 0ull)
            break;
        const bool walk = status == 0;
        const bool di = i + 1 < m, dj = j + 1 < n;
        bool ok_dn = di, ok_dg = di && dj, ok_rt = dj;
        if (BANDED) {
            ok_dn = ok_dn && band_ok(band, i + 1, j);
            ok_dg = ok_dg && band_ok(band, i + 1, j + 1);
            ok_rt = ok_rt && band_ok(band, i, j + 1);
        }
        const float c_dn = ok_dn ? point_cost<D>(q1, r0) : tsk_inf();
        const float c_dg = ok_dg ? point_cost<D>(q1, r1) : tsk_inf();
        const float c_rt = ok_rt ? point_cost<D>(q0, r1) : tsk_inf();
        // first strict minimum in the order (i+1,j), (i+1,j+1), (i,j+1)
        const bool pick_dn = c_dn <= c_dg && c_dn <= c_rt;
        const bool pick_dg = !pick_dn && c_dg <= c_rt;
        const float cst = pick_dn ? c_dn : (pick_dg ? c_dg : c_rt);
        steps += walk ? 1 : 0;
        if (walk && cst == tsk_inf())
            status = 2;
        const bool mov = status == 0;
        if (mov)
            g = DIST == DIST_DK ? fmaxf(g, cst) : cst + g;
        const bool adv_i = mov && (pick_dn || pick_dg);
        const bool adv_j = mov && !pick_dn;
        i += adv_i ? 1 : 0;
        j += adv_j ? 1 : 0;
        if ((mv & (B - 1)) == 0) {
            // Every B moves of the wave: take in the threshold read at the
            // previous refill, write the points loaded then, then issue the
            // next loads (points, threshold), so each wait here covers loads
            // a block of moves old.  A lane's j grows by at most one a move.
            if (tau)
                eps = fminf(eps, bits_f(tau_next));
#pragma unroll
            for (int t = 0; t < B; ++t)
#pragma unroll
                for (int e = 0; e < D; ++e)
                    ring[((pjb + 3 * B + t) & (RN - 1)) * DP + e] = pf[t][e];
            pjb = j & ~(B - 1);
#pragma unroll
            for (int t = 0; t < B; ++t)
#pragma unroll
                for (int e = 0; e < D; ++e)
                    pf[t][e] = c[(int64_t)min(pjb + 3 * B + t, n - 1) * D + e];
            if (tau)
                tau_next = load_relaxed_u32(tau);
        }
        const int ni = min(i + 2, m - 1);
        const int nj = min(j + 2, n - 1) & (RN - 1);
#pragma unroll
        for (int e = 0; e < D; ++e) {
            const float qn = qs[ni * DP + e];
            const float rn = ring[nj * DP + e];
            q0[e] = adv_i ? q1[e] : q0[e];
            q1[e] = adv_i ? q2[e] : q1[e];
            q2[e] = adv_i ? qn : q2[e];
            r0[e] = adv_j ? r1[e] : r0[e];
            r1[e] = adv_j ? r2[e] : r1[e];
            r2[e] = adv_j ? rn : r2[e];
        }
        if (mov && g > eps)
            status = 3;
    }
    steps_out = steps;
    completed = status == 1;
    return status == 2 ? tsk_inf() : g;
}

// The walk with the band test only where a band exists.
template <int D, int DIST>
__device__ float greedy_walk_lds(const float *qs, int m, const float *__restrict__ c, int n,
                                 float *ring, const Band &band, float eps, const uint32_t *tau,
                                 int &steps_out, bool &completed)
{
    if (band.all)
        return greedy_walk_ring<D, DIST, false>(qs, m, c, n, ring, band, eps, tau, steps_out,
                                                completed);
    return greedy_walk_ring<D, DIST, true>(qs, m, c, n, ring, band, eps, tau, steps_out,
                                           completed);
}

// Inserts the lanes' keys that can still matter into a query's top-k slots.
// If more than k lanes of the wave want to insert, only the wave's k
// smallest keys can be among the query's k smallest, so the others skip
// the atomics.
__device__ __forceinline__ void wave_topk_insert(unsigned long long *slots, int k, bool want,
                                                 unsigned long long key, uint32_t *tau)
{
    const unsigned long long mask = __ballot(want);
    if (mask == 0ull)
        return;
    if (__popcll(mask) > k) {
        // every lane walks the same list, so the shuffles are uniform
        int rank = 0;
        unsigned long long rest = mask;
        while (rest) {
            const int l = __ffsll((long long)rest) - 1;
            rest &= rest - 1;
            const unsigned long long other = __shfl(key, l, 64);
            rank += other < key ? 1 : 0;
        }
        want = want && rank < k;
    }
    if (want) {
        topk_insert(slots, k, key);
        tau_from_slots(slots, k, tau);
    }
}

// DTW bound pass for an index of equal-length series: LB_Box of every
// (query, candidate) pair with the query's envelope around each candidate
// point (eq. (1), roles exchanged), fp32, summed over the candidate's
// points in order.  Each candidate point is loaded once (coalesced SoA) and
// scored against the QG queries of the block; the envelopes are wave-uniform
// and arrive through scalar loads.
template <int D, int QG, bool DEBUG>
__global__ __launch_bounds__(256) void k_bound_lb(BoundArgs a, const float *__restrict__ env)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int q0 = blockIdx.y * QG;
    const int nqg = min(QG, a.nq - q0);
    const bool valid = c < a.N;
    const int64_t tile = c >> 6;
    const int lane = (int)(c & 63);
    const int n = a.env_n; // every series has this length
    const float *tb = valid ? a.soa + a.tile_off[tile] + lane : a.soa;
    cfloat *E = (cfloat *)env + (int64_t)q0 * n * 2 * D;
    float acc[QG];
#pragma unroll
    for (int g = 0; g < QG; ++g)
        acc[g] = 0.0f;
    for (int j = 0; j < n; ++j) {
        float x[D];
#pragma unroll
        for (int k = 0; k < D; ++k)
            x[k] = tb[((int64_t)j * D + k) * 64];
#pragma unroll
        for (int g = 0; g < QG; ++g) {
            // groups past the last query reuse query q0's envelope; their sums
            // are never written
            const int gg = g < nqg ? g : 0;
            cfloat *e = E + ((int64_t)gg * n + j) * 2 * D;
            float t = 0.0f;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const float lo = e[k], hi = e[D + k];
                // distance to [lo, hi]: lo - x below, x - hi above, 0 inside;
                // an empty window ([+inf, -inf]) gives +inf by itself
                const float d = fmaxf(fmaxf(lo - x[k], x[k] - hi), 0.0f);
                t = (k == 0) ? d * d : __builtin_fmaf(d, d, t);
            }
            acc[g] = t + acc[g];
        }
    }
    unsigned long long pruned = 0, pairs = 0;
    if (DEBUG) {
        if (valid)
#pragma unroll
            for (int g = 0; g < QG; ++g)
                if (g < nqg)
                    a.dbg_lb[(int64_t)(q0 + g) * a.N + c] = acc[g];
        return;
    }
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
                a.lbv[(int64_t)q * a.N + c] = keep ? acc[g] : tsk_inf();
                pruned += keep ? 0 : 1;
                ++pairs;
            }
        }
    }
    wave_count(a.ctr, C_BOUND_PRUNED, pruned);
    wave_count(a.ctr, C_PAIRS, pairs);
    wave_count(a.ctr, C_BOUND_STEPS, valid ? (unsigned long long)n * nqg : 0ull);
}

// Sum over the 16 lanes of a row through DPP adds: swap neighbours, swap
// pairs within quads, mirror within half-rows, mirror within the row.  At
// every stage the two lanes that meet add the same two values, so all 16
// lanes end with the same sum.
template <int CTRL> __device__ __forceinline__ float dpp_f32(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// Sum over the 8 lanes of a half-row through DPP adds: swap neighbours,
// swap pairs within quads, mirror within the half-row.  At every stage the
// two lanes that meet add the same two values, so all 8 lanes end with the
// same sum.
__device__ __forceinline__ float row8_sum(float v)
{
    v += dpp_f32<0xB1>(v);  // quad_perm [1,0,3,2]
    v += dpp_f32<0x4E>(v);  // quad_perm [2,3,0,1]
    v += dpp_f32<0x141>(v); // row_half_mirror
    return v;
}

// LB_Box with early abandoning per pair (equal lengths).  A block takes one
// query (its envelope staged in LDS) and four runs of LBP_CANDS candidates,
// one per wave; blocks are ordered candidate-major.  Each group of 8 lanes holds one (query, candidate) pair;
// per step lane l of the group adds the box terms of positions
// pos + LBP_P l .. pos + LBP_P l + LBP_P - 1 (contiguous AoS points and
// envelope entries), and the group sums its 8 lanes: 8 LBP_P positions per
// step.  A group stops as soon as its partial sum exceeds the threshold
// (every term is >= 0, so the full sum would too) and takes the next
// candidate of its wave's run.
// The terms are those of k_bound_lb, but the summation order differs from
// the sequential one for which LB_fp32 <= DTW_fp32 holds exactly; any order
// of n <= 4096 non-negative fp32 terms is within (n-1) 2^-24 (relative) of
// the exact sum, so the sum scaled by (1 - 2^-9) (rounding included) is <=
// the sequential sum and thus <= the fp32 DTW.  That scaled value is the
// pair's bound: compared with the threshold and stored in lbv.
constexpr int LBP_CANDS = 256;
constexpr int LBP_P = 8;

template <int D>
__global__ __launch_bounds__(256) void k_bound_lb_pp(BoundArgs a)
{
    extern __shared__ float senv[]; // [n][2][D] of this block's query
    const int lane = threadIdx.x & 63;
    const int grp = lane >> 3, gl = lane & 7;
    const int64_t runs = (a.N + LBP_CANDS - 1) / LBP_CANDS;
    // consecutive blocks take the same candidates for different queries, so
    // the candidates are read from L2 by all but the first
    const int q = (int)(blockIdx.x % a.nq);
    const int64_t run = (int64_t)(blockIdx.x / a.nq) * 4 + (threadIdx.x >> 6);
    const int n = a.env_n;
    const float *E = a.env + (int64_t)q * n * 2 * D;
    for (int i = threadIdx.x; i < n * 2 * D; i += blockDim.x)
        senv[i] = E[i];
    __syncthreads();
    if (run >= runs)
        return;
    const int c_end = (int)min((run + 1) * LBP_CANDS, a.N);
    constexpr float SCALE = 1.0f - 1.0f / 512.0f;
    constexpr int STEP = 8 * LBP_P; // positions per group step
    float tau = bits_f(load_relaxed_u32(a.tau + q));
    int c = (int)(run * LBP_CANDS) + grp; // groups start on consecutive candidates
    if (c >= c_end)
        c = -1;
    int next = (int)(run * LBP_CANDS) + 8;
    // this lane's first point of the current step (equal lengths: the
    // candidate's offset is c n)
    const float *xp = c >= 0 ? a.aos + ((int64_t)c * n + LBP_P * gl) * D : a.aos;
    int pos = 0;
    float part = 0.0f;
    unsigned long long pruned = 0, pairs = 0, terms = 0;
    for (int it = 0; __ballot(c >= 0) != 0ull; ++it) {
        const int p0 = pos + LBP_P * gl;
        float t = 0.0f;
        if (c >= 0 && p0 < n) {
            const float *e = senv + p0 * 2 * D;
            auto term = [&](const float *x, const float *ep) -> float {
                float tu = 0.0f;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const float d = fmaxf(fmaxf(ep[k] - x[k], x[k] - ep[D + k]), 0.0f);
                    tu = (k == 0) ? d * d : __builtin_fmaf(d, d, tu);
                }
                return tu;
            };
            if (p0 + LBP_P <= n) {
                // whole positions: the envelope entries are 16-byte aligned
                // (p0 is a multiple of 4) and read as vectors
                float xv[LBP_P * D], ev[2 * LBP_P * D];
#pragma unroll
                for (int i = 0; i < LBP_P * D; ++i)
                    xv[i] = xp[i];
                const float4 *e4 = reinterpret_cast<const float4 *>(e);
#pragma unroll
                for (int i = 0; i < LBP_P * D / 2; ++i) {
                    const float4 v = e4[i];
                    ev[4 * i] = v.x;
                    ev[4 * i + 1] = v.y;
                    ev[4 * i + 2] = v.z;
                    ev[4 * i + 3] = v.w;
                }
#pragma unroll
                for (int u = 0; u < LBP_P; ++u)
                    t += term(xv + u * D, ev + u * 2 * D);
                terms += LBP_P;
            } else {
                for (int u = 0; u < n - p0; ++u)
                    t += term(xp + u * D, e + u * 2 * D);
                terms += n - p0;
            }
        }
        part += row8_sum(t);
        pos += STEP;
        xp += STEP * D;
        if ((it & 3) == 3)
            tau = bits_f(load_relaxed_u32(a.tau + q));
        bool fin = false;
        if (c >= 0) {
            const float lb = part * SCALE;
            if (lb > tau || pos >= n) {
                fin = true;
                if (gl == 0) {
                    const bool keep = lb <= tau;
                    a.lbv[(int64_t)q * a.N + c] = keep ? lb : tsk_inf();
                    pruned += keep ? 0 : 1;
                    ++pairs;
                }
            }
        }
        // finished groups take the next candidates of the run, in group order
        const unsigned long long need = __ballot(fin && gl == 0);
        if (need) {
            if (fin) {
                const int nc = next + __popcll(need & ((1ull << (grp * 8)) - 1ull));
                c = nc < c_end ? nc : -1;
                pos = 0;
                part = 0.0f;
                xp = c >= 0 ? a.aos + ((int64_t)c * n + LBP_P * gl) * D : a.aos;
            }
            next += __popcll(need);
        }
    }
    wave_count(a.ctr, C_BOUND_PRUNED, pruned);
    wave_count(a.ctr, C_PAIRS, pairs);
    wave_count(a.ctr, C_BOUND_STEPS, terms);
}

// LDS of k_bound_lb_pp, and the largest the launcher uses it with.
inline size_t lb_pp_lds_bytes(int D, int n) { return (size_t)n * 2 * D * sizeof(float); }
constexpr size_t LB_PP_MAX_LDS = 64 * 1024;

// Corner pass: every warping path starts at (0,0) and ends at (m-1,n-1),
// and both cells lie in any band, so for DK max(c(0,0), c(m-1,n-1)) <= the
// squared DK, and for DTW c(0,0) + c(m-1,n-1) <= DTW (two distinct cells of
// every path unless m = n = 1; in fp32 the DP's last value is
// fl(c(m-1,n-1) + p) with p >= c(0,0), so by monotone rounding it is >=
// fl(c(0,0) + c(m-1,n-1))).  One lane per candidate, a group of QG queries
// per block (their end points via scalar loads); lbv gets the bound if it
// does not exceed the running threshold, else +inf.
template <int D, int QG, int DIST>
__global__ __launch_bounds__(256) void k_corner(BoundArgs a)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int q0 = blockIdx.y * QG;
    const int nqg = min(QG, a.nq - q0);
    if (c >= a.N)
        return;
    const int64_t tile = c >> 6;
    const int lane = (int)(c & 63);
    const int n = a.len[c];
    const float *tb = a.soa + a.tile_off[tile] + lane;
    float c0[D], cl[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        c0[k] = tb[(0 * D + k) * 64];
        cl[k] = tb[((int64_t)(n - 1) * D + k) * 64];
    }
    unsigned long long pruned = 0;
    // the group's thresholds first: independent loads, one latency
    float tq[QG];
#pragma unroll
    for (int g = 0; g < QG; ++g)
        tq[g] = g < nqg ? bits_f(load_relaxed_u32(a.tau + q0 + g)) : 0.0f;
#pragma unroll
    for (int g = 0; g < QG; ++g) {
        if (g >= nqg)
            break;
        const int q = q0 + g;
        const int64_t o0 = a.qoff[q], o1 = a.qoff[q + 1];
        cfloat *Q = (cfloat *)a.qv;
        float qa[D], qz[D];
#pragma unroll
        for (int e = 0; e < D; ++e) {
            qa[e] = Q[o0 * D + e];
            qz[e] = Q[(o1 - 1) * D + e];
        }
        const float ca = point_cost<D>(qa, c0), cz = point_cost<D>(qz, cl);
        float lb;
        if (DIST == DIST_DK)
            lb = fmaxf(ca, cz);
        else
            lb = (o1 - o0 > 1 || n > 1) ? ca + cz : ca;
        const bool keep = lb <= tq[g];
        a.lbv[(int64_t)q * a.N + c] = keep ? lb : tsk_inf();
        pruned += keep ? 0 : 1;
    }
    wave_count(a.ctr, C_BOUND_PRUNED, pruned);
    wave_count(a.ctr, C_PAIRS, (unsigned long long)nqg);
}

// DK greedy pass over the compacted survivors (Sec. 4.3, first loop): a wave
// takes 64 survivors of one query (query staged in LDS) and walks Alg. 1 on
// each with early return at the running threshold; completed walks lower the
// threshold through the query's upper-bound slots.
template <int D>
__global__ __launch_bounds__(64) void k_walk_dk(FastArgs a, const float *__restrict__ qv,
                                                 unsigned long long *ubslots, int maxm)
{
    constexpr int DP = PadDim<D>::value;
    extern __shared__ float qs[];
    // LDS: the query (maxm rows), then one candidate ring per lane
    float *ring = qs + maxm * DP + threadIdx.x * WALK_RING_STRIDE;
    unsigned long long steps_cnt = 0, late = 0;
    const int64_t total = (int64_t)a.nq * ((*a.max_cnt + 63) / 64);
    int staged = -1;
    Chunk ch;
    while (next_chunk(a, total, ch, late)) {
        const int q = ch.q, m = ch.m;
        if (q != staged) {
            __syncthreads();
            const float *src = qv + a.qoff[q] * D;
            for (int t = threadIdx.x; t < m * DP; t += 64) {
                const int row = t / DP, e = t % DP;
                qs[t] = e < D ? src[row * D + e] : 0.0f;
            }
            __syncthreads();
            staged = q;
        }
        bool want = false;
        float g = tsk_inf();
        if (ch.act) {
            const int n = a.len[ch.c];
            const Band b = pair_band(a.ba, m, n);
            int steps;
            bool done;
            const float tq = bits_f(load_relaxed_u32(a.tau + q));
            g = greedy_walk_lds<D, DIST_DK>(qs, m, a.aos + a.off[ch.c] * D, n, ring, b, tq,
                                             a.tau + q, steps, done);
            steps_cnt += steps;
            want = done && g != tsk_inf() && g <= bits_f(load_relaxed_u32(a.tau + q));
        }
        wave_topk_insert(ubslots + (int64_t)q * a.k, a.k, want,
                         make_key(g, (uint32_t)(ch.act ? ch.c : 0)), a.tau + q);
    }
    wave_count(a.ctr, C_BOUND_STEPS, steps_cnt);
}

// DTW threshold seed for equal lengths: the diagonal path (i, i) is a
// warping path inside every band, and with monotone rounding its fp32 sum in
// path order is >= the fp32 DTW, so the k-th smallest diagonal sum over the
// first S candidates of each query bounds the k-th smallest DTW from above.
// No sequential walk: one lane per candidate, query rows wave-uniform
// (scalar loads), candidate rows per lane.  Candidates whose length differs
// from the query's are skipped.
template <int D, int DIST>
__global__ __launch_bounds__(64) void k_seed_diag(const float *__restrict__ qv,
                                                  const int64_t *__restrict__ qoff, int nq,
                                                  const float *__restrict__ aos,
                                                  const int64_t *__restrict__ off,
                                                  const int32_t *__restrict__ len, int64_t N,
                                                  const int32_t *__restrict__ order, int S, int k,
                                                  unsigned long long *seedslots, uint32_t *tau,
                                                  unsigned long long *ctr)
{
    const int q = blockIdx.y;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t o0 = qoff[q];
    const int m = (int)(qoff[q + 1] - o0);
    cfloat *Q = (cfloat *)qv + o0 * D;
    int c = 0;
    bool ok = false;
    if (p < S) {
        c = order ? order[(int64_t)q * N + p] : p;
        ok = len[c] == m;
    }
    const float *cp = aos + off[ok ? c : 0] * D;
    float ub = 0.0f;
    for (int i = 0; i < m; ++i) {
        float qq[D], cc[D];
#pragma unroll
        for (int e = 0; e < D; ++e)
            qq[e] = Q[(int64_t)i * D + e];
        load_point<D>(cp + (int64_t)(ok ? i : 0) * D, cc);
        const float cst = point_cost<D>(qq, cc);
        // the diagonal is a warping path: its cost sum bounds DTW, its
        // largest cost bounds the squared DK
        ub = DIST == DIST_DK ? fmaxf(cst, ub) : cst + ub;
    }
    wave_topk_insert(seedslots + (int64_t)q * k, k, ok, make_key(ub, (uint32_t)c), tau + q);
    wave_count(ctr, C_SEED_PAIRS, ok ? 1ull : 0ull);
}

// Threshold seed with the LDS query and the prefetching walk (see k_seed).
template <int D, int DIST>
__global__ __launch_bounds__(64) void k_seed_ring(const float *__restrict__ qv,
                                                  const int64_t *__restrict__ qoff, int nq,
                                                  const float *__restrict__ aos,
                                                  const int64_t *__restrict__ off,
                                                  const int32_t *__restrict__ len, int64_t N,
                                                  const int32_t *__restrict__ order, int P0, int S,
                                                  int maxm, int k, BandArgs ba,
                                                  unsigned long long *seedslots,
                                                  uint32_t *tau, unsigned long long *ctr,
                                                  float *dbg_ub, int32_t *dbg_steps)
{
    // Candidates P0..S-1 of the query's order.  dbg_ub != null: write every
    // walk's value and move count ([q][p]) and insert nothing
    // (tsk_pair_bounds).
    constexpr int DP = PadDim<D>::value;
    extern __shared__ float qs[];
    const int q = blockIdx.y;
    const int m = (int)(qoff[q + 1] - qoff[q]);
    // LDS: the query (maxm rows), then one candidate ring per lane
    float *ring = qs + maxm * DP + threadIdx.x * WALK_RING_STRIDE;
    const float *src = qv + qoff[q] * D;
    for (int t = threadIdx.x; t < m * DP; t += blockDim.x) {
        const int row = t / DP, e = t % DP;
        qs[t] = e < D ? src[row * D + e] : 0.0f;
    }
    __syncthreads();
    const int p = P0 + blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long steps_cnt = 0, pairs = 0;
    bool want = false;
    float g = tsk_inf();
    int c = 0;
    if (p < S) {
        c = order ? order[(int64_t)q * N + p] : p;
        const int n = len[c];
        const Band b = pair_band(ba, m, n);
        int steps;
        bool done;
        // walks of the first 64 candidates are complete; the others return
        // early against the threshold those set
        const bool early = p >= 64 && !dbg_ub;
        const float eps = early ? bits_f(load_relaxed_u32(tau + q)) : tsk_inf();
        g = greedy_walk_lds<D, DIST>(qs, m, aos + off[c] * D, n, ring, b, eps,
                                      early ? tau + q : nullptr, steps, done);
        want = done && g != tsk_inf() && g <= bits_f(load_relaxed_u32(tau + q));
        steps_cnt = steps;
        pairs = 1;
        if (dbg_ub) {
            dbg_ub[(int64_t)q * N + p] = g;
            dbg_steps[(int64_t)q * N + p] = steps;
        }
    }
    if (dbg_ub)
        return;
    wave_topk_insert(seedslots + (int64_t)q * k, k, want, make_key(g, (uint32_t)c), tau + q);
    wave_count(ctr, C_SEED_STEPS, steps_cnt);
    wave_count(ctr, C_SEED_PAIRS, pairs);
}

// ------------------------------------------------------------------ LB_Box, both orientations
// Boxes around the candidate (eq. (1) in the paper's own orientation: the
// candidate enveloped, summed over the query's points), for an index of
// equal-length series and queries of that length: cenv[c][i] is the
// per-dimension [min, max] of the candidate points the band lets align with
// query row i (brute-force window; an empty one gives [+inf, -inf]).
// cenv: [N][n][2][D].
template <int D>
__global__ __launch_bounds__(256) void k_cenv(const float *__restrict__ aos,
                                              const int64_t *__restrict__ off, int64_t N, int n,
                                              BandArgs ba, float *__restrict__ cenv)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * n)
        return;
    const int64_t c = t / n;
    const int i = (int)(t % n);
    const Band b = pair_band(ba, n, n);
    int lo, hi;
    band_cols(b, i, n, lo, hi);
    const float *C = aos + off[c] * D;
    float mn[D], mx[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        mn[k] = tsk_inf();
        mx[k] = -tsk_inf();
    }
    for (int j = lo; j <= hi; ++j) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const float v = C[j * D + k];
            mn[k] = fminf(mn[k], v);
            mx[k] = fmaxf(mx[k], v);
        }
    }
    float *e = cenv + (c * n + i) * 2 * D;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        e[k] = mn[k];
        e[D + k] = mx[k];
    }
}

// The candidate-envelope LB_Box of every survivor of the query-envelope
// bound (queries of another length than the series are left as they are),
// summed in query-row order in fp32 with the point cost's operation order,
// so it stays <= the fp32 DTW like the other orientation.  The survivor's
// bound becomes the larger of the two; the DP stage drops the pair if that
// exceeds the threshold.  One lane per survivor; grid (.., queries).
template <int D>
__global__ __launch_bounds__(256) void k_bound_lb_rev(const float *__restrict__ qv,
                                                      const int64_t *__restrict__ qoff, int n,
                                                      const float *__restrict__ cenv,
                                                      const int32_t *__restrict__ surv,
                                                      const int32_t *__restrict__ surv_cnt,
                                                      int64_t N, float *__restrict__ lbv)
{
    const int q = blockIdx.y;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = (int)(qoff[q + 1] - qoff[q]);
    if (m != n || idx >= surv_cnt[q])
        return;
    const int c = surv[(int64_t)q * N + idx];
    const float *Q = qv + qoff[q] * D;
    const float *E = cenv + (int64_t)c * n * 2 * D;
    float acc = 0.0f;
    for (int i = 0; i < m; ++i) {
        float t = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const float x = Q[i * D + k];
            const float d = fmaxf(fmaxf(E[i * 2 * D + k] - x, x - E[i * 2 * D + D + k]), 0.0f);
            t = (k == 0) ? d * d : __builtin_fmaf(d, d, t);
        }
        acc = t + acc;
    }
    float *p = lbv + (int64_t)q * N + c;
    *p = fmaxf(*p, acc);
}

// LB_Box of the survivors of a first-stage bound (equal lengths, the query
// envelope of k_env), only for the pairs left in surv: a wave per pair, its
// 64 lanes on 64 consecutive candidate points at a time (coalesced loads of
// the candidate), the same per-point terms as k_bound_lb, summed in
// parallel.  The sum of any order of n <= 4096 non-negative fp32 terms is
// within (n-1) 2^-24 (relative) of the exact sum, so the sum scaled by
// (1 - 2^-9) (rounding included) is <= the sequential sum of k_bound_lb,
// hence <= the fp32 DTW; that scaled value is the pair's bound.  A partial
// sum above the query's threshold stops the pair (every term is >= 0) and
// it leaves with +inf; otherwise lbv gets the bound, which the DP stage
// compares with the threshold again.  A block takes tasks of LBS_TASK
// survivors of one query from a work counter (queries interleaved), its
// waves a quarter each; with ENV_LDS the query's envelope is staged in LDS
// once per task instead of being read by every pair.
// DIST_DK: the DK box bound instead, the largest term (Sec. 3's boxes; the
// squared DK is the largest cost on the best path, which aligns each
// candidate point with a query row of its window, at a cost no smaller than
// the term), compared with the squared-DK threshold.  A maximum rounds
// nothing and each term is at most the fp32 cost of any cell of its window
// (same operation order, monotone rounding), so no scaling.
constexpr int LBS_TASK = 64;

template <int D, bool ENV_LDS, int DIST>
__global__ __launch_bounds__(256) void k_bound_lb_surv(BoundArgs a, const int32_t *__restrict__ surv,
                                                       const int32_t *__restrict__ surv_cnt,
                                                       const int32_t *__restrict__ max_cnt,
                                                       unsigned long long *__restrict__ work)
{
    extern __shared__ float senv[]; // [n][2][D] of the task's query (ENV_LDS)
    __shared__ unsigned long long task_s;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int n = a.env_n;
    const int64_t per_q = (*max_cnt + LBS_TASK - 1) / LBS_TASK;
    const int64_t total = (int64_t)a.nq * per_q;
    const float scale = 1.0f - 0x1.0p-9f;
    unsigned long long terms = 0, pruned = 0;
    int staged = -1;
    for (;;) {
        __syncthreads(); // the previous task (and its envelope) is done with
        if (threadIdx.x == 0)
            task_s = atomicAdd(work, 1ull);
        __syncthreads();
        const unsigned long long t = task_s;
        if (t >= (unsigned long long)total)
            break;
        const int q = (int)(t % (unsigned long long)a.nq);
        const int r0 = (int)(t / (unsigned long long)a.nq) * LBS_TASK;
        const int cnt = surv_cnt[q];
        if (r0 >= cnt)
            continue;
        const float *E = a.env + (int64_t)q * n * 2 * D;
        if (ENV_LDS) {
            if (q != staged) {
                for (int i = threadIdx.x; i < n * 2 * D; i += blockDim.x)
                    senv[i] = E[i];
                __syncthreads();
                staged = q;
            }
            E = senv;
        }
        const int per_w = LBS_TASK / 4;
        const int r1 = min(r0 + (wv + 1) * per_w, cnt);
        for (int r = r0 + wv * per_w; r < r1; ++r) {
            const float tau = bits_f(load_relaxed_u32(a.tau + q));
            const int c = __builtin_amdgcn_readfirstlane(surv[(int64_t)q * a.N + r]);
            const float *cp = a.aos + a.off[c] * D;
            float acc = 0.0f;
            bool over = false;
            int j0 = 0;
            for (; j0 < n; j0 += 64) {
                const int j = j0 + lane;
                if (j < n) {
                    float x[D];
                    load_point<D>(cp + (int64_t)j * D, x);
                    const float *e = E + j * 2 * D;
                    float tt = 0.0f;
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        const float d = fmaxf(fmaxf(e[k] - x[k], x[k] - e[D + k]), 0.0f);
                        tt = (k == 0) ? d * d : __builtin_fmaf(d, d, tt);
                    }
                    acc = DIST == DIST_DK ? fmaxf(acc, tt) : acc + tt;
                }
                if (DIST == DIST_DTW && a.lb_prefix > 0 && j0 + 64 == a.lb_prefix && j0 + 64 < n) {
                    // after the prefix: stop once the partial bound exceeds
                    // tau, or give up on a pair whose partial bound, scaled
                    // to all n points, stays below tau (the partial sum of
                    // non-negative terms is itself a lower bound, the one
                    // the pair keeps)
                    const float part = wave_sum(acc) * scale;
                    if (part > tau) {
                        over = true;
                        j0 += 64;
                        break;
                    }
                    if (part * ((float)n / (float)a.lb_prefix) < tau) {
                        j0 += 64;
                        break;
                    }
                }
                if ((j0 & 255) == 192 && j0 + 64 < n) {
                    // every 256 points: stop once the partial bound exceeds tau
                    const float part = DIST == DIST_DK ? wave_max(acc) : wave_sum(acc) * scale;
                    if (part > tau) {
                        over = true;
                        j0 += 64;
                        break;
                    }
                }
            }
            terms += (unsigned long long)min(j0, n);
            const float lb = DIST == DIST_DK ? wave_max(acc) : wave_sum(acc) * scale;
            const bool drop = over || lb > tau;
            pruned += drop ? 1 : 0;
            if (lane == 0)
                a.lbv[(int64_t)q * a.N + c] = drop ? tsk_inf() : lb;
        }
    }
    if (lane != 0) {
        terms = 0;
        pruned = 0;
    }
    wave_count(a.ctr, C_BOUND_STEPS, terms);
    wave_count(a.ctr, C_BOUND_PRUNED, pruned);
}

} // namespace tsk
