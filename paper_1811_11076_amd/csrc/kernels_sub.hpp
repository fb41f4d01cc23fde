// Subsequence search (Sec. 4.1-4.2): the DK of a query S against the best
// matching contiguous part T[a..b] of a long series T, a match starting and
// ending anywhere (Alg. 2 and Alg. 3 with SUB).
//
// Work items are (query, series, chunk of start columns).  A chunk's DP is
// the SUB recurrence restricted to matches that start inside the chunk:
// D(0,k) = c(0,k) for k in the chunk (a virtual -inf predecessor), D(0,k) =
// max(c(0,k), D(0,k-1)) after it, D(i,k) = max(c(i,k), min(D(i-1,k),
// D(i,k-1), D(i-1,k-1))) above row 0; it may run past the chunk's end.  The
// start sets of the chunks partition the columns, so the minimum over the
// chunks of their best last-row value is the subsequence DK, and the first
// column reaching it is the first over the chunks.
#pragma once
#include "kernels.hpp"

namespace tsk {

constexpr int SUB_MAX_ROWS = 16;                   // R: query rows per lane
constexpr int SUB_MAX_QLEN = 64 * SUB_MAX_ROWS;     // longest query
constexpr int SUB_WALK_CAP_MUL = 4;                 // greedy walk: at most 4 (m + C) moves

struct SubArgs {
    const float *qv;          // queries of the group, AoS
    const int64_t *qoff;      // [nq + 1] relative offsets
    int nq;
    const float *ser;         // long series, AoS [sum n][D]
    const int64_t *soff;      // [N + 1]
    int64_t N;
    const int64_t *coff;      // [N + 1] prefix of chunks per series
    int64_t chunks;           // chunks per query (coff[N])
    int C;                    // start columns per chunk
    int k;
    uint32_t *pseed;          // [nq][N] greedy bound of the pair (fp32 bits)
    unsigned long long *pbest;// [nq][N] (key bits << 32) | end column
    uint32_t *pcnt;           // [nq][N] chunks of the pair finished
    float *clb;               // [nq * chunks] row-0 minimum of each chunk
    int32_t *cj;              // [nq * chunks] its first column, relative to the chunk
    uint32_t *pclb;           // [nq][N] smallest row-0 cost of the pair (fp32 bits)
    int64_t *live;            // items left for the DP after the row-0 test
    unsigned long long *nlive;// their count
    uint32_t *plive;          // [nq][N] live items per pair
    unsigned long long *seedslots, *resslots; // [nq][k]
    uint32_t *tau;            // [nq] running threshold (fp32 bits)
    unsigned long long *work; // item counter of the DP kernel
    unsigned long long *ctr;  // C_* counters
    // finishing pass
    int64_t *out_ids, *out_end, *out_start;
    float *out_dist;
};

// Item t -> query, series, chunk: queries interleave (t % nq), then the
// chunks of all series in order.
struct SubItem {
    int q;
    int c;
    int64_t a0, a1, n; // start columns [a0, a1) of series c (length n)
};

__device__ __forceinline__ SubItem sub_item(const SubArgs &a, int64_t t)
{
    SubItem it;
    it.q = (int)(t % a.nq);
    const int64_t r = t / a.nq;
    int64_t lo = 0, hi = a.N - 1; // last series with coff[c] <= r
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (a.coff[mid] <= r)
            lo = mid;
        else
            hi = mid - 1;
    }
    it.c = (int)lo;
    it.n = a.soff[lo + 1] - a.soff[lo];
    it.a0 = (r - a.coff[lo]) * (int64_t)a.C;
    it.a1 = min(it.a0 + (int64_t)a.C, it.n);
    return it;
}

// Row-0 minimum of each item: the first column of the chunk minimising
// c(s_0, t_j), and the pair's minimum over its chunks.  Every match
// starting in the chunk costs at least the chunk's minimum.  One thread per
// item; consecutive items are the queries of one chunk, so a wave's lanes
// read the same column, four columns per iteration (loads issued together).
template <int D>
__global__ __launch_bounds__(256) void k_sub_rowmin(SubArgs a)
{
    const int64_t total = (int64_t)a.nq * a.chunks;
    unsigned long long scans = 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const SubItem it = sub_item(a, t);
        const float *T = a.ser + a.soff[it.c] * D;
        float s0[D];
        load_point<D>(a.qv + a.qoff[it.q] * D, s0);
        float g = tsk_inf();
        int64_t j = it.a0, jj = it.a0;
        for (; jj + 4 <= it.a1; jj += 4) {
            float p[4][D];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                load_point<D>(T + (jj + u) * D, p[u]);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float c = point_cost<D>(s0, p[u]);
                if (c < g) {
                    g = c;
                    j = jj + u;
                }
            }
        }
        for (; jj < it.a1; ++jj) {
            float p[D];
            load_point<D>(T + jj * D, p);
            const float c = point_cost<D>(s0, p);
            if (c < g) {
                g = c;
                j = jj;
            }
        }
        scans += (unsigned long long)(it.a1 - it.a0);
        a.clb[t] = g;
        a.cj[t] = (int32_t)(j - it.a0);
        atomicMin(a.pclb + (int64_t)it.q * a.N + it.c, f_bits(g));
    }
    if (scans)
        ctr_add(a.ctr, C_BOUND_STEPS, scans);
}

// Greedy bound (Alg. 2), one thread per item, walking from the item's
// row-0 minimum: moves to the cheapest of (i+1,j), (i+1,j+1), (i,j+1) (the
// first of them on ties; past the last column +inf) until the last row;
// the path's maximum cost bounds the pair's subsequence DK from above.
// Pass 0 walks only from the items holding the pair's smallest row-0 cost,
// which contain Alg. 2's own start (the first column minimising c(s_0, t_j)
// over the whole series); pass 1 from every other item whose row-0 minimum
// is still below the pair's bound (no other walk can lower it).  A walk
// stops once above the pair's bound or after a move budget; only walks that
// reach the last row lower the bound.
template <int D>
__global__ __launch_bounds__(256) void k_sub_walk(SubArgs a, int pass)
{
    const int64_t total = (int64_t)a.nq * a.chunks;
    unsigned long long moves = 0, done = 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const SubItem it = sub_item(a, t);
        const int64_t pair = (int64_t)it.q * a.N + it.c;
        const float g0 = a.clb[t];
        const bool first = f_bits(g0) == a.pclb[pair];
        uint32_t *ps = a.pseed + pair;
        float eps = bits_f(*ps); // a stale (larger) value only costs a walk
        if (pass == 0 ? !first : (first || !(g0 < eps)))
            continue;
        eps = bits_f(load_relaxed_u32(ps));
        const int64_t m = a.qoff[it.q + 1] - a.qoff[it.q];
        const float *S = a.qv + a.qoff[it.q] * D;
        const float *T = a.ser + a.soff[it.c] * D;
        int64_t i = 0, j = it.a0 + a.cj[t], st = 0;
        float g = g0;
        const int64_t cap = SUB_WALK_CAP_MUL * (m + a.C);
        float si[D], sn[D], tj[D], tn[D];
        load_point<D>(S, si);
        load_point<D>(T + j * D, tj);
        while (i != m - 1 && st < cap) {
            load_point<D>(S + (i + 1) * D, sn);
            const bool right = j + 1 < it.n;
            if (right)
                load_point<D>(T + (j + 1) * D, tn);
            const float c_dn = point_cost<D>(sn, tj);
            const float c_dg = right ? point_cost<D>(sn, tn) : tsk_inf();
            const float c_rt = right ? point_cost<D>(si, tn) : tsk_inf();
            float c;
            if (c_dn <= c_dg && c_dn <= c_rt) {
                c = c_dn;
                ++i;
#pragma unroll
                for (int e = 0; e < D; ++e)
                    si[e] = sn[e];
            } else if (c_dg <= c_rt) {
                c = c_dg;
                ++i;
                ++j;
#pragma unroll
                for (int e = 0; e < D; ++e) {
                    si[e] = sn[e];
                    tj[e] = tn[e];
                }
            } else {
                c = c_rt;
                ++j;
#pragma unroll
                for (int e = 0; e < D; ++e)
                    tj[e] = tn[e];
            }
            ++st;
            g = fmaxf(g, c);
            if ((st & 31) == 0)
                eps = bits_f(load_relaxed_u32(ps));
            if (g > eps)
                break;
        }
        moves += (unsigned long long)st;
        if (i == m - 1 && g <= eps) {
            atomicMin(ps, f_bits(g));
            ++done;
        }
    }
    if (moves)
        ctr_add(a.ctr, C_BOUND_STEPS, moves);
    if (done)
        ctr_add(a.ctr, C_SEED_PAIRS, done);
}

// Pair bounds -> the query's seed slots (k smallest, distinct series) and
// threshold; one thread per (query, series).
static __global__ void k_sub_seed_topk(SubArgs a)
{
    const int64_t total = (int64_t)a.nq * a.N;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t v = a.pseed[t];
        if (v == TSK_INF_BITS)
            continue;
        const int q = (int)(t / a.N);
        const uint32_t c = (uint32_t)(t % a.N);
        topk_insert(a.seedslots + (int64_t)q * a.k, a.k, ((unsigned long long)v << 32) | c);
        tau_from_slots(a.seedslots + (int64_t)q * a.k, a.k, a.tau + q);
    }
}

// One chunk's (or the reverse pass's) column sweep on one wave.  Lane l
// holds query rows l R .. l R + R - 1 (qr, +inf cost past the query) and at
// step s works on column j + s - l of the current sweep (a skewed wavefront:
// the row below arrives from lane l-1 of the previous step).  Columns are
// T + k * stride for k in [0, ncols); starts are allowed in [a0, a1).
//
// Sparse search (Alg. 3): a sweep begins at the next start column whose
// row-0 cost is <= tau (found 64 columns at a time).  A cell above tau only
// feeds cells above tau; with sigma(i, k) = k + floor(i / R) a path moves
// sigma by 0, 1 or 2, so once two consecutive steps hold no live cell every
// later cell is dead except those fed by a later start: the sweep ends and
// the search for the next live start resumes after lane 0's column.
// Returns the smallest last-row value <= tau and the first column holding it
// (+inf, -1 if none).  tau comes from thr() (non-increasing), re-read every
// 64 steps, and is capped at the largest finite float: an unreachable cell
// (+inf) is dead even before any threshold exists, so a sweep ends at the
// latest two steps after its last lane has left the series (a bound the loop
// also enforces).
template <int D, int R, typename Thr>
__device__ void sub_sweep(const float (&qr)[R][D], const float (&q0)[D], int m,
                          const float *__restrict__ T, int64_t stride, int64_t ncols, int64_t a0,
                          int64_t a1, Thr thr, float &best, int64_t &bcol,
                          unsigned long long &cells, unsigned long long &valid,
                          unsigned long long &scanned)
{
    const int lane = threadIdx.x & 63;
    const int lm = (m - 1) / R, rm = (m - 1) - lm * R; // the last row's lane and slot
    const int rows_here = m - R * lane;                 // valid rows of this lane (may be <= 0)
    best = tsk_inf();
    bcol = -1;
    constexpr float FMAX = 3.402823466e38f;
    float tau = fminf(thr(), FMAX);
    int64_t pos = a0;
    while (pos < a1) {
        // next start column with a live row-0 cell
        int64_t j = -1;
        while (pos < a1) {
            const int64_t col = pos + lane;
            bool ok = false;
            if (col < a1) {
                float p[D];
                load_point<D>(T + col * stride, p);
                ok = point_cost<D>(q0, p) <= tau;
            }
            const unsigned long long bal = __ballot(ok);
            scanned += 64;
            if (bal) {
                j = pos + (__ffsll((long long)bal) - 1);
                break;
            }
            pos += 64;
        }
        if (j < 0)
            break;
        float Dp[R];
#pragma unroll
        for (int r = 0; r < R; ++r)
            Dp[r] = tsk_inf();
        float my_top = tsk_inf(), recv_prev = tsk_inf();
        bool alive_prev = true;
        // the point of step s + 1 is loaded one step ahead
        auto point_at = [&](int64_t col, float (&out)[D]) {
            const int64_t cc = col < 0 ? 0 : (col >= ncols ? ncols - 1 : col);
            load_point<D>(T + cc * stride, out);
        };
        float pnext[D];
        point_at(j - lane, pnext);
        // at step ncols - j + 62 lane 63 holds the last column
        const int64_t smax = ncols - j + 62;
        for (int64_t s = 0;; ++s) {
            const int64_t col = j + s - lane;
            float pv[D];
#pragma unroll
            for (int e = 0; e < D; ++e)
                pv[e] = pnext[e];
            point_at(col + 1, pnext);
            const float recv = __shfl_up(my_top, 1, 64);
            const bool on = col >= j && col < ncols;
            float down, diag;
            if (lane == 0) {
                // row 0: virtual predecessor -inf in a start column, else +inf
                down = col < a1 ? -tsk_inf() : tsk_inf();
                diag = down;
            } else {
                down = recv;
                diag = recv_prev;
            }
            float vmin = tsk_inf(), vlast = tsk_inf();
            float Dc[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const bool ok = on && r < rows_here;
                const float cst = ok ? point_cost<D>(qr[r], pv) : tsk_inf();
                const float pred = min3f(diag, down, Dp[r]);
                const float v = fmaxf(cst, pred);
                valid += __popcll(__ballot(ok));
                diag = Dp[r];
                down = v;
                Dc[r] = v;
                vmin = fminf(vmin, v);
                if (r == rm)
                    vlast = v;
            }
#pragma unroll
            for (int r = 0; r < R; ++r)
                Dp[r] = Dc[r];
            recv_prev = recv;
            my_top = Dc[R - 1];
            if (lane == lm && on && vlast <= tau && vlast < best) {
                best = vlast;
                bcol = col;
            }
            cells += R;
            const bool alive_now = __ballot(vmin <= tau) != 0ull;
            if ((!alive_now && !alive_prev) || s >= smax) {
                pos = j + s + 1;
                break;
            }
            alive_prev = alive_now;
            if ((s & 63) == 63)
                tau = fminf(thr(), FMAX);
        }
    }
    // the result sits in lane lm
    best = __shfl(best, lm, 64);
    bcol = (int64_t)__shfl((long long)bcol, lm, 64);
}

// Rows of the query held by this lane: row i = l R + r, or reversed
// (row i = S[m-1-i]) for the start pass; past the query zeros (masked).
template <int D, int R>
__device__ __forceinline__ void sub_load_rows(const float *S, int m, bool rev, float (&qr)[R][D])
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = R * lane + r;
        if (i < m) {
            load_point<D>(S + (int64_t)(rev ? m - 1 - i : i) * D, qr[r]);
        } else {
#pragma unroll
            for (int e = 0; e < D; ++e)
                qr[r][e] = 0.0f;
        }
    }
}

// Threshold of a pair: min(query threshold, the pair's greedy bound, the
// pair's best value so far).
__device__ __forceinline__ float sub_thr(const SubArgs &a, int q, int64_t pair)
{
    const float tq = bits_f(load_relaxed_u32(a.tau + q));
    const float ts = bits_f(load_relaxed_u32(a.pseed + pair));
    const float tb = bits_f((uint32_t)(load_relaxed_u64(a.pbest + pair) >> 32));
    return fminf(tq, fminf(ts, tb)); // an empty pbest reads as NaN: ignored
}

// Items whose row-0 minimum is within their pair's threshold (after the
// seed) go to the live list, counted per pair; the rest cannot hold a match
// within the threshold and are dropped.  One thread per item.
static __global__ __launch_bounds__(256) void k_sub_compact(SubArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t total = (int64_t)a.nq * a.chunks;
    unsigned long long dropped = 0;
    for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x; t0 < total;
         t0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = t0 + threadIdx.x;
        bool live = false;
        int64_t pair = 0;
        if (t < total) {
            const SubItem it = sub_item(a, t);
            pair = (int64_t)it.q * a.N + it.c;
            // no sweep has run yet: the threshold is the seed's
            live = a.clb[t] <= fminf(bits_f(a.tau[it.q]), bits_f(a.pseed[pair]));
            dropped += live ? 0 : 1;
        }
        const unsigned long long bal = __ballot(live);
        unsigned long long base = 0;
        if (lane == 0 && bal)
            base = atomicAdd(a.nlive, (unsigned long long)__popcll(bal));
        base = uniform_u64(base);
        if (live) {
            a.live[base + __popcll(bal & ((1ull << lane) - 1ull))] = t;
            atomicAdd(a.plive + pair, 1u);
        }
    }
    if (dropped)
        ctr_add(a.ctr, C_BOUND_PRUNED, dropped);
}

// The DP over the live items: persistent waves take items from a counter
// and sweep them (the sweep re-tests row-0 costs against the current
// threshold).  A sweep's best (value, column) lowers the pair's entry; the
// pair's last live item inserts the pair into the query's result slots
// (each series once, with its final value, if within the threshold) and
// lowers the threshold.  The fences order an item's result before its count
// and the last item's reads after it.
template <int D, int R>
__global__ __launch_bounds__(256) void k_sub_dp(SubArgs a)
{
    const int lane = threadIdx.x & 63;
    const unsigned long long total = *a.nlive;
    unsigned long long cells = 0, valid = 0, scanned = 0, started = 0, hits = 0, none = 0;
    for (;;) {
        unsigned long long w = 0;
        if (lane == 0)
            w = atomicAdd(a.work, 1ull);
        w = uniform_u64(w);
        if (w >= total)
            break;
        const int64_t t = a.live[w];
        const SubItem it = sub_item(a, t);
        const int64_t pair = (int64_t)it.q * a.N + it.c;
        const int m = (int)(a.qoff[it.q + 1] - a.qoff[it.q]);
        auto thr = [&]() -> float {
            const float v = lane == 0 ? sub_thr(a, it.q, pair) : 0.0f;
            return bits_f(__builtin_amdgcn_readfirstlane(f_bits(v)));
        };
        ++started;
        const float *S = a.qv + a.qoff[it.q] * D;
        float qr[R][D], q0[D];
        sub_load_rows<D, R>(S, m, false, qr);
        load_point<D>(S, q0);
        float best;
        int64_t bcol;
        sub_sweep<D, R>(qr, q0, m, a.ser + a.soff[it.c] * D, D, it.n, it.a0, it.a1, thr, best,
                        bcol, cells, valid, scanned);
        if (best != tsk_inf())
            ++hits;
        else
            ++none;
        if (lane == 0) {
            if (best != tsk_inf())
                atomicMin(a.pbest + pair, ((unsigned long long)f_bits(best) << 32) | (uint32_t)bcol);
            __threadfence();
            const uint32_t prev = atomicAdd(a.pcnt + pair, 1u);
            if (prev + 1 == a.plive[pair]) {
                __threadfence();
                const unsigned long long pb = load_relaxed_u64(a.pbest + pair);
                if (pb != TSK_KEY_EMPTY) {
                    const uint32_t key = (uint32_t)(pb >> 32);
                    if (bits_f(key) <= bits_f(load_relaxed_u32(a.tau + it.q))) {
                        unsigned long long *slots = a.resslots + (int64_t)it.q * a.k;
                        topk_insert(slots, a.k, ((unsigned long long)key << 32) | (uint32_t)it.c);
                        tau_from_slots(slots, a.k, a.tau + it.q);
                    }
                }
            }
        }
    }
    if (lane == 0) {
        if (cells)
            ctr_add(a.ctr, C_DP_CELLS, cells * 64ull);
        if (valid)
            ctr_add(a.ctr, C_VALID_CELLS, valid);
        if (scanned)
            ctr_add(a.ctr, C_BOUND_STEPS, scanned);
        if (started)
            ctr_add(a.ctr, C_DP_STARTED, started);
        if (hits)
            ctr_add(a.ctr, C_DP_COMPLETED, hits);
        if (none)
            ctr_add(a.ctr, C_DP_ABANDONED, none);
    }
}

// Output rows: ids, distances (correctly rounded sqrt of the squared key),
// end columns; (-1, +inf, -1) for empty ranks.  One thread per (query, rank).
static __global__ void k_sub_finalize(SubArgs a)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)a.nq * a.k)
        return;
    const int q = (int)(t / a.k);
    const unsigned long long key = a.resslots[t];
    int64_t id = -1, end = -1;
    float dist = tsk_inf();
    if (key != TSK_KEY_EMPTY) {
        id = (int64_t)(uint32_t)(key & 0xFFFFFFFFull);
        dist = sqrt_rn_f32(bits_f((uint32_t)(key >> 32)));
        end = (int64_t)(uint32_t)(a.pbest[(int64_t)q * a.N + id] & 0xFFFFFFFFull);
    }
    a.out_ids[t] = id;
    a.out_dist[t] = dist;
    a.out_end[t] = end;
}

// Match starts: for a reported (key, end e) the latest a with
// DK(S, T[a..e]) = key.  DK is unchanged when both series are reversed, so
// this is the first column k' of the sweep of reversed S over T[e], T[e-1],
// ..., starting only at k' = 0, whose last-row value equals key: a = e - k'.
// One wave per (query, rank), threshold fixed at key.
template <int D, int R>
__global__ __launch_bounds__(256) void k_sub_start(SubArgs a)
{
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t total = (int64_t)a.nq * a.k;
    unsigned long long cells = 0, valid = 0, scanned = 0;
    for (int64_t t = gw; t < total; t += (int64_t)gridDim.x * (blockDim.x >> 6)) {
        const unsigned long long key = a.resslots[t];
        if (key == TSK_KEY_EMPTY) {
            if ((threadIdx.x & 63) == 0)
                a.out_start[t] = -1;
            continue;
        }
        const int q = (int)(t / a.k);
        const int64_t c = (int64_t)(uint32_t)(key & 0xFFFFFFFFull);
        const float kv = bits_f((uint32_t)(key >> 32));
        const int64_t e = (int64_t)(uint32_t)(a.pbest[(int64_t)q * a.N + c] & 0xFFFFFFFFull);
        const int m = (int)(a.qoff[q + 1] - a.qoff[q]);
        const float *S = a.qv + a.qoff[q] * D;
        float qr[R][D], q0[D];
        sub_load_rows<D, R>(S, m, true, qr);
        load_point<D>(S + (int64_t)(m - 1) * D, q0);
        float best;
        int64_t bcol;
        sub_sweep<D, R>(qr, q0, m, a.ser + (a.soff[c] + e) * D, -(int64_t)D, e + 1, 0, 1,
                        [&]() { return kv; }, best, bcol, cells, valid, scanned);
        if ((threadIdx.x & 63) == 0)
            a.out_start[t] = (bcol >= 0 && best == kv) ? e - bcol : -1;
    }
    if ((threadIdx.x & 63) == 0 && cells)
        ctr_add(a.ctr, C_DP_CELLS, cells * 64ull);
}

} // namespace tsk
