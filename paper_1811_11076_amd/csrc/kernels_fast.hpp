// Lane-per-pair DP kernels for the common shapes (gfx950, wave64).
//
// A wave takes 64 surviving candidates of ONE query and runs their DPs in
// lockstep, one candidate per lane, column by column over the candidate.
// Pairs a kernel cannot represent exactly are appended to a fallback list
// and finished by the general wave-per-pair DP (k_dp_wave).
#pragma once

#include "kernels.hpp"

namespace tsk {

// Rows of padding (+inf points) around each staged query.
constexpr int QPAD = 128;

// Read-only memory seen through the constant address space: uniform loads
// from it become scalar (SMEM) loads into SGPRs.  Only used for buffers that
// earlier kernels wrote (the scalar cache is invalidated at kernel start).
typedef __attribute__((address_space(4))) const float cfloat;

template <int D> struct PadDim {
    static constexpr int value = pad_dim(D);
};

struct FastArgs {
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
    unsigned long long *work; // [0] task counter, [1] fallback count
    int2 *fb;                 // fallback (query, candidate) list
    const float *qpad;        // [nq][qrows][DP]: query rows at QPAD.., +inf around
    int qrows;
    int task;                 // survivors per wave task (k_dp_tube)
    int32_t *qcur;            // per-query survivor cursors (k_dp_band), zeroed per call
    float *range_out;         // range query: [nq][N] keys of hits, else null (top-k)
    int qmajor;               // task order of the lane-per-pair kernels: query-major
    int dk_virtual;           // k_dp_band on unbanded DK: a band of (W-1)/2 whose edge
                              // cells must stay above tau (else the general DP)
    unsigned long long *ctr;
};

// Staged query: rows -QPAD .. m-1+QPAD of every query, points padded to DP
// floats, rows outside the query set to +inf (a point at infinity has an
// infinite cost to every finite point, so such cells never hold a finite
// value).
template <int D>
__global__ void k_qpad(const float *__restrict__ qv, const int64_t *__restrict__ qoff, int nq,
                       int qrows, float *__restrict__ qpad)
{
    constexpr int DP = PadDim<D>::value;
    const int q = blockIdx.y;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq || r >= qrows)
        return;
    const int m = (int)(qoff[q + 1] - qoff[q]);
    const int row = r - QPAD;
    float *dst = qpad + ((int64_t)q * qrows + r) * DP;
#pragma unroll
    for (int k = 0; k < DP; ++k) {
        float v = tsk_inf();
        if (row >= 0 && row < m && k < D)
            v = qv[(qoff[q] + row) * D + k];
        dst[k] = (k < D || row < 0 || row >= m) ? v : 0.0f;
    }
}

__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

// One fast-kernel task: the 64-candidate chunk r of query q.  Fills c (-1 if
// none), act (lane runs the fast DP), and handles late pruning / fallback.
struct Chunk {
    int q, m, c;
    bool act;
};

__device__ __forceinline__ bool next_chunk(const FastArgs &a, int64_t total, Chunk &ch,
                                           unsigned long long &late)
{
    for (;;) {
        unsigned long long t = 0;
        if (threadIdx.x == 0)
            t = atomicAdd(a.work, 1ull);
        t = uniform_u64(t);
        // unsigned: a counter value can never pass as a negative index
        if (t >= (unsigned long long)total)
            return false;
        const int q = uniform_i((int)(t % (unsigned long long)a.nq));
        const int r = (int)(t / (unsigned long long)a.nq);
        const int cnt = a.surv_cnt[q];
        const int base = r * 64;
        if (base >= cnt)
            continue;
        ch.q = q;
        ch.m = uniform_i((int)(a.qoff[q + 1] - a.qoff[q]));
        ch.c = -1;
        ch.act = false;
        const int idx = base + (int)threadIdx.x;
        if (idx < cnt) {
            const int c = a.surv[(int64_t)q * a.N + idx];
            if (a.lbv[(int64_t)q * a.N + (a.lb_inv ? a.lb_inv[c] : c)] > bits_f(load_relaxed_u32(a.tau + q)))
                ++late;
            else {
                ch.c = c;
                ch.act = true;
            }
        }
        return true;
    }
}

// Dense variant for the lockstep banded kernel: a task names a query; the
// wave then claims that query's survivors from its cursor until all 64 lanes
// hold a pair still within the threshold (or the list ends), so survivors
// that the tightening threshold has already pruned leave no idle lanes.
// slot: 64 ints of the block's LDS (the block is one wave).
__device__ __forceinline__ bool next_dense_chunk(const FastArgs &a, int64_t total, Chunk &ch,
                                                 unsigned long long &late, int32_t *slot)
{
    const int lane = (int)threadIdx.x;
    for (;;) {
        unsigned long long t = 0;
        if (lane == 0)
            t = atomicAdd(a.work, 1ull);
        t = uniform_u64(t);
        // unsigned: a counter value can never pass as a negative index
        if (t >= (unsigned long long)total)
            return false;
        // query-major tasks (the waves in flight share few queries, whose
        // rows stay in the scalar cache) or query-interleaved
        const unsigned long long per_q = (unsigned long long)(total / a.nq);
        const int q = uniform_i(a.qmajor ? (int)(t / per_q) : (int)(t % (unsigned long long)a.nq));
        const int cnt = uniform_i(a.surv_cnt[q]);
        if (uniform_i(__hip_atomic_load(a.qcur + q, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT)) >= cnt)
            continue; // this query's list is used up
        const float tau = bits_f(load_relaxed_u32(a.tau + q));
        int filled = 0;
        __syncthreads(); // the previous task's reads of slot are done
        for (;;) {
            const int need = 64 - filled;
            int base = 0;
            if (lane == 0)
                base = atomicAdd(a.qcur + q, need);
            base = uniform_i(base);
            if (base >= cnt)
                break;
            bool keep = false;
            int c = -1;
            const int idx = base + lane;
            if (lane < need && idx < cnt) {
                c = a.surv[(int64_t)q * a.N + idx];
                keep = !(a.lbv[(int64_t)q * a.N + (a.lb_inv ? a.lb_inv[c] : c)] > tau);
                late += keep ? 0 : 1;
            }
            const unsigned long long mk = __ballot(keep);
            if (keep)
                slot[filled + __popcll(mk & ((1ull << lane) - 1ull))] = c;
            filled += __popcll(mk);
            if (filled == 64 || base + need >= cnt)
                break;
        }
        if (filled == 0)
            continue;
        __syncthreads(); // slot entries written by other lanes are visible
        ch.q = q;
        ch.m = uniform_i((int)(a.qoff[q + 1] - a.qoff[q]));
        ch.act = lane < filled;
        ch.c = ch.act ? slot[lane] : -1;
        return true;
    }
}

__device__ __forceinline__ void push_fallback(const FastArgs &a, int q, int c)
{
    const unsigned long long slot = atomicAdd(a.work + 1, 1ull);
    a.fb[slot] = make_int2(q, c);
}

__device__ __forceinline__ void finish_lane(const FastArgs &a, int q, int c, float res,
                                            unsigned long long &completed)
{
    if (a.range_out) {
        // range query: the threshold is the fixed radius; record the hit
        if (res != tsk_inf() && res <= bits_f(load_relaxed_u32(a.tau + q))) {
            ++completed;
            a.range_out[(int64_t)q * a.N + c] = res;
        }
        return;
    }
    if (res != tsk_inf() && res <= bits_f(load_relaxed_u32(a.tau + q))) {
        ++completed;
        topk_insert(a.resslots + (int64_t)q * a.k, a.k, make_key(res, (uint32_t)c));
        tau_from_slots(a.resslots + (int64_t)q * a.k, a.k, a.tau + q);
    }
}

// ------------------------------------------------------------------ banded, equal lengths
// Pairs with n == m and band half-width w (2w+1 <= W; no band = w of m-1).
// Each lane keeps the band part of the current column in W registers:
// slot k of column j holds D(j - w + k, j).  Because the band moves down by
// one row per column, the lower-left predecessor of slot k is slot k of the
// previous column and the left predecessor is slot k+1, so the column is
// updated in place in ascending k (Sec. 2.1 recurrence; Sec. 2.2 band).
// Slots beyond 2w and rows outside the query read +inf query points, so
// they never hold a finite value.  The query rows are the same for the
// whole wave (scalar loads); the candidate point is per lane.  Every path
// visits every column, so a column whose values all exceed tau ends the
// lane's pair (checked every 8 columns).
constexpr int BAND_NC = 2; // columns per iteration of k_dp_band

// Cells inside the band (slot < wact) and the matrix (row 0 .. m-1) among
// the G steps from k0 of an NC-column iteration at column j: column j + r
// takes slots k0 - r .. k0 + G - 1 - r, slot s being row j + r - w + s.
template <int G, int NC>
__device__ __forceinline__ int band_group_cells(int k0, int j, int w, int wact, int m)
{
    int n = 0;
#pragma unroll
    for (int r = 0; r < NC; ++r) {
        const int c = j + r;
        const int lo = max(max(k0 - r, 0), w - c);
        const int hi = min(min(k0 + G - 1 - r, wact - 1), m - 1 - c + w);
        n += max(0, hi - lo + 1);
    }
    return n;
}

template <int D, int DIST, int W, int KMASK>
__global__ __launch_bounds__(64) void k_dp_band(FastArgs a, const float *__restrict__ qpad)
{
    // W slots per column; slots below KMASK are always inside the band for
    // the pairs this instantiation serves (2w+1 >= KMASK), slots from KMASK
    // up are masked against 2w+1 at run time.
    constexpr int DP = PadDim<D>::value;
    constexpr int G = W % 8 == 0 ? 8 : 4;
    static_assert(W % G == 0, "W must be a multiple of 4");
    unsigned long long started = 0, completed = 0, abandoned = 0, late = 0, fallback = 0;
    unsigned long long cells = 0, valid = 0;
    const int64_t total = (int64_t)a.nq * ((*a.max_cnt + 63) / 64);
    __shared__ int32_t slot[64];
    Chunk ch;
    while (next_dense_chunk(a, total, ch, late, slot)) {
        const int q = ch.q, m = ch.m;
        int w = band_w(a.ba.mode, a.ba.r, a.ba.frac, m, m);
        if (w < 0 || w > m - 1)
            w = m - 1;
        // unbanded DK in a virtual band: every path with max <= tau runs
        // through live cells only; one that left the band would cross an
        // edge cell (|i - j| = w) reached in-band, whose in-band value is
        // then <= tau.  So while both edge slots stay above tau (checked
        // against a tau that only falls) the in-band DP is exact.
        const bool vband = DIST == DIST_DK && a.dk_virtual && (W - 1) / 2 < m - 1;
        if (DIST == DIST_DK && a.dk_virtual)
            w = min((W - 1) / 2, m - 1);
        w = uniform_i(w);
        bool act = ch.act;
        if (act && (a.len[ch.c] != m || 2 * w + 1 > W || 2 * w + 1 < KMASK)) {
            push_fallback(a, q, ch.c);
            ++fallback;
            act = false;
        }
        const unsigned long long act_mask = __ballot(act);
        if (act_mask == 0ull)
            continue;
        started += act ? 1 : 0;
        const int wact = 2 * w + 1;
        const float *cp = a.aos + a.off[act ? ch.c : 0] * D;
        const int nl = act ? m : a.len[0]; // idle lanes read candidate 0 in bounds
        // slot k of column j reads query row j - w + k, staged at qpad row
        // QPAD + j - w + k (QPAD >= W keeps every slot inside the buffer)
        cfloat *qbase = (cfloat *)qpad + ((int64_t)q * a.qrows + QPAD - w) * DP;
        float Dv[W];
#pragma unroll
        for (int k = 0; k < W; ++k)
            Dv[k] = (k == w) ? 0.0f : tsk_inf(); // D(-1,-1) = 0 sits in slot w of column -1
        bool alive = act;
        float tau = bits_f(load_relaxed_u32(a.tau + q));
        int j = 0;
        float cv[D];
        load_point<D>(cp, cv);
        bool stop = false;
        {
            // NC columns per iteration.  At step k, slot k - r of column j + r
            // (r = 0 .. NC-1) reads query row j - w + k, so each row is loaded
            // once for NC cells and the NC dependency chains interleave.  Cell
            // (slot s, column j+r) takes its lower-left predecessor from slot s
            // of column j+r-1 (the previous step's value) and its left one from
            // slot s+1 of that column (this step's value); column j's come from
            // the registers of column j-1.  Only column j+NC-1 is written back
            // (slot s once no later step reads it).  The last NC-1 steps finish
            // the top slots of columns j+1.. with rows past j - w + W - 1
            // (inside the +inf padding).
            constexpr int NC = BAND_NC;
            constexpr int TOP = 2 * ((W - 1) / 2);
            constexpr int KS = W + NC - 1;               // steps
            constexpr int KSG = (KS + G - 1) / G * G;    // rounded to whole groups
            float cc[NC][D];
#pragma unroll
            for (int r = 0; r < NC; ++r)
                load_point<D>(cp + (int64_t)min(r, nl - 1) * D, cc[r]);
            auto combine = [](float cst, float pred) -> float {
                return DIST == DIST_DK ? fmaxf(cst, pred) : cst + pred;
            };
            // Dead groups of G steps: a group's cells take their
            // predecessors from inside the group, from Dv[gG .. gG+G]
            // (column j-1, not yet overwritten when the group starts) and
            // from prv[] (the step before the group).  If all of those
            // exceed tau on every live lane, so does every cell of the group
            // (a cell is its cost, >= 0, combined with its smallest
            // predecessor), and no path through them ends within tau: the
            // group is skipped, its cells +inf.  Group g writes back slots
            // gG-1 .. gG+G-2 of column j+NC-1; with gw and gl the first and
            // last groups that wrote a value within tau (on some live lane),
            // the next sweep's live predecessors in Dv lie in groups
            // gw-1 .. gl (gw-1 only if slot gwG-1 or gwG is live), so it
            // runs groups gs .. gl, then on while the group just done
            // leaves a live value in prv[].  Its first query rows are
            // loaded at the end of the sweep before.
            constexpr int NG = KSG / G;
            static_assert(NG <= 32, "group mask");
            // groups computed in the sweep before: only their slots can hold
            // finite values, so only they need clearing when skipped
            uint32_t comp_prev = ~0u;
            int gs = max(0, w / G - 1);      // Dv holds one finite slot, w
            int g_last = min(NG - 1, w / G);
            float qc[G][D], qn[G][D];
#pragma unroll
            for (int u = 0; u < G; ++u)
#pragma unroll
                for (int e = 0; e < D; ++e)
                    qc[u][e] = qbase[(int64_t)(gs * G + u) * DP + e];
            for (; j + NC - 1 < m; j += NC) {
                float nx[NC][D];
#pragma unroll
                for (int r = 0; r < NC; ++r)
                    load_point<D>(cp + (int64_t)min(j + NC + r, nl - 1) * D, nx[r]);
                cfloat *qrow = qbase + (int64_t)j * DP;
                int wl = wact;
                asm volatile("" : "+s"(wl));
                float prv[NC], cur[NC], e0[NC], eT[NC];
#pragma unroll
                for (int r = 0; r < NC; ++r) {
                    prv[r] = tsk_inf();
                    e0[r] = tsk_inf();
                    eT[r] = tsk_inf();
                }
                int hs = 0;    // in-band, in-matrix cells of the computed groups
                int ncomp = 0; // computed groups (G steps of NC cells each)
                int gw = NG, gl = -1, glo = NG;
                bool run = gs < NG;
                uint32_t comp_now = 0;
                float lmin_all = tsk_inf(); // the lane's smallest written value
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    if (g < gs || !run) {
                        if ((comp_prev >> g) & 1u) {
#pragma unroll
                            for (int u = 0; u < G; ++u) {
                                const int sl = g * G + u - (NC - 1);
                                if (g * G + u < KS && sl >= 0 && sl < W)
                                    Dv[sl] = tsk_inf();
                            }
                        }
                        continue;
                    }
                    comp_now |= 1u << g;
                    if (g + 1 < NG) {
#pragma unroll
                        for (int u = 0; u < G; ++u)
#pragma unroll
                            for (int e = 0; e < D; ++e)
                                qn[u][e] = qrow[((g + 1) * G + u) * DP + e];
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    ++ncomp;
                    hs += band_group_cells<G, NC>(g * G, j, w, wact, m);
                    float wmin = tsk_inf(); // values this group writes back
                    float lmin = tsk_inf(); // of them, slots gG-1 and gG
#pragma unroll
                    for (int u = 0; u < G; ++u) {
                        const int k = g * G + u;
                        if (k < KS) {
#pragma unroll
                            for (int r = 0; r < NC; ++r) {
                                const int sl = k - r;
                                if (sl >= 0 && sl < W) {
                                    float cst = point_cost<D>(qc[u], cc[r]);
                                    if (sl >= KMASK)
                                        cst = sl < wl ? cst : tsk_inf();
                                    float diag, left;
                                    if (r == 0) {
                                        diag = Dv[sl];
                                        left = (sl + 1 < W) ? Dv[sl + 1] : tsk_inf();
                                    } else {
                                        diag = prv[r - 1];
                                        left = cur[r - 1];
                                    }
                                    const float v = combine(cst, min3f(prv[r], diag, left));
                                    cur[r] = v;
                                    if (sl == 0)
                                        e0[r] = v;
                                    if (sl == TOP)
                                        eT[r] = v;
                                    if (r == NC - 1) {
                                        Dv[sl] = v;
                                        wmin = fminf(wmin, v);
                                        if (sl <= g * G)
                                            lmin = fminf(lmin, v);
                                    }
                                } else {
                                    cur[r] = tsk_inf();
                                }
                            }
#pragma unroll
                            for (int r = 0; r < NC; ++r)
                                prv[r] = cur[r];
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    lmin_all = fminf(lmin_all, wmin);
                    if (__ballot(alive && wmin <= tau) != 0ull) {
                        if (gw == NG) {
                            gw = g;
                            // group g-1 reads slot gG-1 and gG
                            glo = __ballot(alive && lmin <= tau) != 0ull ? g - 1 : g;
                        }
                        gl = g;
                    }
                    if (g >= g_last) {
                        float pmin = prv[0];
#pragma unroll
                        for (int r = 1; r < NC; ++r)
                            pmin = fminf(pmin, prv[r]);
                        run = __ballot(alive && pmin <= tau) != 0ull;
                    }
#pragma unroll
                    for (int u = 0; u < G; ++u)
#pragma unroll
                        for (int e = 0; e < D; ++e)
                            qc[u][e] = qn[u][e];
                }
                // the next sweep's range, and its first query rows
                comp_prev = comp_now;
                gs = gw < NG ? max(0, glo) : NG;
                g_last = gl;
                {
                    cfloat *qnext = qrow + (int64_t)NC * DP + (int64_t)min(gs, NG - 1) * G * DP;
#pragma unroll
                    for (int u = 0; u < G; ++u)
#pragma unroll
                        for (int e = 0; e < D; ++e)
                            qc[u][e] = qnext[u * DP + e];
                }
#pragma unroll
                for (int r = 0; r < NC; ++r)
#pragma unroll
                    for (int e = 0; e < D; ++e)
                        cc[r][e] = nx[r][e];
                valid += (unsigned long long)hs * __popcll(__ballot(alive));
                cells += (unsigned long long)ncomp * G * NC;
                if (vband) {
                    bool edge = false;
#pragma unroll
                    for (int r = 0; r < NC; ++r)
                        edge = edge || e0[r] <= tau || eT[r] <= tau;
                    if (alive && edge) {
                        push_fallback(a, q, ch.c);
                        ++fallback;
                        --started;
                        alive = false;
                        act = false;
                    }
                }
                if ((j + NC) / 8 != j / 8) { // about every 8 columns
                    // the column's smallest value: every slot was written
                    // by a computed group or holds +inf
                    const float cm = lmin_all;
                    tau = bits_f(load_relaxed_u32(a.tau + q));
                    alive = alive && cm <= tau;
                    if (__ballot(alive) == 0ull) {
                        j += NC;
                        stop = true;
                        break;
                    }
                }
            }
#pragma unroll
            for (int e = 0; e < D; ++e)
                cv[e] = cc[0][e]; // the next column's point, for the single-column tail
        }
        for (; !stop && j < m; ++j) {
            float cn[D];
            load_point<D>(cp + (int64_t)min(j + 1, nl - 1) * D, cn);
            cfloat *qrow = qbase + (int64_t)j * DP;
            // an opaque copy: the per-slot masks are rebuilt in SALU each
            // column instead of being hoisted (W live masks would spill)
            int wl = wact;
            asm volatile("" : "+s"(wl));
            float down = tsk_inf();
            // Query rows go through SGPRs in groups of G slots: the loads of
            // group g+1 are issued before group g is computed; the scheduling
            // barriers keep a whole column of rows from being hoisted.
            float qc[G][D], qn[G][D];
#pragma unroll
            for (int u = 0; u < G; ++u)
#pragma unroll
                for (int e = 0; e < D; ++e)
                    qc[u][e] = qrow[u * DP + e];
#pragma unroll
            for (int g = 0; g < W / G; ++g) {
                if (g + 1 < W / G) {
#pragma unroll
                    for (int u = 0; u < G; ++u)
#pragma unroll
                        for (int e = 0; e < D; ++e)
                            qn[u][e] = qrow[((g + 1) * G + u) * DP + e];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < G; ++u) {
                    const int k = g * G + u;
                    float cst = point_cost<D>(qc[u], cv);
                    if (k >= KMASK)
                        cst = k < wl ? cst : tsk_inf();
                    const float left = (k + 1 < W) ? Dv[k + 1] : tsk_inf();
                    const float pred = min3f(down, Dv[k], left);
                    const float v = DIST == DIST_DK ? fmaxf(cst, pred) : cst + pred;
                    Dv[k] = v;
                    down = v;
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < G; ++u)
#pragma unroll
                    for (int e = 0; e < D; ++e)
                        qc[u][e] = qn[u][e];
            }
#pragma unroll
            for (int e = 0; e < D; ++e)
                cv[e] = cn[e];
            const int h = min(j + w, m - 1) - max(j - w, 0) + 1;
            valid += (unsigned long long)h * __popcll(__ballot(alive));
            cells += W;
            if (vband) {
                constexpr int TOP = 2 * ((W - 1) / 2);
                if (alive && (Dv[0] <= tau || Dv[TOP] <= tau)) {
                    push_fallback(a, q, ch.c);
                    ++fallback;
                    --started;
                    alive = false;
                    act = false;
                }
            }
            if ((j & 7) == 7) {
                float cm = Dv[0];
#pragma unroll
                for (int k = 1; k < W; ++k)
                    cm = fminf(cm, Dv[k]);
                tau = bits_f(load_relaxed_u32(a.tau + q));
                alive = alive && cm <= tau;
                if (__ballot(alive) == 0ull) {
                    ++j;
                    break;
                }
            }
        }
        float res = tsk_inf();
        if (j >= m) {
#pragma unroll
            for (int k = 0; k < W; ++k)
                res = (k == w) ? Dv[k] : res;
        }
        if (act) {
            if (!alive)
                res = tsk_inf();
            if (res == tsk_inf())
                ++abandoned;
            finish_lane(a, q, ch.c, res, completed);
        }
    }
    wave_count(a.ctr, C_DP_STARTED, started);
    wave_count(a.ctr, C_DP_COMPLETED, completed);
    wave_count(a.ctr, C_DP_ABANDONED, abandoned);
    wave_count(a.ctr, C_BOUND_PRUNED, late);
    wave_count(a.ctr, C_FALLBACK, fallback);
    if (threadIdx.x == 0) {
        ctr_add(a.ctr, C_DP_CELLS, cells * 64ull);
        ctr_add(a.ctr, C_VALID_CELLS, valid);
    }
}

// ------------------------------------------------------------------ sparse DK tube
// Unbanded DK with the sparse-DK semantics of Alg. 3 (Sec. 4.2): a cell above
// tau is dead, and a pair with no live cell left in a column is > tau.  Dead
// cells keep their (exact) values: max(cost, min(preds)) of cells whose
// predecessors are all above tau is above tau too, so they never lower a
// live cell, and liveness is tested against tau (which only falls) instead
// of killing them.
// Each lane keeps a window of W consecutive rows [lo, lo+W) and computes
// NT columns over it per iteration, so each query row read from LDS serves
// NT cells.  Cells below lo are dead (nothing below a dead prefix can come
// back: every predecessor is lower or to the left), so after each iteration
// lo moves up past up to 2 NT - 1 (at most W - 1) leading dead slots of the
// last column.
// Cells above the window are reached only through a top slot (of the same
// column, or of an earlier column of the same window), so as long as all
// the columns' top slots stay dead the window holds every live cell and the
// values in it are exact; a live top slot sends the pair to the general DP,
// and only then is a window without live cells no proof that the pair is
// above tau.  In the iteration holding a pair's last column the end cell is
// exact when its row is in the window (every row up to it is held); one
// above the window is reached through a top slot, so there a live top slot
// sends the pair to the general DP too.
// A wave takes a chunk of up to a.task survivors of one query (query rows in
// LDS).  Lanes advance independently, each on its own pair and column; a
// lane whose pair ends takes the chunk's next survivor, so the wave stays
// busy until the chunk drains.
// LDS slot of the 16-byte quarter i of the staged query rows: with 8-float
// rows a row's two halves swap when bit 2 of the row is set, so the lanes'
// rows (each at its own offset) spread over all eight 16-byte bank groups
// of a 128-byte line instead of four.
// Columns per iteration of k_dp_tube: each LDS row read serves NT cells;
// more columns keep the window in place longer, so more pairs outgrow it
// (equal lengths, d = 6, W = 16: 2, 4, 6, 8 columns took 3.1, 2.55, 2.5,
// 2.3 ms per launch but handed 0, 24, 4 600 and 254 000 pairs per call to
// the general DP, whose time made 4 the fastest).  Pairs of different
// lengths follow a slanted path that rises up to m/n rows per column, so
// they take 2.
constexpr int TUBE_NC_EQUAL = 4;
constexpr int TUBE_NC_UNEVEN = 2;

template <int DP> __device__ __forceinline__ int tube_slot(int i)
{
    if (DP != 8)
        return i;
    return i ^ ((i >> 3) & 1);
}

template <int D, int W, int NT>
__global__ __launch_bounds__(64) void k_dp_tube(FastArgs a)
{
    constexpr int DP = PadDim<D>::value;
    // most slots the window moves per iteration
    constexpr int SH = 2 * NT - 1 < W - 1 ? 2 * NT - 1 : W - 1;
    static_assert(NT >= 2, "tube columns per iteration");
    extern __shared__ float qs[];
    unsigned long long started = 0, completed = 0, abandoned = 0, late = 0, fallback = 0;
    unsigned long long cells = 0, valid = 0;
    const int T = a.task;
    const int64_t total = (int64_t)a.nq * ((*a.max_cnt + T - 1) / T);
    const int lane = threadIdx.x;
    int staged = -1;
    for (;;) {
        unsigned long long t = 0;
        if (lane == 0)
            t = atomicAdd(a.work, 1ull);
        t = uniform_u64(t);
        if (t >= (unsigned long long)total)
            break;
        const unsigned long long per_q = (unsigned long long)(total / a.nq);
        const int q = uniform_i(a.qmajor ? (int)(t / per_q) : (int)(t % (unsigned long long)a.nq));
        const int base = (int)(a.qmajor ? t % per_q : t / (unsigned long long)a.nq) * T;
        const int cnt = a.surv_cnt[q];
        if (base >= cnt)
            continue;
        const int end = uniform_i(min(base + T, cnt));
        const int m = uniform_i((int)(a.qoff[q + 1] - a.qoff[q]));
        if (q != staged) {
            // query rows 0 .. m-1+W (those past m-1 are +inf)
            __syncthreads();
            const float4 *src =
                reinterpret_cast<const float4 *>(a.qpad + ((int64_t)q * a.qrows + QPAD) * DP);
            float4 *dst = reinterpret_cast<float4 *>(qs);
            const int n4 = (m + W) * DP / 4;
            for (int i = lane; i < n4; i += 64)
                dst[tube_slot<DP>(i)] = src[i];
            __syncthreads();
            staged = q;
        }
        float tau = bits_f(load_relaxed_u32(a.tau + q));
        int next = base;
        bool running = false;
        int c = 0, n = 1, j = 0, lo = 0;
        const float *cp = a.aos;
        float Dv[W];
#pragma unroll
        for (int k = 0; k < W; ++k)
            Dv[k] = tsk_inf();
        for (int it = 0;; ++it) {
            // idle lanes take the chunk's next survivors
            const unsigned long long need = __ballot(!running);
            if (need != 0ull && next < end) {
                const int rank = __popcll(need & ((1ull << lane) - 1ull));
                const int idx = next + rank;
                if (!running && idx < end) {
                    const int cc = a.surv[(int64_t)q * a.N + idx];
                    if (a.lbv[(int64_t)q * a.N + (a.lb_inv ? a.lb_inv[cc] : cc)] > tau) {
                        ++late;
                    } else {
                        c = cc;
                        n = a.len[c];
                        cp = a.aos + a.off[c] * D;
                        j = 0;
                        lo = 0;
#pragma unroll
                        for (int k = 0; k < W; ++k)
                            Dv[k] = tsk_inf();
                        running = true;
                        ++started;
                    }
                }
                next = uniform_i(min(end, next + (int)__popcll(need)));
            }
            if (__ballot(running) == 0ull) {
                if (next >= end)
                    break;
                continue;
            }
            if ((it & 7) == 0)
                tau = bits_f(load_relaxed_u32(a.tau + q));
            // NT columns per iteration over the same window rows: each row
            // read from LDS serves a cell of each of columns j .. j+NT-1
            float cv[NT][D];
#pragma unroll
            for (int r = 0; r < NT; ++r)
                load_point<D>(cp + (int64_t)min(j + r, n - 1) * D, cv[r]);
            float down[NT], dgp[NT];
#pragma unroll
            for (int r = 0; r < NT; ++r) {
                down[r] = tsk_inf();
                dgp[r] = tsk_inf();
            }
            float diag0 = (j == 0) ? 0.0f : tsk_inf(); // D(-1,-1) = 0 feeds (0,0)
            float vminl = tsk_inf();
            float V[NT - 1][W]; // columns j .. j+NT-2 (Dv becomes column j+NT-1)
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const int row = lo + k;
                float qq[D];
                {
                    // whole rows with 16-byte LDS reads (rows are DP floats,
                    // 16-byte aligned); scattered rows conflict less that way
                    // than dword pairs that straddle rows
                    const float4 *r4 = reinterpret_cast<const float4 *>(qs);
                    float rv[DP];
#pragma unroll
                    for (int h = 0; h < DP / 4; ++h) {
                        const float4 v = r4[tube_slot<DP>(row * (DP / 4) + h)];
                        rv[4 * h] = v.x;
                        rv[4 * h + 1] = v.y;
                        rv[4 * h + 2] = v.z;
                        rv[4 * h + 3] = v.w;
                    }
#pragma unroll
                    for (int e = 0; e < D; ++e)
                        qq[e] = rv[e];
                }
                float prev = 0.0f; // column r-1's value in this row
#pragma unroll
                for (int r = 0; r < NT; ++r) {
                    const float cst = point_cost<D>(qq, cv[r]);
                    float v;
                    if (r == 0) {
                        const float old = Dv[k];
                        v = fmaxf(cst, min3f(down[0], old, diag0));
                        diag0 = old;
                    } else {
                        // left is (row, column r-1), lower-left (row-1, r-1)
                        v = fmaxf(cst, min3f(down[r], prev, dgp[r]));
                        dgp[r] = prev;
                    }
                    down[r] = v;
                    if (r < NT - 1) {
                        V[r < NT - 1 ? r : 0][k] = v;
                    } else {
                        Dv[k] = v;
                        vminl = fminf(vminl, v);
                    }
                    prev = v;
                }
            }
            cells += (unsigned long long)NT * W;
            // cells of the window inside the matrix (rows past m-1 are
            // padding), in the columns that belong to the pair
            valid += running ? (unsigned long long)(min(NT, n - j) * max(0, min(W, m - lo))) : 0ull;
            if (running) {
                const int slot = m - 1 - lo;
                const int rend = n - 1 - j; // the pair's last column, if < NT
                bool top = false;           // a live top slot up to rend
#pragma unroll
                for (int r = 0; r < NT; ++r) {
                    const float t = r < NT - 1 ? V[r < NT - 1 ? r : 0][W - 1] : Dv[W - 1];
                    top = top || (r <= rend && t <= tau);
                }
                if (rend < NT) {
                    if (slot >= W && top) {
                        // the end row lies above the window while a top slot
                        // is live: the end cell may be reached up the last
                        // columns through rows the window does not hold
                        push_fallback(a, q, c);
                        ++fallback;
                        --started; // the general DP counts it
                    } else {
                        float res = tsk_inf();
#pragma unroll
                        for (int r = 0; r < NT; ++r)
#pragma unroll
                            for (int k = 0; k < W; ++k) {
                                const float t = r < NT - 1 ? V[r < NT - 1 ? r : 0][k] : Dv[k];
                                res = (r == rend && k == slot) ? t : res;
                            }
                        res = res <= tau ? res : tsk_inf();
                        if (res == tsk_inf())
                            ++abandoned;
                        finish_lane(a, q, c, res, completed);
                    }
                    running = false;
                } else if (top) {
                    push_fallback(a, q, c);
                    ++fallback;
                    --started; // the general DP counts it
                    running = false;
                } else if (!(vminl <= tau)) {
                    ++abandoned;
                    running = false;
                }
            }
            // drop up to SH leading dead slots of the last column (idle
            // lanes keep lo), in steps of 1, 2, 4, ...
            int sh = SH;
#pragma unroll
            for (int k = SH - 1; k >= 0; --k)
                sh = Dv[k] <= tau ? k : sh;
            sh = running ? sh : 0;
#pragma unroll
            for (int step = 1; step <= SH; step *= 2) {
                const bool mv = (sh & step) != 0;
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    const float d = (k + step < W) ? Dv[k + step] : tsk_inf();
                    Dv[k] = mv ? d : Dv[k];
                }
            }
            lo += sh;
            j += running ? NT : 0;
        }
    }
    wave_count(a.ctr, C_DP_STARTED, started);
    wave_count(a.ctr, C_DP_COMPLETED, completed);
    wave_count(a.ctr, C_DP_ABANDONED, abandoned);
    wave_count(a.ctr, C_BOUND_PRUNED, late);
    wave_count(a.ctr, C_FALLBACK, fallback);
    wave_count(a.ctr, C_VALID_CELLS, valid);
    if (threadIdx.x == 0)
        ctr_add(a.ctr, C_DP_CELLS, cells * 64ull);
}

} // namespace tsk
