// Host launchers of the kernels, one translation unit per kernel family so
// the library builds in parallel.
#pragma once

#include "kernels_bound.hpp"
#include "kernels_lbu.hpp"

namespace tsk {

// Window sizes of the banded kernel; a call uses the smallest W >= 2w+1.
// Slots below the previous size are inside the band for every pair that
// instantiation serves, so only the slots above it are masked.
constexpr int BAND_WS[] = {16, 32, 52, 56, 64, 104, 128};
constexpr int N_BAND_WS = 7;
// the 52-slot kernel for bands of 49..52 slots (w = 24, 25): only slots 49
// and up are masked at run time
constexpr int BAND_W52_TIGHT = 7;

struct SeedRingArgs {
    const float *qv;
    const int64_t *qoff;
    int nq;
    int maxm;
    const float *aos;
    const int64_t *off;
    const int32_t *len;
    int64_t N;
    const int32_t *order;
    int P0, S, k;
    BandArgs ba;
    unsigned long long *seedslots;
    uint32_t *tau;
    unsigned long long *ctr;
    float *dbg_ub;      // debug: per-pair walk value, or null
    int32_t *dbg_steps; // debug: per-pair move count
};

// LDS of the 64-lane greedy-walk kernels: the query, then a candidate ring
// per lane, WALK_RING_STRIDE floats apart.
inline size_t walk_lds_bytes(int D, int maxm)
{
    const int DP = pad_dim(D);
    return ((size_t)maxm * DP + 64 * WALK_RING_STRIDE) * sizeof(float);
}

void launch_bound_lb(int D, const BoundArgs &a, bool debug, hipStream_t s);
// candidate envelopes (k_cenv) then the candidate-envelope LB_Box of the
// survivors (k_bound_lb_rev); equal-length index of length n
void launch_bound_lb_rev(int D, const float *aos, const int64_t *off, int64_t N, int n,
                         BandArgs ba, float *cenv, const float *qv, const int64_t *qoff, int nq,
                         const int32_t *surv, const int32_t *surv_cnt, float *lbv, hipStream_t s);
void launch_bound_lb_pp(int D, const BoundArgs &a, hipStream_t s);
void launch_seed_ring(int D, int dist, const SeedRingArgs &r, hipStream_t s);
void launch_corner(int D, int dist, const BoundArgs &a, hipStream_t s);
// LB_Box (DTW) or the DK box bound (DK) of the compacted survivors (query
// envelope in a.env), lbv updated
void launch_bound_lb_surv(int D, int dist, const BoundArgs &a, const int32_t *surv,
                          const int32_t *surv_cnt, const int32_t *max_cnt,
                          unsigned long long *work, int blocks, hipStream_t s);
void launch_seed_diag(int D, int dist, const SeedRingArgs &r, hipStream_t s);
void launch_walk_dk(int D, const FastArgs &a, const float *qv, unsigned long long *ubslots,
                    int blocks, int maxm, hipStream_t s);
void launch_band(int D, int dist, int wsel, const FastArgs &a, int blocks, hipStream_t s);
// equal: every query of the chunk and every series have one length (the
// tube then computes more columns per iteration)
void launch_tube(int D, const FastArgs &a, int rows, bool equal, int blocks, int maxm, hipStream_t s);
void launch_dp_wave(int D, int dist, int mode, const DpArgs &a, int blocks, hipStream_t s);
void launch_qtable(int D, const float *qv, const int64_t *qoff, int nq, const int64_t *tab_off,
                   float *tab, hipStream_t s);
void launch_bound_lbu(int D, const BoundArgs &a, const BucketArgs &bk, const float *tab,
                      const int64_t *tab_off, int qg, bool debug, hipStream_t s);
void launch_pack_bucket(int D, const float *aos, const int64_t *off, const BucketArgs &bk,
                        float *soa, hipStream_t s);

} // namespace tsk
