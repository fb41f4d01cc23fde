// Bound-pass kernels (k_bound_dk, k_bound_lb, k_seed_ring) and launchers.
#include "launch.hpp"

namespace tsk {

namespace {
template <int D> void bound_lb_pp_d(const BoundArgs &a, hipStream_t s)
{
    const int64_t runs = (a.N + LBP_CANDS - 1) / LBP_CANDS;
    const int64_t blocks = (int64_t)a.nq * ((runs + 3) / 4);
    hipLaunchKernelGGL((k_bound_lb_pp<D>), dim3((unsigned)blocks), dim3(256),
                       lb_pp_lds_bytes(D, a.env_n), s, a);
}

template <int D> void bound_lb_d(const BoundArgs &a, bool debug, hipStream_t s)
{
    // 8 queries share each candidate load (VALU-bound while the database
    // sits in the MALL); 16 when asked for (a.qgroup), for databases that
    // stream from HBM
    if (!debug && a.qgroup == 16) {
        constexpr int QG = 16;
        dim3 grid((unsigned)((a.N + 255) / 256), (unsigned)((a.nq + QG - 1) / QG));
        hipLaunchKernelGGL((k_bound_lb<D, QG, false>), grid, dim3(256), 0, s, a, a.env);
        return;
    }
    constexpr int QG = 8;
    dim3 grid((unsigned)((a.N + 255) / 256), (unsigned)((a.nq + QG - 1) / QG));
    if (debug)
        hipLaunchKernelGGL((k_bound_lb<D, QG, true>), grid, dim3(256), 0, s, a, a.env);
    else
        hipLaunchKernelGGL((k_bound_lb<D, QG, false>), grid, dim3(256), 0, s, a, a.env);
}

template <int D>
void seed_ring_d(int dist, const SeedRingArgs &r, hipStream_t s)
{
    dim3 grid((r.S - r.P0 + 63) / 64, r.nq);
    const size_t lds = walk_lds_bytes(D, r.maxm);
    if (dist == DIST_DK)
        hipLaunchKernelGGL((k_seed_ring<D, DIST_DK>), grid, dim3(64), lds, s, r.qv, r.qoff, r.nq,
                           r.aos, r.off, r.len, r.N, r.order, r.P0, r.S, r.maxm, r.k, r.ba, r.seedslots,
                           r.tau, r.ctr, r.dbg_ub, r.dbg_steps);
    else
        hipLaunchKernelGGL((k_seed_ring<D, DIST_DTW>), grid, dim3(64), lds, s, r.qv, r.qoff, r.nq,
                           r.aos, r.off, r.len, r.N, r.order, r.P0, r.S, r.maxm, r.k, r.ba, r.seedslots,
                           r.tau, r.ctr, r.dbg_ub, r.dbg_steps);
}
template <int D> void seed_diag_d(int dist, const SeedRingArgs &r, hipStream_t s)
{
    dim3 grid((r.S + 63) / 64, r.nq);
    if (dist == DIST_DK)
        hipLaunchKernelGGL((k_seed_diag<D, DIST_DK>), grid, dim3(64), 0, s, r.qv, r.qoff, r.nq,
                           r.aos, r.off, r.len, r.N, r.order, r.S, r.k, r.seedslots, r.tau, r.ctr);
    else
        hipLaunchKernelGGL((k_seed_diag<D, DIST_DTW>), grid, dim3(64), 0, s, r.qv, r.qoff, r.nq,
                           r.aos, r.off, r.len, r.N, r.order, r.S, r.k, r.seedslots, r.tau, r.ctr);
}

template <int D> void corner_d(int dist, const BoundArgs &a, hipStream_t s)
{
    // 16 queries per block: each candidate's end points are read once per 16
    constexpr int QG = 16;
    dim3 grid((unsigned)((a.N + 255) / 256), (unsigned)((a.nq + QG - 1) / QG));
    if (dist == DIST_DK)
        hipLaunchKernelGGL((k_corner<D, QG, DIST_DK>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_corner<D, QG, DIST_DTW>), grid, dim3(256), 0, s, a);
}

template <int D, int DIST>
void bound_lb_surv_dd(const BoundArgs &a, const int32_t *surv, const int32_t *surv_cnt,
                      const int32_t *max_cnt, unsigned long long *work, int blocks, hipStream_t s)
{
    const size_t lds = (size_t)a.env_n * 2 * D * sizeof(float);
    if (lds <= 64 * 1024)
        hipLaunchKernelGGL((k_bound_lb_surv<D, true, DIST>), dim3(blocks), dim3(256), lds, s, a,
                           surv, surv_cnt, max_cnt, work);
    else
        hipLaunchKernelGGL((k_bound_lb_surv<D, false, DIST>), dim3(blocks), dim3(256), 0, s, a,
                           surv, surv_cnt, max_cnt, work);
}

template <int D>
void bound_lb_surv_d(int dist, const BoundArgs &a, const int32_t *surv, const int32_t *surv_cnt,
                     const int32_t *max_cnt, unsigned long long *work, int blocks, hipStream_t s)
{
    if (dist == DIST_DK)
        bound_lb_surv_dd<D, DIST_DK>(a, surv, surv_cnt, max_cnt, work, blocks, s);
    else
        bound_lb_surv_dd<D, DIST_DTW>(a, surv, surv_cnt, max_cnt, work, blocks, s);
}

template <int D>
void walk_d(const FastArgs &a, const float *qv, unsigned long long *ubslots, int blocks, int maxm,
            hipStream_t s)
{
    const size_t lds = walk_lds_bytes(D, maxm);
    hipLaunchKernelGGL((k_walk_dk<D>), dim3(blocks), dim3(64), lds, s, a, qv, ubslots, maxm);
}
} // namespace

#define TSK_SWITCH_D(D_, CALL)                                                                     \
    switch (D_) {                                                                                  \
    case 1: CALL(1); break;                                                                        \
    case 2: CALL(2); break;                                                                        \
    case 3: CALL(3); break;                                                                        \
    case 4: CALL(4); break;                                                                        \
    case 5: CALL(5); break;                                                                        \
    case 6: CALL(6); break;                                                                        \
    case 7: CALL(7); break;                                                                        \
    case 8: CALL(8); break;                                                                        \
    case 12: CALL(12); break;                                                                      \
    case 16: CALL(16); break;                                                                      \
    case 24: CALL(24); break;                                                                      \
    case 32: CALL(32); break;                                                                      \
    default: break;                                                                                \
    }

void launch_bound_lb(int D, const BoundArgs &a, bool debug, hipStream_t s)
{
#define CALL(d) bound_lb_d<d>(a, debug, s)
    TSK_SWITCH_D(D, CALL)
#undef CALL
}

namespace {
template <int D>
void bound_lb_rev_d(const float *aos, const int64_t *off, int64_t N, int n, BandArgs ba,
                    float *cenv, const float *qv, const int64_t *qoff, int nq,
                    const int32_t *surv, const int32_t *surv_cnt, float *lbv, hipStream_t s)
{
    const int64_t cells = N * n;
    hipLaunchKernelGGL(k_cenv<D>, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, s, aos, off,
                       N, n, ba, cenv);
    hipLaunchKernelGGL(k_bound_lb_rev<D>, dim3((unsigned)((N + 255) / 256), nq), dim3(256), 0, s,
                       qv, qoff, n, cenv, surv, surv_cnt, N, lbv);
}
} // namespace

void launch_bound_lb_rev(int D, const float *aos, const int64_t *off, int64_t N, int n,
                         BandArgs ba, float *cenv, const float *qv, const int64_t *qoff, int nq,
                         const int32_t *surv, const int32_t *surv_cnt, float *lbv, hipStream_t s)
{
#define CALL(d) bound_lb_rev_d<d>(aos, off, N, n, ba, cenv, qv, qoff, nq, surv, surv_cnt, lbv, s)
    TSK_SWITCH_D(D, CALL)
#undef CALL
}

void launch_bound_lb_pp(int D, const BoundArgs &a, hipStream_t s)
{
#define CALL(d) bound_lb_pp_d<d>(a, s)
    TSK_SWITCH_D(D, CALL)
#undef CALL
}

void launch_seed_diag(int D, int dist, const SeedRingArgs &r, hipStream_t s)
{
#define CALL(d) seed_diag_d<d>(dist, r, s)
    TSK_SWITCH_D(D, CALL)
#undef CALL
}

void launch_corner(int D, int dist, const BoundArgs &a, hipStream_t s)
{
#define CALL(d) corner_d<d>(dist, a, s)
    TSK_SWITCH_D(D, CALL)
#undef CALL
}

void launch_bound_lb_surv(int D, int dist, const BoundArgs &a, const int32_t *surv,
                          const int32_t *surv_cnt, const int32_t *max_cnt,
                          unsigned long long *work, int blocks, hipStream_t s)
{
#define CALL(d) bound_lb_surv_d<d>(dist, a, surv, surv_cnt, max_cnt, work, blocks, s)
    TSK_SWITCH_D(D, CALL)
#undef CALL
}

void launch_walk_dk(int D, const FastArgs &a, const float *qv, unsigned long long *ubslots,
                    int blocks, int maxm, hipStream_t s)
{
#define CALL(d) walk_d<d>(a, qv, ubslots, blocks, maxm, s)
    TSK_SWITCH_D(D, CALL)
#undef CALL
}

void launch_seed_ring(int D, int dist, const SeedRingArgs &r, hipStream_t s)
{
#define CALL(d) seed_ring_d<d>(dist, r, s)
    TSK_SWITCH_D(D, CALL)
#undef CALL
}

} // namespace tsk
