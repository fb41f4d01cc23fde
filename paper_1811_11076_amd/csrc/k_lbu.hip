// LB_Box over length buckets (databases of uneven lengths) and launchers.
#include "launch.hpp"
#include "kernels_lbu.hpp"

namespace tsk {

namespace {
template <int D> void qtable_d(const float *qv, const int64_t *qoff, int nq,
                               const int64_t *tab_off, float *tab, hipStream_t s)
{
    hipLaunchKernelGGL(k_qtable<D>, dim3(nq), dim3(256), 0, s, qv, qoff, tab_off, tab);
}

template <int D>
void bound_lbu_d(const BoundArgs &a, const BucketArgs &bk, const float *tab,
                 const int64_t *tab_off, int qg, bool debug, hipStream_t s)
{
    // the query group trades candidate reuse against scalar-load pressure
#define TSK_LBU(QG)                                                                                \
    do {                                                                                           \
        dim3 grid((unsigned)bk.n_tiles, (unsigned)((a.nq + QG - 1) / QG));                         \
        if (debug)                                                                                 \
            hipLaunchKernelGGL((k_bound_lbu<D, QG, true>), grid, dim3(64), 0, s, a, bk, tab,       \
                               tab_off);                                                           \
        else                                                                                       \
            hipLaunchKernelGGL((k_bound_lbu<D, QG, false>), grid, dim3(64), 0, s, a, bk, tab,      \
                               tab_off);                                                           \
    } while (0)
    // the group's envelopes stay within 32 KB of LDS: up to 8 queries for
    // 8 dimensions, 4 for 12 and 16, 2 for 24 and 32
    constexpr int QG_MAX = D <= 8 ? 8 : (D <= 16 ? 4 : 2);
    if (qg <= 2 || QG_MAX == 2) {
        TSK_LBU(2);
        return;
    }
    if constexpr (QG_MAX >= 4) {
        if (qg <= 4 || QG_MAX == 4) {
            TSK_LBU(4);
            return;
        }
    }
    if constexpr (QG_MAX >= 8)
        TSK_LBU(8);
#undef TSK_LBU
}

template <int D> void pack_bucket_d(const float *aos, const int64_t *off, const BucketArgs &bk,
                                    float *soa, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_bucket<D>, dim3((unsigned)bk.n_tiles), dim3(256), 0, s, aos, off,
                       bk, soa);
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

void launch_qtable(int D, const float *qv, const int64_t *qoff, int nq, const int64_t *tab_off,
                   float *tab, hipStream_t s)
{
#define CALL(d) qtable_d<d>(qv, qoff, nq, tab_off, tab, s)
    TSK_SWITCH_D(D, CALL)
#undef CALL
}

void launch_bound_lbu(int D, const BoundArgs &a, const BucketArgs &bk, const float *tab,
                      const int64_t *tab_off, int qg, bool debug, hipStream_t s)
{
#define CALL(d) bound_lbu_d<d>(a, bk, tab, tab_off, qg, debug, s)
    TSK_SWITCH_D(D, CALL)
#undef CALL
}

void launch_pack_bucket(int D, const float *aos, const int64_t *off, const BucketArgs &bk,
                        float *soa, hipStream_t s)
{
#define CALL(d) pack_bucket_d<d>(aos, off, bk, soa, s)
    TSK_SWITCH_D(D, CALL)
#undef CALL
}

} // namespace tsk
