// General wave-per-pair DP kernel (k_dp_wave) and its launcher.
#include "launch.hpp"

namespace tsk {

namespace {
template <int D, int R> void wave_r(int dist, int mode, const DpArgs &a, int blocks, hipStream_t s)
{
    dim3 grid(blocks), block(256);
#define TSK_DPW(DI, MO) hipLaunchKernelGGL((k_dp_wave<D, DI, MO, R>), grid, block, 0, s, a)
    if (dist == DIST_DK) {
        if (mode == DPW_ALLPAIRS) TSK_DPW(DIST_DK, DPW_ALLPAIRS);
        else if (mode == DPW_FALLBACK) TSK_DPW(DIST_DK, DPW_FALLBACK);
        else TSK_DPW(DIST_DK, DPW_SURV);
    } else {
        if (mode == DPW_ALLPAIRS) TSK_DPW(DIST_DTW, DPW_ALLPAIRS);
        else if (mode == DPW_FALLBACK) TSK_DPW(DIST_DTW, DPW_FALLBACK);
        else TSK_DPW(DIST_DTW, DPW_SURV);
    }
#undef TSK_DPW
}

template <int D> void wave_d(int dist, int mode, const DpArgs &a, int blocks, hipStream_t s)
{
    // above 8 dimensions one row per lane (a lane holds its rows' points in
    // registers: 4 rows of 32 floats would crowd out the rest)
    if constexpr (D > 8)
        wave_r<D, 1>(dist, mode, a, blocks, s);
    else if (a.rows_per_lane == 1)
        wave_r<D, 1>(dist, mode, a, blocks, s);
    else if (a.rows_per_lane == 2)
        wave_r<D, 2>(dist, mode, a, blocks, s);
    else
        wave_r<D, 4>(dist, mode, a, blocks, s);
}
} // namespace

void launch_dp_wave(int D, int dist, int mode, const DpArgs &a, int blocks, hipStream_t s)
{
    switch (D) {
    case 1: wave_d<1>(dist, mode, a, blocks, s); break;
    case 2: wave_d<2>(dist, mode, a, blocks, s); break;
    case 3: wave_d<3>(dist, mode, a, blocks, s); break;
    case 4: wave_d<4>(dist, mode, a, blocks, s); break;
    case 5: wave_d<5>(dist, mode, a, blocks, s); break;
    case 6: wave_d<6>(dist, mode, a, blocks, s); break;
    case 7: wave_d<7>(dist, mode, a, blocks, s); break;
    case 8: wave_d<8>(dist, mode, a, blocks, s); break;
    case 12: wave_d<12>(dist, mode, a, blocks, s); break;
    case 16: wave_d<16>(dist, mode, a, blocks, s); break;
    case 24: wave_d<24>(dist, mode, a, blocks, s); break;
    case 32: wave_d<32>(dist, mode, a, blocks, s); break;
    default: break;
    }
}

} // namespace tsk
