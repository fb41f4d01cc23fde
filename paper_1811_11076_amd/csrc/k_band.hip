// Banded lane-per-pair DP kernels (k_dp_band) and their launcher.
#include "launch.hpp"

namespace tsk {

namespace {
template <int D, int DIST> void band_d(int wsel, const FastArgs &a, int blocks, hipStream_t s)
{
    dim3 grid(blocks), block(64);
    switch (wsel) {
    case 0: hipLaunchKernelGGL((k_dp_band<D, DIST, 16, 1>), grid, block, 0, s, a, a.qpad); break;
    case 1: hipLaunchKernelGGL((k_dp_band<D, DIST, 32, 17>), grid, block, 0, s, a, a.qpad); break;
    case 2: hipLaunchKernelGGL((k_dp_band<D, DIST, 52, 33>), grid, block, 0, s, a, a.qpad); break;
    case 3: hipLaunchKernelGGL((k_dp_band<D, DIST, 56, 53>), grid, block, 0, s, a, a.qpad); break;
    case 4: hipLaunchKernelGGL((k_dp_band<D, DIST, 64, 57>), grid, block, 0, s, a, a.qpad); break;
    case 5: hipLaunchKernelGGL((k_dp_band<D, DIST, 104, 65>), grid, block, 0, s, a, a.qpad); break;
    case 6: hipLaunchKernelGGL((k_dp_band<D, DIST, 128, 105>), grid, block, 0, s, a, a.qpad); break;
    case BAND_W52_TIGHT:
        hipLaunchKernelGGL((k_dp_band<D, DIST, 52, 49>), grid, block, 0, s, a, a.qpad);
        break;
    default: break;
    }
}

template <int D> void band_dist(int dist, int wsel, const FastArgs &a, int blocks, hipStream_t s)
{
    if (dist == DIST_DK)
        band_d<D, DIST_DK>(wsel, a, blocks, s);
    else
        band_d<D, DIST_DTW>(wsel, a, blocks, s);
}
} // namespace

void launch_band(int D, int dist, int wsel, const FastArgs &a, int blocks, hipStream_t s)
{
    switch (D) {
    case 1: band_dist<1>(dist, wsel, a, blocks, s); break;
    case 2: band_dist<2>(dist, wsel, a, blocks, s); break;
    case 3: band_dist<3>(dist, wsel, a, blocks, s); break;
    case 4: band_dist<4>(dist, wsel, a, blocks, s); break;
    case 5: band_dist<5>(dist, wsel, a, blocks, s); break;
    case 6: band_dist<6>(dist, wsel, a, blocks, s); break;
    case 7: band_dist<7>(dist, wsel, a, blocks, s); break;
    case 8: band_dist<8>(dist, wsel, a, blocks, s); break;
    default: break;
    }
}

} // namespace tsk
