// Sparse-DK lane-per-pair kernel (k_dp_tube) and its launcher.
#include "launch.hpp"

namespace tsk {

namespace {
template <int D, int NT> void tube_dn(const FastArgs &a, int rows, int blocks, int maxm, hipStream_t s)
{
    constexpr int DP = PadDim<D>::value;
    const size_t lds = (size_t)(maxm + 32) * DP * sizeof(float);
    if (rows == 8)
        hipLaunchKernelGGL((k_dp_tube<D, 8, NT>), dim3(blocks), dim3(64), lds, s, a);
    else if (rows == 16)
        hipLaunchKernelGGL((k_dp_tube<D, 16, NT>), dim3(blocks), dim3(64), lds, s, a);
    else
        hipLaunchKernelGGL((k_dp_tube<D, 32, NT>), dim3(blocks), dim3(64), lds, s, a);
}

template <int D> void tube_d(const FastArgs &a, int rows, bool equal, int blocks, int maxm, hipStream_t s)
{
    if (equal)
        tube_dn<D, TUBE_NC_EQUAL>(a, rows, blocks, maxm, s);
    else
        tube_dn<D, TUBE_NC_UNEVEN>(a, rows, blocks, maxm, s);
}
} // namespace

void launch_tube(int D, const FastArgs &a, int rows, bool equal, int blocks, int maxm, hipStream_t s)
{
    switch (D) {
    case 1: tube_d<1>(a, rows, equal, blocks, maxm, s); break;
    case 2: tube_d<2>(a, rows, equal, blocks, maxm, s); break;
    case 3: tube_d<3>(a, rows, equal, blocks, maxm, s); break;
    case 4: tube_d<4>(a, rows, equal, blocks, maxm, s); break;
    case 5: tube_d<5>(a, rows, equal, blocks, maxm, s); break;
    case 6: tube_d<6>(a, rows, equal, blocks, maxm, s); break;
    case 7: tube_d<7>(a, rows, equal, blocks, maxm, s); break;
    case 8: tube_d<8>(a, rows, equal, blocks, maxm, s); break;
    default: break;
    }
}

} // namespace tsk
