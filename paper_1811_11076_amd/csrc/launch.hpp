// Host launchers of the kernels, one translation unit per kernel family so
// the library builds in parallel.
#pragma once

#include "kernels_fast.hpp"

namespace tsk {

// Window sizes of the banded kernel; a call uses the smallest W >= 2w+1.
// Slots below the previous size are inside the band for every pair that
// instantiation serves, so only the slots above it are masked.
constexpr int BAND_WS[] = {16, 32, 56, 64, 104, 128};
constexpr int N_BAND_WS = 6;

void launch_band(int D, int dist, int wsel, const FastArgs &a, int blocks, hipStream_t s);
void launch_tube(int D, const FastArgs &a, int blocks, int maxm, hipStream_t s);
void launch_dp_wave(int D, int dist, int mode, const DpArgs &a, int blocks, hipStream_t s);

} // namespace tsk
