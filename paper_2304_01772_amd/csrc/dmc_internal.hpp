// Internal declarations of the differentiable Monte Carlo kernels (relaxed
// Ising chain with per-bond couplings).  Not part of the C ABI.
#pragma once
#include "spinmc_internal.hpp"

namespace spinmc {

struct DmcArgs {
    float* s;              // spins [R][Ly][Lx]
    const float* Jx;       // couplings of the bonds (y,x)-(y,x+1) [R][Ly][Lx]
    const float* Jy;       // couplings of the bonds (y,x)-(y+1,x) [R][Ly][Lx]
    int32_t R, Lx, Ly;
    float beta, alpha, h;
    uint32_t key0, key1, rid0;
};

// n_sweeps sweeps from sweep counter t0; save receives the pre-pass spins of
// the updated colour, [2 n_sweeps][R][Ly Lx/2].
hipError_t launch_dmc_forward(const DmcArgs& a, uint64_t t0, int n_sweeps, float* save,
                              hipStream_t s);
// Reverse replay: a.s holds the final spins on entry and the initial spins on
// exit; gs holds dL/ds_final on entry and dL/ds_initial on exit; gJx, gJy
// accumulate; work is [2][R][Ly Lx/2].
hipError_t launch_dmc_backward(const DmcArgs& a, uint64_t t0, int n_sweeps, const float* save,
                               float* gs, float* gJx, float* gJy, float* work, hipStream_t s);

}  // namespace spinmc
