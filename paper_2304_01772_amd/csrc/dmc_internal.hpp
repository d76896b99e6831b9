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

// Energy H per replica (FP64, e_out[R]) and optionally dH/ds (FP32,
// [R][Ly][Lx]) of the spins a.s with the couplings a.Jx, a.Jy and field a.h.
hipError_t launch_dmc_energy(const DmcArgs& a, double* e_out, float* grad, hipStream_t s);
// out[i] = -1 if base[i] - eta g[i] < 0 else +1 (g may be null: base alone).
hipError_t launch_dmc_discretize(int64_t n, const float* base, const float* g, float eta,
                                 float* out, hipStream_t s);

}  // namespace spinmc
