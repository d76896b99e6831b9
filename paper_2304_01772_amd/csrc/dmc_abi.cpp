// C ABI of the differentiable Monte Carlo kernels and the generic Adam step
// (argument checks and launches).
#include <hip/hip_runtime.h>

#include <cmath>

#include "dmc_internal.hpp"
#include "spinmc.h"

using namespace spinmc;

namespace {

int status(hipError_t e) { return e == hipSuccess ? SPINMC_OK : SPINMC_E_DEVICE; }

bool valid(const spinmc_dmc_params* p) {
    return p && p->R >= 1 && p->Lx >= 2 && p->Ly >= 2 && (p->Lx & 1) == 0 && (p->Ly & 1) == 0 &&
           (int64_t)p->Lx * p->Ly <= (1 << 28) && p->n_sweeps >= 0 && std::isfinite(p->beta) &&
           std::isfinite(p->alpha) && p->alpha >= 0.f && std::isfinite(p->h) &&
           (uint64_t)p->rid0 + (uint64_t)p->R <= (1ull << 32) &&
           p->t0 <= (1ull << 31) && p->t0 + (uint64_t)p->n_sweeps <= (1ull << 31);
}

DmcArgs args(const spinmc_dmc_params* p, float* s, const float* Jx, const float* Jy) {
    DmcArgs a{};
    a.s = s;
    a.Jx = Jx;
    a.Jy = Jy;
    a.R = p->R;
    a.Lx = p->Lx;
    a.Ly = p->Ly;
    a.beta = p->beta;
    a.alpha = p->alpha;
    a.h = p->h;
    a.key0 = (uint32_t)(p->seed & 0xffffffffu);
    a.key1 = (uint32_t)(p->seed >> 32);
    a.rid0 = p->rid0;
    return a;
}

}  // namespace

extern "C" {

int64_t spinmc_dmc_save_floats(const spinmc_dmc_params* p) {
    if (!valid(p)) return SPINMC_E_INVALID;
    return (int64_t)2 * p->n_sweeps * p->R * p->Ly * (p->Lx / 2);
}

int64_t spinmc_dmc_work_floats(const spinmc_dmc_params* p) {
    if (!valid(p)) return SPINMC_E_INVALID;
    return (int64_t)2 * p->R * p->Ly * (p->Lx / 2);
}

int spinmc_dmc_forward(const spinmc_dmc_params* p, void* dev_s, const void* dev_Jx,
                       const void* dev_Jy, void* dev_save, void* stream) {
    if (!valid(p) || !dev_s || !dev_Jx || !dev_Jy || (p->n_sweeps > 0 && !dev_save))
        return SPINMC_E_INVALID;
    if (p->n_sweeps == 0) return SPINMC_OK;
    return status(launch_dmc_forward(args(p, (float*)dev_s, (const float*)dev_Jx,
                                          (const float*)dev_Jy),
                                     p->t0, p->n_sweeps, (float*)dev_save, (hipStream_t)stream));
}

int spinmc_dmc_backward(const spinmc_dmc_params* p, void* dev_s, const void* dev_Jx,
                        const void* dev_Jy, const void* dev_save, void* dev_gs, void* dev_gJx,
                        void* dev_gJy, void* dev_work, void* stream) {
    if (!valid(p) || !dev_s || !dev_Jx || !dev_Jy || !dev_gs || !dev_gJx || !dev_gJy ||
        (p->n_sweeps > 0 && (!dev_save || !dev_work)))
        return SPINMC_E_INVALID;
    if (p->n_sweeps == 0) return SPINMC_OK;
    return status(launch_dmc_backward(args(p, (float*)dev_s, (const float*)dev_Jx,
                                           (const float*)dev_Jy),
                                      p->t0, p->n_sweeps, (const float*)dev_save, (float*)dev_gs,
                                      (float*)dev_gJx, (float*)dev_gJy, (float*)dev_work,
                                      (hipStream_t)stream));
}

int spinmc_dmc_energy(const spinmc_dmc_params* p, const void* dev_s, const void* dev_Jx,
                      const void* dev_Jy, void* dev_energy, void* dev_grad, void* stream) {
    if (!valid(p) || !dev_s || !dev_Jx || !dev_Jy || !dev_energy) return SPINMC_E_INVALID;
    return status(launch_dmc_energy(args(p, (float*)dev_s, (const float*)dev_Jx,
                                         (const float*)dev_Jy),
                                    (double*)dev_energy, (float*)dev_grad, (hipStream_t)stream));
}

int spinmc_dmc_discretize(int64_t n, const void* dev_base, const void* dev_g, float eta,
                          void* dev_out, void* stream) {
    if (n < 0 || n > ((int64_t)1 << 31) || (n > 0 && (!dev_base || !dev_out)) ||
        !std::isfinite(eta))
        return SPINMC_E_INVALID;
    if (n == 0) return SPINMC_OK;
    return status(launch_dmc_discretize(n, (const float*)dev_base, (const float*)dev_g, eta,
                                        (float*)dev_out, (hipStream_t)stream));
}

int spinmc_adam(void* params, const void* grad, void* m, void* v, int64_t n, int32_t step,
                float lr, float beta1, float beta2, float eps, void* stream) {
    if (!params || !grad || !m || !v || n < 1 || n > (int64_t)1 << 31 || step < 1 ||
        !(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
        !(eps > 0.f))
        return SPINMC_E_INVALID;
    return status(launch_mlp_adam((float*)params, (const float*)grad, (float*)m, (float*)v,
                                  (int)n, step, lr, beta1, beta2, eps, (hipStream_t)stream));
}
}
