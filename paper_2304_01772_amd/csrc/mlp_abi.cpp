// C ABI of the surrogate MLP kernels (argument checks and launches).
#include <hip/hip_runtime.h>

#include "spinmc.h"
#include "spinmc_internal.hpp"

namespace spinmc {
int mlp_num_params();
int mlp_scratch_floats(int B);
}  // namespace spinmc

using namespace spinmc;

namespace {
int status(hipError_t e) { return e == hipSuccess ? SPINMC_OK : SPINMC_E_DEVICE; }
}  // namespace

extern "C" {

int spinmc_mlp_num_params(void) { return mlp_num_params(); }

int spinmc_mlp_act_floats(int32_t B) { return B > 0 ? B * 256 : SPINMC_E_INVALID; }

int spinmc_mlp_workspace_floats(int32_t B) {
    return B > 0 ? mlp_scratch_floats(B) : SPINMC_E_INVALID;
}

int spinmc_mlp_forward(const void* params, const void* x, int32_t B, void* y, void* act,
                       void* stream) {
    if (!params || !x || !y || B < 1) return SPINMC_E_INVALID;
    return status(launch_mlp_forward((const float*)params, (const float*)x, B, (float*)y,
                                     (float*)act, (hipStream_t)stream));
}

int spinmc_mlp_backward(const void* params, const void* x, const void* act, const void* t,
                        const void* w, int32_t B, void* grad, void* dx, void* loss,
                        void* workspace, void* stream) {
    if (!params || !x || !act || !t || !w || !grad || !workspace || B < 1)
        return SPINMC_E_INVALID;
    return status(launch_mlp_backward((const float*)params, (const float*)x, (const float*)act,
                                      (const float*)t, (const float*)w, B, (float*)grad,
                                      (float*)dx, (float*)loss, (float*)workspace,
                                      (hipStream_t)stream));
}

int spinmc_mlp_train_step(void* params, const void* x, const void* t, const void* w, int32_t B,
                          void* grad, void* m, void* v, int32_t step, float lr, float beta1,
                          float beta2, float eps, void* loss, void* act, void* workspace,
                          void* stream) {
    if (!params || !x || !t || !w || !m || !v || !act || !workspace || B < 1 || step < 1 ||
        !(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
        !(eps > 0.f))
        return SPINMC_E_INVALID;
    return status(launch_mlp_train_step((float*)params, (const float*)x, (const float*)t,
                                        (const float*)w, B, (float*)grad, (float*)m, (float*)v,
                                        step, lr, beta1, beta2, eps, (float*)loss, (float*)act,
                                        (float*)workspace, (hipStream_t)stream));
}

int spinmc_mlp_adam(void* params, const void* grad, void* m, void* v, int32_t step, float lr,
                    float beta1, float beta2, float eps, void* stream) {
    if (!params || !grad || !m || !v || step < 1 || !(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
        !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return SPINMC_E_INVALID;
    return status(launch_mlp_adam((float*)params, (const float*)grad, (float*)m, (float*)v,
                                  mlp_num_params(), step, lr, beta1, beta2, eps,
                                  (hipStream_t)stream));
}
}
