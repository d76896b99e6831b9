// Energy of the Ising lattice with one coupling per bond, its gradient with
// respect to the spins, and the quantised spin update: the pieces of the
// spin-value optimisation (Results, optimisation of the spin values) that
// the relaxed chain does not already provide.
//
//   H(s)   = -sum_{y,x} s[y][x] (Jx[y][x] s[y][x+1] + Jy[y][x] s[y+1][x]) - h sum s
//   dH/ds  = -(Jx[y][x] s[y][x+1] + Jx[y][x-1] s[y][x-1] + Jy[y][x] s[y+1][x]
//              + Jy[y-1][x] s[y-1][x] + h)
//   out    = -1 where base - eta g < 0, +1 elsewhere (the discretisation
//            step of Algorithm 2 applied after a gradient step)
#include "dmc_internal.hpp"

namespace spinmc {

namespace {
constexpr int kEnergyThreads = 1024;
}

// One workgroup per replica; every thread sums its sites (stride 1024) in
// FP64, then a fixed-order tree over the workgroup: the result does not
// depend on timing.  grad (optional) receives dH/ds in FP32.
__global__ void __launch_bounds__(kEnergyThreads) k_dmc_energy(DmcArgs a, double* e_out,
                                                               float* grad) {
    __shared__ double part[kEnergyThreads];
    const int Lx = a.Lx, Ly = a.Ly;
    const int n = Lx * Ly;
    const int r = blockIdx.x;
    const size_t off = (size_t)r * n;
    const float* s = a.s + off;
    const float* Jx = a.Jx + off;
    const float* Jy = a.Jy + off;
    float* g = grad ? grad + off : nullptr;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += kEnergyThreads) {
        const int y = i / Lx, x = i - y * Lx;
        const int xr = x + 1 == Lx ? 0 : x + 1, xl = x == 0 ? Lx - 1 : x - 1;
        const int yd = y + 1 == Ly ? 0 : y + 1, yu = y == 0 ? Ly - 1 : y - 1;
        const float sv = s[i];
        const float sr = s[y * Lx + xr], sd = s[yd * Lx + x];
        acc -= (double)sv * ((double)Jx[i] * (double)sr + (double)Jy[i] * (double)sd) +
               (double)a.h * (double)sv;
        if (g) {
            const float hloc = Jx[i] * sr + Jx[y * Lx + xl] * s[y * Lx + xl] + Jy[i] * sd +
                               Jy[yu * Lx + x] * s[yu * Lx + x] + a.h;
            g[i] = -hloc;
        }
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kEnergyThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) e_out[r] = part[0];
}

__global__ void __launch_bounds__(256) k_dmc_discretize(int64_t n, const float* base,
                                                        const float* g, float eta, float* out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float v = g ? base[i] - eta * g[i] : base[i];
    out[i] = v < 0.f ? -1.f : 1.f;
}

hipError_t launch_dmc_energy(const DmcArgs& a, double* e_out, float* grad, hipStream_t s) {
    hipLaunchKernelGGL(k_dmc_energy, dim3(a.R), dim3(kEnergyThreads), 0, s, a, e_out, grad);
    return hipGetLastError();
}

hipError_t launch_dmc_discretize(int64_t n, const float* base, const float* g, float eta,
                                 float* out, hipStream_t s) {
    const int64_t nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_dmc_discretize, dim3((unsigned)nb), dim3(256), 0, s, n, base, g, eta,
                       out);
    return hipGetLastError();
}

}  // namespace spinmc
