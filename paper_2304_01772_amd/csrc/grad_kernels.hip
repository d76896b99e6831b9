// Fluctuation (covariance) estimator of Ising observable gradients.
//
// For a Boltzmann weight exp(-beta H(s; theta)) every equilibrium
// expectation satisfies d<O>/dtheta = <dO/dtheta> - beta Cov(O, dH/dtheta).
// This replaces the logistic relaxation of Algorithm 2 (Methods) for
// gradients of equilibrium observables.  With the Ising energy of Eq. (1),
// H = -Jx Bx - Jy By - h M, so -dH/dtheta = X = (Bx, By, M) for
// theta = (Jx, Jy, h).  Observables: e = H/N and |m| = |M|/N.
//
// All moments are integer sums over the recorded samples (exact int64, the
// covariance numerators n S_ab - S_a S_b in int128), turned into FP64 once:
// one workgroup per replica, deterministic.
#include "spinmc_internal.hpp"

namespace spinmc {

namespace {
constexpr int kSums = 13;

__device__ __forceinline__ double cov_of(long long Sab, long long Sa, long long Sb, long long n) {
    const __int128 num = (__int128)n * (__int128)Sab - (__int128)Sa * (__int128)Sb;
    return (double)num / ((double)n * (double)n);
}
}  // namespace

__global__ void __launch_bounds__(256) k_cov_grad(const RepDev* reps, int R,
                                                  const int32_t* stats, int n_rec, int burn_in,
                                                  int width, const double* gout, double* means,
                                                  double* grads, double* dtheta) {
    __shared__ long long red[kSums][256];
    const int r = blockIdx.x;
    const RepDev D = reps[r];
    long long s[kSums];
#pragma unroll
    for (int i = 0; i < kSums; ++i) s[i] = 0;
    // eight samples' loads in flight per lane before their products
    constexpr int kU = 8;
    const int step = (int)blockDim.x;
    for (int k0 = burn_in + (int)threadIdx.x; k0 < n_rec; k0 += kU * step) {
        int3 v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int k = k0 + u * step;
            v[u] = make_int3(0, 0, 0);
            if (k < n_rec) {
                const int32_t* row = stats + ((size_t)k * R + r) * width;
                v[u] = make_int3(row[0], row[1], row[2]);
            }
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const long long M = v[u].x, Bx = v[u].y, By = v[u].z;  // zero rows add nothing
            const long long aM = M < 0 ? -M : M;
            s[0] += Bx;
            s[1] += By;
            s[2] += M;
            s[3] += aM;
            s[4] += Bx * Bx;
            s[5] += By * By;
            s[6] += M * M;
            s[7] += Bx * By;
            s[8] += Bx * M;
            s[9] += By * M;
            s[10] += aM * Bx;
            s[11] += aM * By;
            s[12] += aM * M;
        }
    }
#pragma unroll
    for (int i = 0; i < kSums; ++i) red[i][threadIdx.x] = s[i];
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int i = 0; i < kSums; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const long long n = n_rec - burn_in;
    long long S[kSums];
    for (int i = 0; i < kSums; ++i) S[i] = red[i][0];
    const double N = (double)D.Lx * (double)D.Ly;
    const double Jx = D.Jx, Jy = D.Jy, h = D.h, beta = D.beta;
    // covariance matrix of X = (Bx, By, M)
    double C[3][3];
    C[0][0] = cov_of(S[4], S[0], S[0], n);
    C[1][1] = cov_of(S[5], S[1], S[1], n);
    C[2][2] = cov_of(S[6], S[2], S[2], n);
    C[0][1] = C[1][0] = cov_of(S[7], S[0], S[1], n);
    C[0][2] = C[2][0] = cov_of(S[8], S[0], S[2], n);
    C[1][2] = C[2][1] = cov_of(S[9], S[1], S[2], n);
    double CaX[3];
    CaX[0] = cov_of(S[10], S[3], S[0], n);
    CaX[1] = cov_of(S[11], S[3], S[1], n);
    CaX[2] = cov_of(S[12], S[3], S[2], n);
    const double mX[3] = {(double)S[0] / (double)n, (double)S[1] / (double)n,
                          (double)S[2] / (double)n};
    double g[2][3];
    for (int j = 0; j < 3; ++j) {
        const double cov_e = -(Jx * C[0][j] + Jy * C[1][j] + h * C[2][j]) / N;
        g[0][j] = -mX[j] / N + beta * cov_e;
        g[1][j] = beta * CaX[j] / N;
    }
    if (means) {
        // <e>, <|m|>, <m^2>, chi = beta N (<m^2> - <|m|>^2) with the variance of
        // |M| from its exact integer moments
        means[4 * r + 0] = -(Jx * mX[0] + Jy * mX[1] + h * mX[2]) / N;
        means[4 * r + 1] = ((double)S[3] / (double)n) / N;
        means[4 * r + 2] = ((double)S[6] / (double)n) / (N * N);
        means[4 * r + 3] = beta * cov_of(S[6], S[3], S[3], n) / N;
    }
    if (grads)
        for (int o = 0; o < 2; ++o)
            for (int j = 0; j < 3; ++j) grads[(size_t)6 * r + 3 * o + j] = g[o][j];
    if (dtheta)
        for (int j = 0; j < 3; ++j)
            dtheta[(size_t)3 * r + j] = gout[2 * r] * g[0][j] + gout[2 * r + 1] * g[1][j];
}

hipError_t launch_cov_grad(const RepDev* reps, int R, const int32_t* stats, int n_rec,
                           int burn_in, int width, const double* gout, double* means,
                           double* grads, double* dtheta, hipStream_t s) {
    hipLaunchKernelGGL(k_cov_grad, dim3(R), dim3(256), 0, s, reps, R, stats, n_rec, burn_in,
                       width, gout, means, grads, dtheta);
    return hipGetLastError();
}

}  // namespace spinmc
