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
// covariance numerators n S_ab - S_a S_b in int128), turned into FP64 once,
// so every order of summation gives the same bits.  Short records: one
// workgroup per replica.  Long records: chunk sums with one lane per replica
// (rows of consecutive replicas are contiguous), then one thread per replica
// adds its chunks.
// the 64-bit wavefront reduction (__ockl_wfred_add_i64) of the HIP headers
#define HIP_ENABLE_EXTRA_WARP_SYNC_TYPES 1
#include "grad_internal.hpp"

#include <mutex>

namespace spinmc {

namespace {
constexpr int kSums = kCovSums;

__device__ __forceinline__ double cov_of(long long Sab, long long Sa, long long Sb, long long n) {
    const __int128 num = (__int128)n * (__int128)Sab - (__int128)Sa * (__int128)Sb;
    return (double)num / ((double)n * (double)n);
}

// adds one sample (M, Bx, By) to the 13 sums (a zero row adds nothing)
__device__ __forceinline__ void cov_add(long long (&s)[kSums], const int3 v) {
    const long long M = v.x, Bx = v.y, By = v.z;
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

// The ten covariances of a replica, term q = 0..9 from its 13 sums over n
// samples [sum Bx, By, M, |M|, Bx^2, By^2, M^2, Bx By, Bx M, By M, |M| Bx,
// |M| By, |M| M]: Cov(Bx,Bx), (By,By), (M,M), (Bx,By), (Bx,M), (By,M),
// (|M|,Bx), (|M|,By), (|M|,M), (|M|,|M|).  Each is one int128 numerator and
// one FP64 division, so the lanes of a wave take one term each.
__device__ __forceinline__ double cov_term(int q, const long long (&S)[kSums], long long n) {
    // (ab, a, b) indices into S per term
    const int ab = q < 9 ? 4 + q : 6, a = q < 3 ? q : (q < 6 ? (q == 5 ? 1 : 0) : 3);
    const int b = q < 3 ? q : (q == 3 ? 1 : (q < 6 ? 2 : (q == 9 ? 3 : q - 6)));
    return cov_of(S[ab], S[a], S[b], n);
}

// Outputs of replica r from its sums S over n samples and the covariances
// cv[q] = cov_term(q, S, n).
__device__ void cov_finish(const RepDev& D, int r, const long long (&S)[kSums], long long n,
                           const double* cv, const double* gout, double* means, double* grads,
                           double* dtheta) {
    const double N = (double)D.Lx * (double)D.Ly;
    const double Jx = D.Jx, Jy = D.Jy, h = D.h, beta = D.beta;
    // covariance matrix of X = (Bx, By, M), and of |M| with X
    const double C[3][3] = {{cv[0], cv[3], cv[4]}, {cv[3], cv[1], cv[5]}, {cv[4], cv[5], cv[2]}};
    const double CaX[3] = {cv[6], cv[7], cv[8]};
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
        means[4 * r + 3] = beta * cv[9] / N;
    }
    if (grads)
        for (int o = 0; o < 2; ++o)
            for (int j = 0; j < 3; ++j) grads[(size_t)6 * r + 3 * o + j] = g[o][j];
    if (dtheta)
        for (int j = 0; j < 3; ++j)
            dtheta[(size_t)3 * r + j] = gout[2 * r] * g[0][j] + gout[2 * r + 1] * g[1][j];
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
        for (int u = 0; u < kU; ++u) cov_add(s, v[u]);
    }
#pragma unroll
    for (int i = 0; i < kSums; ++i) red[i][threadIdx.x] = s[i];
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int i = 0; i < kSums; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + w];
        __syncthreads();
    }
    __shared__ double cv[10];
    long long S[kSums];
    for (int i = 0; i < kSums; ++i) S[i] = red[i][0];
    const long long n = n_rec - burn_in;
    if (threadIdx.x < 10) cv[threadIdx.x] = cov_term((int)threadIdx.x, S, n);
    __syncthreads();
    if (threadIdx.x == 0) cov_finish(D, r, S, n, cv, gout, means, grads, dtheta);
}

// Stage 1: workgroup (x, chunk) covers replicas 64 x .. 64 x + 63 and the
// kCovChunk samples from burn_in + kCovChunk chunk on; thread (g, l) =
// (threadIdx / 64, threadIdx % 64) sums 16 of them (all loads in flight) for
// replica 64 x + l, and the four groups meet in LDS.  A wave's loads of one
// sample are the contiguous rows of 64 replicas.  Output:
// partial[(r n_chunks + chunk) kCovSums + i].
__global__ void __launch_bounds__(256) k_cov_partial(int R, const int32_t* stats, int n_rec,
                                                     int burn_in, int width, int n_chunks,
                                                     long long* partial) {
    static_assert(kCovChunk == 4 * 16, "four groups of 16 samples");
    __shared__ long long red[3][kSums][64];
    const int l = (int)threadIdx.x & 63, g = (int)threadIdx.x >> 6;
    const int r = (int)blockIdx.x * 64 + l;
    const int chunk = (int)blockIdx.y;
    const int k0 = burn_in + chunk * kCovChunk + 16 * g;
    long long s[kSums];
#pragma unroll
    for (int i = 0; i < kSums; ++i) s[i] = 0;
    int3 v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        v[u] = make_int3(0, 0, 0);
        if (r < R && k0 + u < n_rec) {
            const int32_t* row = stats + ((size_t)(k0 + u) * R + r) * width;
            v[u] = make_int3(row[0], row[1], row[2]);
        }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) cov_add(s, v[u]);
    if (g > 0)
#pragma unroll
        for (int i = 0; i < kSums; ++i) red[g - 1][i][l] = s[i];
    __syncthreads();
    if (g != 0 || r >= R) return;
    long long* out = partial + ((size_t)r * n_chunks + chunk) * kSums;
#pragma unroll
    for (int i = 0; i < kSums; ++i) out[i] = s[i] + red[0][i][l] + red[1][i][l] + red[2][i][l];
}

// Stage 2: one wave per replica; lane j adds chunks j, j + 64, ..., the
// wavefront reduction gives every lane the sums, lanes 0..9 take one
// covariance each, lane 0 evaluates the outputs.
__global__ void __launch_bounds__(64) k_cov_final(const RepDev* reps, int n_chunks,
                                                  long long n, const long long* partial,
                                                  const double* gout, double* means,
                                                  double* grads, double* dtheta) {
    const int r = (int)blockIdx.x;
    const int lane = (int)threadIdx.x;
    long long S[kSums];
#pragma unroll
    for (int i = 0; i < kSums; ++i) S[i] = 0;
    for (int ch = lane; ch < n_chunks; ch += 64) {
        const long long* p = partial + ((size_t)r * n_chunks + ch) * kSums;
#pragma unroll
        for (int i = 0; i < kSums; ++i) S[i] += p[i];
    }
    // the wave's sums in every lane (one full wave, reconverged after the loop)
#pragma unroll
    for (int i = 0; i < kSums; ++i) S[i] = __ockl_wfred_add_i64(S[i]);
    __shared__ double cv[10];
    if (lane < 10) cv[lane] = cov_term(lane, S, n);  // every lane holds the sums
    __syncthreads();
    if (lane != 0) return;
    const RepDev D = reps[r];
    cov_finish(D, r, S, n, cv, gout, means, grads, dtheta);
}

hipError_t launch_cov_grad_split(const RepDev* reps, int R, const int32_t* stats, int n_rec,
                                 int burn_in, int width, const double* gout, double* means,
                                 double* grads, double* dtheta, long long* partial,
                                 hipStream_t s) {
    const int n = n_rec - burn_in;
    const int n_chunks = (n + kCovChunk - 1) / kCovChunk;
    hipLaunchKernelGGL(k_cov_partial, dim3((R + 63) / 64, n_chunks), dim3(256), 0, s, R, stats,
                       n_rec, burn_in, width, n_chunks, partial);
    hipLaunchKernelGGL(k_cov_final, dim3(R), dim3(64), 0, s, reps, n_chunks, (long long)n,
                       partial, gout, means, grads, dtheta);
    return hipGetLastError();
}

// Chunk sums of the allocation-free entry point (spinmc_grad_noalloc): one
// array per device for the life of the process.  Host code never passes the
// name itself (a host-side stand-in); cov_scratch resolves its device address
// once per device.  k_cov_partial writes every entry k_cov_final reads, so no
// call depends on what an earlier one left there.
static __device__ __align__(256) long long scratch[kCovScratchEntries];

hipError_t cov_scratch(int device, long long** out) {
    static std::mutex mu;
    static long long* ptr[kCovScratchDevices] = {};
    *out = nullptr;
    if (device < 0 || device >= kCovScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // the device must be current
        long long* p = nullptr;
        e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return e != hipSuccess ? e : hipErrorInvalidSymbol;
        ptr[device] = p;
    }
    *out = ptr[device];
    return hipSuccess;
}

hipError_t launch_cov_grad(const RepDev* reps, int R, const int32_t* stats, int n_rec,
                           int burn_in, int width, const double* gout, double* means,
                           double* grads, double* dtheta, hipStream_t s) {
    hipLaunchKernelGGL(k_cov_grad, dim3(R), dim3(256), 0, s, reps, R, stats, n_rec, burn_in,
                       width, gout, means, grads, dtheta);
    return hipGetLastError();
}

}  // namespace spinmc
