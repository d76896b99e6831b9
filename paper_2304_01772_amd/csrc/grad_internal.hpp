// Internal declarations of the split covariance estimator.  Not part of the
// C ABI.
#pragma once
#include "spinmc_internal.hpp"

namespace spinmc {

// Records of at least kCovSplitMin samples take the split form: stage 1 sums
// chunks of kCovChunk samples, 64 replicas per workgroup (a wave reads 64
// consecutive replicas' rows of one sample), stage 2 adds a replica's chunks
// in one wave and evaluates its outputs.  The sums are exact integers, so the split
// changes no bit of the result.
constexpr int kCovChunk = 64;
constexpr int kCovSplitMin = 512;
constexpr int kCovSums = 13;

// int64 entries of the stage-1 buffer for R replicas and n samples
inline size_t cov_partial_entries(int R, int n) {
    return (size_t)((n + kCovChunk - 1) / kCovChunk) * kCovSums * (size_t)R;
}

// Capacity of the per-device static chunk-sum array behind
// spinmc_grad_noalloc: 4 MiB of int64 entries (for 256 replicas, records of
// up to 10,048 samples), for devices 0 .. kCovScratchDevices - 1.
constexpr size_t kCovScratchEntries = ((size_t)4 << 20) / sizeof(long long);
constexpr int kCovScratchDevices = 64;

// Device address of that array on `device`, which must be the current
// device the first time it is asked for (resolved once per device).
hipError_t cov_scratch(int device, long long** out);

hipError_t launch_cov_grad_split(const RepDev* reps, int R, const int32_t* stats, int n_rec,
                                 int burn_in, int width, const double* gout, double* means,
                                 double* grads, double* dtheta, long long* partial,
                                 hipStream_t s);

}  // namespace spinmc
