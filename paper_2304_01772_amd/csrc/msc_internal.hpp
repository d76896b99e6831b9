// Internal declarations of the multispin-coded Ising kernels (32 replicas
// per uint32 word).  Not part of the C ABI.
#pragma once
#include "spinmc_internal.hpp"

namespace spinmc {

constexpr int kModelIsingMsc = 5;
constexpr int kMscClasses = 18;  // 9 [s > 0] + 3 (Sx/2 + 1) + (Sy/2 + 1)

struct MscArgs {
    const RepDev* reps;       // per group: Lx, Ly, rid, lat_off (bytes)
    uint32_t* lat;            // packed words, two colour planes per group
    const uint64_t* tab;      // [G][18] thresholds (2^32 = always)
    const uint64_t* t_base;   // device sweep counter
    int32_t* stats;           // [rows][32 G][width]
    uint32_t key0, key1;
    int32_t G, width;         // groups; stats rows hold 32 G replicas
    int32_t max_blocks;       // max over groups of Lx Ly / 8
    int32_t max_sites;
};

hipError_t launch_msc_init(const MscArgs& a, hipStream_t s);
hipError_t launch_msc_pass(const MscArgs& a, int c, int sweep_off, hipStream_t s);
// Adds [M, Bx, By] of replica 32 g + b to stats row rec_row (zeroed first).
hipError_t launch_msc_stats(const MscArgs& a, int rec_row, hipStream_t s);

}  // namespace spinmc
