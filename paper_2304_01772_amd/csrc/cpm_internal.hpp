// Internal declarations of the resident CPM kernel.  Not part of the C ABI.
#pragma once
#include "spinmc_internal.hpp"

namespace spinmc {

// LDS bytes of the resident kernel: thresholds, per-cell tables of cell_cap
// entries, and the ids of the largest replica.
size_t cpm_resident_lds_bytes(int tab_lds_bytes, int cell_cap, int max_sites);

// n_steps unrecorded Monte Carlo steps of every replica in one launch, one
// workgroup per replica (range 1 with every Lx % 8 == 0, or range 2; the LDS
// above at most 64 KiB); the device step counter is not advanced.
hipError_t launch_cpm_resident(const CpmArgs& a, int n_steps, int tab_lds_bytes, int cell_cap,
                               int max_sites, hipStream_t s);

}  // namespace spinmc
