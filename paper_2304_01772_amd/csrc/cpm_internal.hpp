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

// Tiled persistent passes (range 1, Lx % 8 == 0, TH | Ly, TW | Lx, TH even,
// TW % 8 == 0): n_steps unrecorded Monte Carlo steps, one 256-thread
// workgroup per tile of every replica (n_blocks = R x tiles per replica, the
// same tile count for every replica); bar: one uint32 per replica, zero at
// launch; the device step counter is not advanced.
size_t cpm_tiled_lds_bytes(int tab_lds_bytes, int cell_cap, int TH, int TW);
hipError_t cpm_tiled_occupancy(int tab_lds_bytes, int cell_cap, int TH, int TW, int* per_cu);
hipError_t launch_cpm_tiled(const CpmArgs& a, int n_steps, int TH, int TW, int tab_lds_bytes,
                            int cell_cap, int n_blocks, uint32_t* bar, uint32_t* abort_flag,
                            hipStream_t s);

}  // namespace spinmc
