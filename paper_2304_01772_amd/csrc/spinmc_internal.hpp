// Internal types shared by the host runtime and the gfx950 kernels of
// libspinmc.  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spinmc {

constexpr int kModelIsing = 0;
constexpr int kModelPotts = 1;
constexpr int kModelCpm = 2;

// Stream tags: the fourth Philox counter word.
constexpr uint32_t kTagMain = 0u;
constexpr uint32_t kTagFallback = 1u;
constexpr uint32_t kTagInit = 2u;

constexpr int kIsingClasses = 18;
constexpr int kMaxPottsQ = 128;   // labels fit in 7 bits (SWAR equality test)
constexpr int kMaxCpmTypes = 4;
constexpr int kMaxRpb = 16;       // replicas per resident workgroup

// Resident kernel paths: per-site (any model or width), Ising chunks, Potts chunks.
constexpr int kResGeneric = 0;
constexpr int kResIsing = 1;
constexpr int kResPotts = 2;

// Per-replica record, device visible.
struct RepDev {
    int32_t model, Lx, Ly, W;     // W = bytes per plane row = Lx/2 (Ising/Potts)
    int32_t q;                    // Potts q; CPM number of cells
    uint32_t rid;
    int64_t lat_off;              // byte offset of the lattice in the lattice buffer
    int32_t tab_off, tab_n;       // thresholds: hi16 at tab_off+i, lo16 at tab_off+tab_n+i
    int32_t hist_off;             // Potts: histogram offset (int32 entries)
    int32_t cell_off;             // CPM: offset of the per-cell arrays (entries)
    int32_t n_types;              // CPM
    int32_t K1;                   // CPM: k in [1,K1) from the table (entry k-1); [K1,K0) T=1
    int32_t js_off;               // CPM: fixed-point adhesion table offset (int32)
    int32_t S;                    // CPM: fixed-point scale
    int32_t pad2;
    int64_t K0;                   // CPM: k >= K0 has T = 0 (never accepted)
    int64_t LS;                   // CPM: lambda * S
    float Jx, Jy, h, pad1;
    double beta;
};

// One unit of streamed work: rows [y0, y0 + rows) of both planes of a replica.
struct TileDev {
    int32_t rep, y0, rows, pad;
};

// One unit of a persistent workgroup's work (rows [y0, y0 + rows) of both
// planes of replica rep): a whole replica (slab = -1) or one row slab of a
// replica cut into slabs owned by different workgroups, with the pass flags
// of this slab and of the slabs above and below it.
struct PersistItem {
    int32_t rep, y0, rows;
    int32_t slab, up, down;
    int32_t pad[2];
};

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 bit
// multiplies and xors; round r uses key + r * (0x9E3779B9, 0xBB67AE85).
// Each round is two v_mad_u64_u32 and two three-input xors (v_bitop3_b32,
// truth table 0x96), which the compiler does not form by itself.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// Launch parameters common to the lattice kernels.
struct SweepArgs {
    const RepDev* reps;
    const TileDev* tiles;
    const int32_t* rep_list;      // resident kernels: replicas handled (one per workgroup)
    const uint32_t* tab;          // thresholds
    uint8_t* lat;                 // lattices
    const uint64_t* t_base;       // device sweep counter (start of the call)
    int32_t* stats;               // [n_rec][R][width] or null
    int32_t* hist;                // Potts histograms
    uint32_t key0, key1;
    int32_t R, width;
    int32_t n_sweeps, record_every;
    int32_t sweep_off;            // resident kernels: first sweep of the launch within the call
    int32_t n_units;
    int32_t tab_lds_bytes;        // bytes of LDS reserved for thresholds (multiple of 16)
    // resident kernels: replicas per workgroup, LDS bytes per replica slot,
    // and the number of entries of rep_list
    int32_t rpb, res_slot_bytes, n_list;
};

// Host-side launchers implemented in the kernel translation units.
hipError_t launch_init(const RepDev* reps, const int32_t* list, int n, uint8_t* lat,
                       uint32_t key0, uint32_t key1, int threads, hipStream_t s);
// Resident groups: chunk groups hold replicas of one model (model selects
// the path); per-site groups may mix models.
hipError_t launch_resident(const SweepArgs& a, int n_list, int model, bool chunk, int threads,
                           size_t lds_bytes, hipStream_t s);
// Allow the resident kernels up to lds_bytes of dynamic LDS (call outside capture).
hipError_t resident_reserve_lds(size_t lds_bytes);
// nt: own-plane loads and stores nontemporal (lattice sets beyond the cache)
hipError_t launch_stream_pass(const SweepArgs& a, int model, int tile0, int n_tiles, int c,
                              int sweep_off, int rec_row, int threads, size_t lds_tab_bytes,
                              bool nt, hipStream_t s);
hipError_t launch_potts_hist_finalize(const SweepArgs& a, const int32_t* list, int n, int rec_row,
                                      hipStream_t s);
// Persistent streamed passes: all 2 n_sweeps colour passes of a chunk of
// unrecorded sweeps over the streamed replicas of one model in one launch of
// n_wg workgroups of 256 threads; workgroup g owns items[item_off[g] ..
// item_off[g + 1]) (slab items alone in their workgroup, and all slab
// workgroups first).  flags: one uint32 per slab, zero at launch; *abort is
// set (and the launch leaves early) when a wait exceeds its bound.  Dynamic
// LDS: items per workgroup x slot_words x 4 bytes (threshold tables).
hipError_t launch_persist(const SweepArgs& a, int model, const PersistItem* items,
                          const int32_t* item_off, int n_wg, uint32_t* flags, uint32_t* abort_flag,
                          int slot_words, size_t lds_bytes, bool nt, hipStream_t s);
// Workgroups of 256 threads of the persistent kernel of a model that one CU
// holds at once with lds_bytes of dynamic LDS.
hipError_t persist_occupancy(int model, bool nt, size_t lds_bytes, int* per_cu);
hipError_t persist_reserve_lds(size_t lds_bytes);
hipError_t launch_fill_i32(int32_t* p, size_t n, int32_t v, hipStream_t s);
hipError_t launch_advance(uint64_t* t, uint64_t n, hipStream_t s);
// t[1] = t[0] (the start counter of resident launches that run beside
// graph replays advancing t[0])
hipError_t launch_copy_counter(uint64_t* t, hipStream_t s);
hipError_t launch_measure(const RepDev* reps, const int32_t* list, int n, int max_sites,
                          const uint8_t* lat, int32_t* stats, int32_t* hist, int width,
                          hipStream_t s);
hipError_t launch_observables(const RepDev* reps, int R, const int32_t* stats, int width,
                              double* obs, hipStream_t s);
hipError_t launch_cov_grad(const RepDev* reps, int R, const int32_t* stats, int n_rec,
                           int burn_in, int width, const double* gout, double* means,
                           double* grads, double* dtheta, hipStream_t s);

// CPM
struct CpmArgs {
    const RepDev* reps;
    const TileDev* tiles;
    const uint32_t* tab;
    int32_t* lat;                 // cell ids (int32, natural layout)
    const int8_t* ctype;
    const int32_t* target;
    int32_t* area;                // areas between calls (and at recorded steps)
    int32_t* snap;                // copy of the areas written by the resident kernel
    // Streamed passes: pass P (= n_col t + c) reads its snapshot as
    // sbuf[P & 1] + dbuf[(P - 1) mod 3], adds its changes into dbuf[P mod 3]
    // and writes sbuf[(P + 1) & 1] (its snapshot) and zeroes dbuf[(P + 1) mod
    // 3] for the next pass; buffers of total_cells entries each.
    int32_t* sbuf;                // [2][total_cells]
    int32_t* dbuf;                // [3][total_cells]
    int32_t total_cells;
    const int32_t* js;            // fixed-point adhesion
    const uint64_t* t_base;
    int32_t* stats;
    uint32_t key0, key1;
    int32_t R, width;
    int32_t range;                // neighbourhood: 1 Moore 3x3, 2 the 5x5 square
};
hipError_t launch_cpm_pass(const CpmArgs& a, int n_tiles, int c, int sweep_off, int threads,
                           size_t lds_tab_bytes, hipStream_t s);
// The 5x5 neighbourhood (range 2): colour c of the 3x3 sublattice, one site
// per lane; tiles of whole multiples of 3 rows.
hipError_t launch_cpm_pass5(const CpmArgs& a, int n_tiles, int c, int sweep_off, int threads,
                            size_t lds_tab_bytes, hipStream_t s);
// Four same-colour sites per lane (threads <= 256), or one site per lane
// with four lanes per Philox quad (threads 512 or 1024), the cell tables and
// the pass's area changes in LDS: needs every Lx a multiple of 8 and
// cell_cap >= n_cells + 1 (a multiple of 16) for every replica; dynamic LDS
// cpm_quad_lds_bytes.
size_t cpm_quad_lds_bytes(int tab_lds_bytes, int cell_cap);
hipError_t launch_cpm_pass_quad(const CpmArgs& a, int n_tiles, int c, int sweep_off,
                                int threads, int tab_lds_bytes, int cell_cap, hipStream_t s);
// Allow both forms of the quad pass up to lds_bytes of dynamic LDS (call
// outside capture).
hipError_t cpm_reserve_lds(size_t lds_bytes);
// Before a call's streamed passes: sbuf[P0 & 1] = area, dbuf[(P0 - 1) mod 3]
// = dbuf[P0 mod 3] = 0 for the pass P0 = n_col (t + sweep_off).
hipError_t launch_cpm_pass_init(const CpmArgs& a, int sweep_off, hipStream_t s);
// After the passes before pass P = n_col (t + sweep_off): area = the
// snapshot pass P would read.
hipError_t launch_cpm_pass_final(const CpmArgs& a, int sweep_off, hipStream_t s);
hipError_t launch_cpm_stats(const CpmArgs& a, int n_tiles, int rec_row, hipStream_t s);
hipError_t launch_cpm_area_recount(const CpmArgs& a, int n_tiles, int total_cells, hipStream_t s);

// Surrogate MLP
hipError_t launch_mlp_forward(const float* params, const float* x, int B, float* y, float* act,
                              hipStream_t s);
hipError_t launch_mlp_backward(const float* params, const float* x, const float* act,
                               const float* t, const float* w, int B, float* grad, float* dx,
                               float* loss, float* scratch, hipStream_t s);
hipError_t launch_mlp_adam(float* params, const float* grad, float* m, float* v, int n, int step,
                           float lr, float b1, float b2, float eps, hipStream_t s);
// forward (pre-activations into act), backward (partials into scratch), and
// the fixed-order reduction fused with the Adam update: three launches
hipError_t launch_mlp_train_step(float* params, const float* x, const float* t, const float* w,
                                 int B, float* grad, float* m, float* v, int step, float lr,
                                 float b1, float b2, float eps, float* loss, float* act,
                                 float* scratch, hipStream_t s);

}  // namespace spinmc
