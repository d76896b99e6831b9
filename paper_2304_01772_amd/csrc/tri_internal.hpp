// Internal declarations of the triangular (three colour planes) and the
// chain / square / simple-cubic (two colour planes) Ising kernels.  Not part
// of the C ABI.
#pragma once
#include "spinmc_internal.hpp"

namespace spinmc {

constexpr int kModelIsingTri = 3;
constexpr int kModelIsingHC = 4;  // chain / square / cubic; RepDev.q holds Lz
constexpr int kTriClasses = 14;  // 7 [s > 0] + (S6 + 6) / 2

struct TriArgs {
    const RepDev* reps;       // Lx, Ly, rid, lat_off (bytes), Jx = J, h
    int8_t* lat;              // int8 spins +-1 in colour planes: triangular three of Ly
                              // rows by Lx / 3, chain / cubic two of Ly Lz rows by Lx / 2
    const uint64_t* tab;      // [R][14] thresholds (2^32 = always)
    const uint64_t* t_base;   // device sweep counter
    int32_t* stats;           // [rows][R][width]
    uint32_t key0, key1;
    int32_t R, width;
    int32_t max_blocks;       // max over replicas of ceil(Lx Ly / 12)
    int32_t max_sites;
    int32_t all_lx12;         // every Lx a multiple of 12: the span kernel
    int32_t model;            // kModelIsingTri or kModelIsingHC (one per context)
    int32_t all_lx8;          // every Lx a multiple of 8: the chain / cubic span kernel
};

hipError_t launch_tri_init(const TriArgs& a, hipStream_t s);
// Colour pass c of sweep *t_base + sweep_off for every replica.
hipError_t launch_tri_pass(const TriArgs& a, int c, int sweep_off, hipStream_t s);
// Adds [M, Bh, Bv, Bd] of every replica to stats row rec_row (zeroed first
// by the caller).
hipError_t launch_tri_stats(const TriArgs& a, int rec_row, hipStream_t s);
hipError_t launch_tri_observables(const TriArgs& a, double* obs, hipStream_t s);
// n_sweeps sweeps of every replica in one launch, lattices in LDS
// (lds_bytes >= the largest lattice; Lx % 12 == 0 triangular, % 8 == 0
// chain / cubic; with re > 0 also 16 B per recorded row of the launch).
// The launch holds sweeps sw0 .. sw0 + n_sweeps - 1 of a call; with re > 0,
// sweep k re of the call stores its statistics in stats row k - 1 (columns
// 0..3; the caller zeroes the rows).
hipError_t launch_nat_resident(const TriArgs& a, int n_sweeps, int sw0, int re, int lds_bytes,
                               hipStream_t s);

}  // namespace spinmc
