// Host runtime of libspinmc: validation, FP64 Metropolis thresholds, device
// memory, state I/O, schedules, and the C ABI declared in include/spinmc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>

#include "cpm_internal.hpp"
#include "grad_internal.hpp"
#include "msc_internal.hpp"
#include "tri_internal.hpp"
#include <vector>

#include "spinmc.h"
#include "spinmc_internal.hpp"

using namespace spinmc;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

constexpr size_t kAlign = 256;
constexpr int kResidentMaxBytes = 128 * 1024;  // lattice bytes kept in LDS by the resident kernel
constexpr int kMaxCpmCells = 1 << 20;
constexpr int kGraphChunk = 50;  // sweeps per captured graph
constexpr int kSide = 4;         // side streams for concurrent resident groups
constexpr size_t kResidentLdsBudget = 150 * 1024;
// Streamed lattice sets beyond this size do not stay in the 256 MB last-level
// cache between passes: their own-plane traffic goes nontemporal by default.
constexpr size_t kNtAutoBytes = 192ull << 20;
constexpr int kCpmLdsCells = 16384;  // cells (medium included) per replica in LDS tables
constexpr size_t kCpmQuadLdsMax = 160 * 1024;  // LDS of one workgroup of the quad pass

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Metropolis threshold of Algorithm 1 for a uniform 32-bit word W:
// accept iff W < T with T = 2^32 when dE <= 0, else ceil(2^32 exp(-beta dE)).
uint64_t metropolis_threshold(double dE, double beta) {
    if (dE <= 0.0) return (uint64_t)1 << 32;
    return (uint64_t)std::ceil(std::ldexp(std::exp(-beta * dE), 32));
}

// Ising, Eq. (1): flipping s with neighbour sums Sx, Sy changes the energy by
// dE = 2 s (Jx Sx + Jy Sy + h); class 9[s>0] + 3(Sx/2+1) + (Sy/2+1).
void ising_thresholds(float Jx, float Jy, float h, double beta, std::vector<uint64_t>& T) {
    T.assign(kIsingClasses, 0);
    for (int si = 0; si < 2; ++si)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                const double s = si ? 1.0 : -1.0;
                const double Sx = 2.0 * a - 2.0, Sy = 2.0 * b - 2.0;
                double u = (double)Jx * Sx;
                u = u + (double)Jy * Sy;
                u = u + (double)h;
                const double dE = 2.0 * s * u;
                T[9 * si + 3 * a + b] = metropolis_threshold(dE, beta);
            }
}

// Potts, Eq. (2): s -> s' changes the energy by dE = -(J dn + h (s' - s)),
// dn = #{neighbours == s'} - #{neighbours == s}; class (dn+4)(2q-1)+(s'-s+q-1).
void potts_thresholds(int q, float J, float h, double beta, std::vector<uint64_t>& T) {
    T.assign((size_t)9 * (2 * q - 1), 0);
    for (int dn = -4; dn <= 4; ++dn)
        for (int ds = -(q - 1); ds <= q - 1; ++ds) {
            double u = (double)J * (double)dn;
            u = u + (double)h * (double)ds;
            const double dE = -u;
            T[(size_t)(dn + 4) * (2 * q - 1) + (ds + q - 1)] = metropolis_threshold(dE, beta);
        }
}

struct HostRep {
    spinmc_replica_desc d{};
    std::vector<float> adh;
    std::vector<int8_t> ctype;
    std::vector<int32_t> target;
    std::vector<uint64_t> T;
    int64_t aux = 0;
    RepDev dev{};
    bool chunk = false;     // W % 16 == 0: 16-byte SWAR path
    bool resident = false;  // fits the resident kernel's LDS
    size_t lat_bytes = 0;
};

}  // namespace

struct spinmc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    uint64_t seed = 0;
    uint64_t t = 0;
    bool poisoned = false;
    int R = 0;
    int width = 8;
    bool cpm = false;
    std::vector<HostRep> reps;
    int max_tab_n = 0;
    int max_sites = 0;
    // device buffers
    uint8_t* d_lat = nullptr;
    size_t lat_bytes = 0;
    RepDev* d_reps = nullptr;
    uint32_t* d_tab = nullptr;
    uint64_t* d_t = nullptr;
    int32_t* d_hist = nullptr;
    int32_t* d_lists = nullptr;  // [all | potts | chunk-resident | generic-resident | stream-exempt]
    std::vector<int32_t> all_list, potts_list, res_chunk, res_gen, stream_rest;
    int off_all = 0, off_potts = 0, off_res_chunk = 0, off_rest = 0;
    TileDev* d_tiles = nullptr;
    int n_tiles = 0;
    int n_tiles_ising = 0;  // streamed Ising tiles come first in d_tiles
    int tiles_rows = 0;
    int tiles_threads = 0;  // CPM: pass threads the tiles were sized for
    spinmc_schedule sched{0, 0, 0, 0};
    bool prepared = false;
    long prepared_key = 0;
    std::vector<int32_t> stream_potts;
    // hipGraphs of whole chunks of unrecorded sweeps, keyed by chunk length
    bool use_graphs = true;
    std::map<int, hipGraphExec_t> graphs;
    // side streams: [0] graph capture origin, [1..kSide] resident groups;
    // events: [0] fork, [1..kSide] joins
    hipStream_t cap[1 + kSide] = {};
    hipEvent_t cap_ev[1 + kSide] = {};
    // resident workgroup groups (replicas of one shape packed rpb per workgroup)
    bool nt_ising = false, nt_potts = false;  // nontemporal own-plane access per model
    struct ResGroup {
        int off, count, rpb, threads, model;
        bool chunk;
        size_t slot;
    };
    std::vector<ResGroup> res_groups;
    // persistent streamed passes (schedule flag SPINMC_SCHED_PERSIST): one
    // plan per model (Ising, Potts) over the streamed replicas
    struct PersistPlan {
        int n_wg = 0, n_slabs = 0, off0 = 0, slot_words = 0;
        size_t lds = 0;
    };
    bool persist = false;
    PersistPlan pplan[2];
    PersistItem* d_pitems = nullptr;
    int32_t* d_poff = nullptr;
    uint32_t* d_pflags = nullptr;  // [0] abort word, [1 .. n_pflags] pass flags of the slabs
    int n_pflags = 0;              // capacity in flags
    int n_pflags_used = 0;
    bool persist_used = false;
    // Cellular Potts
    int8_t* d_ctype = nullptr;
    int32_t* d_target = nullptr;
    int32_t* d_area = nullptr;
    int32_t* d_snap = nullptr;
    int32_t* d_sbuf = nullptr;  // [2][total_cells] pass snapshots of the streamed passes
    int32_t* d_dbuf = nullptr;  // [3][total_cells] pass area changes
    int32_t* d_js = nullptr;
    int total_cells = 0;
    // CPM passes with four sites per lane and LDS cell tables (every Lx a
    // multiple of 8, at most kCpmLdsCells cells per replica)
    bool cpm_quad = false, cpm_lds_reserved = false;
    int cpm_range = 1;  // 1: Moore 3x3, 4 colours; 2: 5x5, 9 colours
    bool cpm_areas_dirty = false;  // set_state since the last area count
    // triangular-lattice Ising (and chain / cubic)
    bool tri = false;
    uint64_t* d_tab64 = nullptr;  // [R][14] thresholds ([G][18] multispin-coded)
    // multispin-coded Ising: reps holds the G groups, R = 32 G
    bool msc = false;
    RepDev* d_reps_obs = nullptr;  // one square-lattice Ising entry per replica
    long long* d_cov_part = nullptr;  // chunk sums of the split covariance estimator
    size_t cov_part_n = 0;
    int cpm_cell_cap = 0;
    uint32_t* d_cpm_bar = nullptr;  // tiled persistent CPM passes: [0] abort word, [1 .. R] barriers
    bool cpm_tiled_used = false;
    // kernel timing
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> prof_recs;
};

namespace {

int check_dev(spinmc_ctx* c, hipError_t e, const char* what) {
    if (e == hipSuccess) return SPINMC_OK;
    c->poisoned = true;
    return fail(SPINMC_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

hipEvent_t next_event(spinmc_ctx* c) {
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[c->ev_used++];
}

// Bracket one kernel launch with events when timing is on.
template <class F>
hipError_t timed(spinmc_ctx* c, int kind, F&& launch, hipStream_t s) {
    if (!c->prof) return launch();
    hipEvent_t a = next_event(c), b = next_event(c);
    if (!a || !b) return launch();
    hipError_t e = hipEventRecord(a, s);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) c->prof_recs.emplace_back(kind, a, b);
    return e;
}

void free_all(spinmc_ctx* c) {
    for (auto& kv : c->graphs) hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    for (int k = 0; k < 1 + kSide; ++k) {
        if (c->cap[k]) hipStreamDestroy(c->cap[k]);
        c->cap[k] = nullptr;
        if (c->cap_ev[k]) hipEventDestroy(c->cap_ev[k]);
        c->cap_ev[k] = nullptr;
    }
    for (hipEvent_t e : c->ev_pool) hipEventDestroy(e);
    c->ev_pool.clear();
    c->ev_used = 0;
    c->prof_recs.clear();
    hipFree(c->d_lat);
    hipFree(c->d_reps);
    hipFree(c->d_tab);
    hipFree(c->d_t);
    hipFree(c->d_hist);
    hipFree(c->d_lists);
    hipFree(c->d_tiles);
    hipFree(c->d_ctype);
    hipFree(c->d_target);
    hipFree(c->d_area);
    hipFree(c->d_snap);
    hipFree(c->d_sbuf);
    hipFree(c->d_dbuf);
    hipFree(c->d_cpm_bar);
    c->d_cpm_bar = nullptr;
    c->d_sbuf = nullptr;
    c->d_dbuf = nullptr;
    hipFree(c->d_js);
    hipFree(c->d_tab64);
    c->d_tab64 = nullptr;
    hipFree(c->d_reps_obs);
    c->d_reps_obs = nullptr;
    hipFree(c->d_cov_part);
    c->d_cov_part = nullptr;
    c->cov_part_n = 0;
    hipFree(c->d_pitems);
    hipFree(c->d_poff);
    hipFree(c->d_pflags);
    c->d_pitems = nullptr;
    c->d_poff = nullptr;
    c->d_pflags = nullptr;
    c->d_ctype = nullptr;
    c->d_target = nullptr;
    c->d_area = nullptr;
    c->d_snap = nullptr;
    c->d_js = nullptr;
    c->d_lat = nullptr;
    c->d_reps = nullptr;
    c->d_tab = nullptr;
    c->d_t = nullptr;
    c->d_hist = nullptr;
    c->d_lists = nullptr;
    c->d_tiles = nullptr;
}

int validate(const spinmc_replica_desc& d, int i, bool& cpm_seen, bool& lat_seen) {
    if (d.model != SPINMC_ISING && d.model != SPINMC_POTTS && d.model != SPINMC_CPM &&
        d.model != SPINMC_ISING_TRI && d.model != SPINMC_ISING_HC && d.model != SPINMC_ISING_MSC)
        return fail(SPINMC_E_INVALID, "replica %d: unknown model %d", i, d.model);
    if (d.model == SPINMC_ISING_MSC) {
        if (d.Lx < 8 || d.Lx % 8 || d.Ly < 2 || (d.Ly & 1))
            return fail(SPINMC_E_INVALID,
                        "replica %d: multispin coding needs Lx a multiple of 8, Ly even >= 2", i);
        if ((int64_t)d.Lx * d.Ly > (1 << 28))
            return fail(SPINMC_E_INVALID, "replica %d: lattice too large", i);
        if (!std::isfinite(d.Jx) || !std::isfinite(d.Jy) || !std::isfinite(d.h))
            return fail(SPINMC_E_INVALID, "replica %d: non-finite coupling or field", i);
        if (!(d.beta >= 0.0) || !std::isfinite(d.beta))
            return fail(SPINMC_E_INVALID, "replica %d: beta must be finite and >= 0", i);
        return SPINMC_OK;
    }
    if (d.model == SPINMC_ISING_HC) {
        const int64_t Lz = d.Lz > 1 ? d.Lz : 1;
        auto ok = [](int64_t L) { return L == 1 || (L >= 2 && L % 2 == 0); };
        if (d.Lx < 2 || (d.Lx & 1) || !ok(d.Ly) || !ok(Lz) || d.Lz < 0)
            return fail(SPINMC_E_INVALID,
                        "replica %d: chain / cubic lattice needs Lx even >= 2, Ly and Lz 1 or even", i);
        if ((int64_t)d.Lx * d.Ly * Lz > (1 << 28))
            return fail(SPINMC_E_INVALID, "replica %d: lattice too large", i);
        if (!std::isfinite(d.Jx) || !std::isfinite(d.h) || d.Jy != d.Jx)
            return fail(SPINMC_E_INVALID, "replica %d: J must be finite, Jy == Jx", i);
        if (!(d.beta >= 0.0) || !std::isfinite(d.beta))
            return fail(SPINMC_E_INVALID, "replica %d: beta must be finite and >= 0", i);
        return SPINMC_OK;
    }
    if (d.model == SPINMC_ISING_TRI) {
        if (d.Lx < 3 || d.Ly < 3 || d.Lx % 3 || d.Ly % 3)
            return fail(SPINMC_E_INVALID,
                        "replica %d: the triangular lattice needs Lx, Ly multiples of 3", i);
        if ((int64_t)d.Lx * d.Ly > (1 << 28))
            return fail(SPINMC_E_INVALID, "replica %d: lattice too large", i);
        if (!std::isfinite(d.Jx) || !std::isfinite(d.h) || d.Jy != d.Jx)
            return fail(SPINMC_E_INVALID, "replica %d: triangular J must be finite, Jy == Jx", i);
        if (!(d.beta >= 0.0) || !std::isfinite(d.beta))
            return fail(SPINMC_E_INVALID, "replica %d: beta must be finite and >= 0", i);
        return SPINMC_OK;
    }
    if (d.Lx < 2 || d.Ly < 2 || (d.Lx & 1) || (d.Ly & 1))
        return fail(SPINMC_E_INVALID, "replica %d: Lx, Ly must be even and >= 2 (got %d x %d)", i,
                    d.Lx, d.Ly);
    if ((int64_t)d.Lx * d.Ly > (1 << 28))
        return fail(SPINMC_E_INVALID, "replica %d: lattice too large", i);
    if (d.model == SPINMC_CPM) {
        cpm_seen = true;
        if (d.q < 1 || d.q > kMaxCpmCells)
            return fail(SPINMC_E_INVALID, "replica %d: CPM needs 1 <= n_cells <= %d", i, kMaxCpmCells);
        if (d.n_types < 1 || d.n_types > kMaxCpmTypes)
            return fail(SPINMC_E_INVALID, "replica %d: CPM needs 1 <= n_types <= %d", i,
                        kMaxCpmTypes);
        if (!d.adhesion || !d.cell_type || !d.target_area)
            return fail(SPINMC_E_INVALID, "replica %d: CPM tables missing", i);
        if (!(d.temperature > 0.0) || !std::isfinite(d.temperature))
            return fail(SPINMC_E_INVALID, "replica %d: CPM temperature must be > 0", i);
        if (!(d.lambda_area >= 0.0f) || !std::isfinite(d.lambda_area))
            return fail(SPINMC_E_INVALID, "replica %d: CPM lambda must be >= 0", i);
        if (d.cell_type[0] != 0)
            return fail(SPINMC_E_INVALID, "replica %d: cell_type[0] (medium) must be 0", i);
        if (d.cpm_range < 0 || d.cpm_range > 2)
            return fail(SPINMC_E_INVALID, "replica %d: cpm_range must be 0, 1 or 2", i);
        if (d.cpm_range == 2 && (d.Lx % 6 != 0 || d.Ly % 6 != 0))
            return fail(SPINMC_E_INVALID,
                        "replica %d: the 5x5 neighbourhood needs Lx, Ly multiples of 6", i);
        for (int k = 0; k <= d.q; ++k)
            if (d.cell_type[k] < 0 || d.cell_type[k] >= d.n_types)
                return fail(SPINMC_E_INVALID, "replica %d: cell type out of range", i);
        for (int a = 0; a < d.n_types; ++a)
            for (int b = 0; b < d.n_types; ++b) {
                const float v = d.adhesion[a * d.n_types + b];
                if (!std::isfinite(v) || v != d.adhesion[b * d.n_types + a])
                    return fail(SPINMC_E_INVALID, "replica %d: adhesion must be finite, symmetric",
                                i);
            }
        return SPINMC_OK;
    }
    lat_seen = true;
    if (!std::isfinite(d.Jx) || !std::isfinite(d.Jy) || !std::isfinite(d.h))
        return fail(SPINMC_E_INVALID, "replica %d: non-finite coupling or field", i);
    if (!(d.beta >= 0.0) || !std::isfinite(d.beta))
        return fail(SPINMC_E_INVALID, "replica %d: beta must be finite and >= 0", i);
    if (d.model == SPINMC_POTTS) {
        if (d.q < 2 || d.q > 255)
            return fail(SPINMC_E_INVALID, "replica %d: Potts q must be in [2, 255]", i);
        if (d.q > kMaxPottsQ)
            return fail(SPINMC_E_UNSUPPORTED, "replica %d: Potts q > %d not supported", i,
                        kMaxPottsQ);
        if (d.Jy != d.Jx)
            return fail(SPINMC_E_UNSUPPORTED, "replica %d: Potts needs Jy == Jx", i);
    }
    return SPINMC_OK;
}

// ----------------------------------------------------------- Cellular Potts
// Fixed point of Eq. (3): the smallest S = 2^s (s <= 8) that makes every
// J[a][b] S and lambda S an integer below 2^20 in magnitude; thresholds
// T(k) = ceil(2^32 exp(-k / (S T_temp))) for k = 1..K1-1, T = 1 for
// K1 <= k < K0, T = 0 from K0 on.
struct CpmFixed {
    int32_t S = 1;
    std::vector<int32_t> JS;
    int64_t LS = 0;
    std::vector<uint64_t> T;
    int32_t K1 = 1;
    int64_t K0 = 1;
};

constexpr int kMaxCpmTable = 16384;  // thresholds staged in LDS (<= 128 KiB)

uint64_t cpm_T(int64_t k, int32_t S, double temp) {
    return (uint64_t)std::ceil(std::ldexp(std::exp(-(double)k / ((double)S * temp)), 32));
}

int cpm_fixed_point(const spinmc_replica_desc& d, int i, CpmFixed& f) {
    const int nt = d.n_types;
    int s;
    for (s = 0; s <= 8; ++s) {
        const double S = std::ldexp(1.0, s);
        bool ok = true;
        for (int k = 0; k < nt * nt && ok; ++k) {
            const double v = (double)d.adhesion[k] * S;
            if (!(std::fabs(v) < 1048576.0) || v != std::floor(v)) ok = false;
        }
        const double l = (double)d.lambda_area * S;
        if (!(std::fabs(l) < 1048576.0) || l != std::floor(l)) ok = false;
        if (ok) break;
    }
    if (s > 8)
        return fail(SPINMC_E_NOT_REPRESENTABLE,
                    "replica %d: adhesion / lambda not exact in a fixed-point scale <= 256", i);
    f.S = 1 << s;
    f.JS.resize((size_t)nt * nt);
    for (int k = 0; k < nt * nt; ++k) f.JS[k] = (int32_t)std::llround((double)d.adhesion[k] * f.S);
    f.LS = (int64_t)std::llround((double)d.lambda_area * f.S);
    f.T.clear();
    int64_t k = 1;
    for (;; ++k) {
        const uint64_t t = cpm_T(k, f.S, d.temperature);
        if (t <= 1) break;
        f.T.push_back(t);
        if ((int64_t)f.T.size() > kMaxCpmTable)
            return fail(SPINMC_E_UNSUPPORTED, "replica %d: CPM temperature too high for the table",
                        i);
    }
    f.K1 = (int32_t)k;
    if (cpm_T(k, f.S, d.temperature) == 0) {
        f.K0 = k;
        return SPINMC_OK;
    }
    // smallest k with T(k) = 0 (exp underflow), by doubling then bisection
    int64_t lo = k, hi = k;
    while (cpm_T(hi, f.S, d.temperature) != 0) {
        lo = hi;
        if (hi > ((int64_t)1 << 61)) {
            f.K0 = INT64_MAX;
            return SPINMC_OK;
        }
        hi *= 2;
    }
    while (hi - lo > 1) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (cpm_T(mid, f.S, d.temperature) == 0)
            hi = mid;
        else
            lo = mid;
    }
    f.K0 = hi;
    return SPINMC_OK;
}

int cpm_prepare_tables(const spinmc_replica_desc* d, int n) {
    for (int i = 0; i < n; ++i) {
        CpmFixed f;
        int rc = cpm_fixed_point(d[i], i, f);
        if (rc) return rc;
    }
    return SPINMC_OK;
}

int create_cpm(const spinmc_replica_desc* d, int n, uint64_t seed, void* stream,
               spinmc_ctx** out);

size_t resident_lds(const spinmc_ctx* c, const HostRep& r) {
    return align_up((size_t)8 * c->max_tab_n, 16) + r.lat_bytes;
}

int enqueue_sweep(spinmc_ctx* c, int n, int re, int32_t* stats);
int persist_check(spinmc_ctx* c);
int cpm_set_state(spinmc_ctx* c, int r, const void* host, size_t bytes);
int cpm_get_state(spinmc_ctx* c, int r, void* host, size_t bytes);
int cpm_sweep(spinmc_ctx* c, int n, int re, int32_t* stats);
int cpm_recount_if_dirty(spinmc_ctx* c);
bool cpm_tiled_plan(spinmc_ctx* c, int* TH, int* TW, int* n_blocks);
int create_tri(const spinmc_replica_desc* d, int n, uint64_t seed, int init, void* stream,
               spinmc_ctx** out);
int tri_set_state(spinmc_ctx* c, int r, const void* host, size_t bytes);
int tri_get_state(spinmc_ctx* c, int r, void* host, size_t bytes);
int tri_sweep(spinmc_ctx* c, int n, int re, int32_t* stats);
int tri_measure(spinmc_ctx* c, int32_t* stats, double* obs);
int create_msc(const spinmc_replica_desc* d, int n, uint64_t seed, int init, void* stream,
               spinmc_ctx** out);
int msc_sweep(spinmc_ctx* c, int n, int re, int32_t* stats);
int msc_measure(spinmc_ctx* c, int32_t* stats, double* obs);
int cpm_measure(spinmc_ctx* c, int32_t* stats, double* obs);
int default_tile_rows(const HostRep& h);
int effective_mode(const spinmc_ctx* c);

}  // namespace

// ===================================================================== ABI
extern "C" {

const char* spinmc_last_error(void) { return g_err.c_str(); }

int spinmc_create(const spinmc_replica_desc* d, int32_t n, uint64_t seed, int32_t init,
                  void* hip_stream, spinmc_ctx** out) {
    if (!d || !out || n < 1) return fail(SPINMC_E_INVALID, "create: null argument or n < 1");
    *out = nullptr;
    if (init != 0 && init != 1) return fail(SPINMC_E_INVALID, "create: init must be 0 or 1");
    bool cpm_seen = false, lat_seen = false;
    int n_tri = 0, n_hc = 0, n_msc = 0;
    for (int i = 0; i < n; ++i) {
        int rc = validate(d[i], i, cpm_seen, lat_seen);
        if (rc) return rc;
        n_tri += d[i].model == SPINMC_ISING_TRI;
        n_hc += d[i].model == SPINMC_ISING_HC;
        n_msc += d[i].model == SPINMC_ISING_MSC;
    }
    if (n_msc > 0 && n_msc < n)
        return fail(SPINMC_E_UNSUPPORTED, "create: multispin-coded groups need a context of their own");
    if (n_msc == n) {
        if ((int64_t)n * 32 > (1 << 30)) return fail(SPINMC_E_INVALID, "create: too many groups");
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
            return fail(SPINMC_E_DEVICE, "create: no HIP device available");
        return create_msc(d, n, seed, init, hip_stream, out);
    }
    if ((n_tri > 0 && n_tri < n) || (n_hc > 0 && n_hc < n))
        return fail(SPINMC_E_UNSUPPORTED, "create: triangular and chain / cubic replicas need a "
                                          "context of their own model");
    if (n_hc == n) {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
            return fail(SPINMC_E_DEVICE, "create: no HIP device available");
        return create_tri(d, n, seed, init, hip_stream, out);
    }
    if (n_tri == n) {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
            return fail(SPINMC_E_DEVICE, "create: no HIP device available");
        return create_tri(d, n, seed, init, hip_stream, out);
    }
    if (cpm_seen && lat_seen)
        return fail(SPINMC_E_UNSUPPORTED, "create: CPM replicas cannot share a context with Ising/Potts");
    if (cpm_seen) {
        for (int i = 1; i < n; ++i)
            if ((d[i].cpm_range == 2) != (d[0].cpm_range == 2))
                return fail(SPINMC_E_INVALID,
                            "create: the CPM replicas of one context must share cpm_range");
        int rc = cpm_prepare_tables(d, n);
        if (rc) return rc;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(SPINMC_E_DEVICE, "create: no HIP device available");
    if (cpm_seen) return create_cpm(d, n, seed, hip_stream, out);
    spinmc_ctx* c = new spinmc_ctx();
    hipGetDevice(&c->device);
    {
        // set-up of spinmc_grad_noalloc's per-device scratch address (the
        // entry point resolves it itself if this fails)
        long long* part = nullptr;
        if (cov_scratch(c->device, &part) != hipSuccess) (void)hipGetLastError();
    }
    c->stream = (hipStream_t)hip_stream;
    c->seed = seed;
    c->R = n;
    c->width = 8;
    c->reps.resize(n);
    size_t lat_off = 0, tab_off = 0, hist_off = 0;
    for (int i = 0; i < n; ++i) {
        HostRep& h = c->reps[i];
        h.d = d[i];
        h.d.adhesion = nullptr;
        h.d.cell_type = nullptr;
        h.d.target_area = nullptr;
        RepDev& r = h.dev;
        r.model = d[i].model;
        r.Lx = d[i].Lx;
        r.Ly = d[i].Ly;
        r.W = d[i].Lx / 2;
        r.q = d[i].model == SPINMC_POTTS ? d[i].q : 2;
        r.rid = d[i].rid;
        r.Jx = d[i].Jx;
        r.Jy = d[i].Jy;
        r.h = d[i].h;
        r.beta = d[i].beta;
        if (r.model == SPINMC_ISING)
            ising_thresholds(d[i].Jx, d[i].Jy, d[i].h, d[i].beta, h.T);
        else
            potts_thresholds(d[i].q, d[i].Jx, d[i].h, d[i].beta, h.T);
        r.tab_n = (int)h.T.size();
        r.tab_off = (int)tab_off;
        tab_off += 2 * h.T.size();
        c->max_tab_n = std::max(c->max_tab_n, r.tab_n);
        h.lat_bytes = (size_t)r.Lx * r.Ly;
        r.lat_off = (int64_t)lat_off;
        lat_off = align_up(lat_off + h.lat_bytes, kAlign);
        r.hist_off = (int)hist_off;
        if (r.model == SPINMC_POTTS) hist_off += (size_t)r.q;
        h.chunk = (r.W % 16) == 0;
        h.resident = h.lat_bytes <= (size_t)kResidentMaxBytes;
        if (!h.chunk && !h.resident) {
            delete c;
            return fail(SPINMC_E_UNSUPPORTED,
                        "replica %d: Lx/2 must be a multiple of 16 for lattices above %d sites", i,
                        kResidentMaxBytes);
        }
        c->max_sites = std::max(c->max_sites, r.Lx * r.Ly);
        c->all_list.push_back(i);
        if (r.model == SPINMC_POTTS) c->potts_list.push_back(i);
    }
    c->lat_bytes = lat_off + 64;
    // host threshold words: hi16 | lo16 halves
    std::vector<uint32_t> tab(std::max<size_t>(tab_off, 1));
    for (int i = 0; i < n; ++i) {
        const HostRep& h = c->reps[i];
        for (int k = 0; k < h.dev.tab_n; ++k) {
            tab[h.dev.tab_off + k] = (uint32_t)(h.T[k] >> 16);
            tab[h.dev.tab_off + h.dev.tab_n + k] = (uint32_t)(h.T[k] & 0xFFFFu);
        }
    }
    std::vector<RepDev> rd(n);
    for (int i = 0; i < n; ++i) rd[i] = c->reps[i].dev;
    auto A = [&](void** p, size_t b) { return hipMalloc(p, std::max<size_t>(b, 16)); };
    hipError_t e = hipSuccess;
    if ((e = A((void**)&c->d_lat, c->lat_bytes)) != hipSuccess ||
        (e = A((void**)&c->d_reps, sizeof(RepDev) * n)) != hipSuccess ||
        (e = A((void**)&c->d_tab, sizeof(uint32_t) * tab.size())) != hipSuccess ||
        (e = A((void**)&c->d_t, 2 * sizeof(uint64_t))) != hipSuccess ||
        (e = A((void**)&c->d_hist, sizeof(int32_t) * std::max<size_t>(hist_off, 1))) != hipSuccess ||
        (e = A((void**)&c->d_lists, sizeof(int32_t) * 5 * n)) != hipSuccess) {
        free_all(c);
        delete c;
        hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? SPINMC_E_NOMEM : SPINMC_E_DEVICE,
                    "create: device allocation failed: %s", hipGetErrorString(e));
    }
    std::vector<int32_t> lists(5 * (size_t)n, 0);
    c->off_all = 0;
    c->off_potts = n;
    c->off_res_chunk = 2 * n;
    c->off_rest = 4 * n;
    std::copy(c->all_list.begin(), c->all_list.end(), lists.begin() + c->off_all);
    std::copy(c->potts_list.begin(), c->potts_list.end(), lists.begin() + c->off_potts);
    const uint64_t zero = 0;
    if ((e = hipMemcpy(c->d_reps, rd.data(), sizeof(RepDev) * n, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(c->d_tab, tab.data(), sizeof(uint32_t) * tab.size(),
                       hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(c->d_t, &zero, sizeof zero, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(c->d_lists, lists.data(), sizeof(int32_t) * lists.size(),
                       hipMemcpyHostToDevice)) ||
        (e = hipMemset(c->d_hist, 0, sizeof(int32_t) * std::max<size_t>(hist_off, 1))) ||
        (e = hipMemset(c->d_lat, 0, c->lat_bytes))) {
        free_all(c);
        delete c;
        return fail(SPINMC_E_DEVICE, "create: upload failed: %s", hipGetErrorString(e));
    }
    if (init == 1) {
        e = launch_init(c->d_reps, c->d_lists + c->off_all, n, c->d_lat,
                        (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32), 256, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            free_all(c);
            delete c;
            return fail(SPINMC_E_DEVICE, "create: init kernel failed: %s", hipGetErrorString(e));
        }
    }
    *out = c;
    return SPINMC_OK;
}

int spinmc_destroy(spinmc_ctx* c) {
    if (!c) return SPINMC_OK;
    if (!c->poisoned) hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
    return SPINMC_OK;
}

int spinmc_num_replicas(const spinmc_ctx* c) { return c ? c->R : SPINMC_E_INVALID; }
int spinmc_stats_width(const spinmc_ctx* c) { return c ? c->width : SPINMC_E_INVALID; }

int spinmc_sweep_counter(const spinmc_ctx* c, uint64_t* t) {
    if (!c || !t) return fail(SPINMC_E_INVALID, "sweep_counter: null argument");
    *t = c->t;
    return SPINMC_OK;
}

// Multispin-coded words between the natural order y Lx + x (host buffers)
// and the device's colour planes (site (y, x) at word (y, x >> 1) of plane
// (x + y) & 1, planes of Ly rows by Lx / 2 words).
static void msc_permute(int Lx, int Ly, const uint32_t* src, uint32_t* dst, bool to_planes) {
    const size_t W = (size_t)Lx / 2;
    for (int y = 0; y < Ly; ++y)
        for (int x = 0; x < Lx; ++x) {
            const size_t nat = (size_t)y * Lx + x;
            const size_t pl = (size_t)((x + y) & 1) * Ly * W + (size_t)y * W + (x >> 1);
            if (to_planes)
                dst[pl] = src[nat];
            else
                dst[nat] = src[pl];
        }
}

int spinmc_set_state(spinmc_ctx* c, int32_t r, const void* host, size_t bytes) {
    if (!c || !host) return fail(SPINMC_E_INVALID, "set_state: null argument");
    if (c->poisoned) return fail(SPINMC_E_DEVICE, "set_state: context poisoned");
    if (r < 0 || r >= c->R) return fail(SPINMC_E_INVALID, "set_state: replica out of range");
    if (c->cpm) return cpm_set_state(c, r, host, bytes);
    if (c->msc) {
        if (r >= (int)c->reps.size()) return fail(SPINMC_E_INVALID, "set_state: group out of range");
        const HostRep& h = c->reps[r];
        if (bytes != h.lat_bytes) return fail(SPINMC_E_INVALID, "set_state: wrong byte count");
        std::vector<uint32_t> planes((size_t)h.dev.Lx * h.dev.Ly);
        msc_permute(h.dev.Lx, h.dev.Ly, (const uint32_t*)host, planes.data(), true);
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess)
            e = hipMemcpy(c->d_lat + h.dev.lat_off, planes.data(), bytes, hipMemcpyHostToDevice);
        return check_dev(c, e, "set_state");
    }
    if (c->tri) return tri_set_state(c, r, host, bytes);
    const HostRep& h = c->reps[r];
    const int Lx = h.dev.Lx, Ly = h.dev.Ly, W = h.dev.W;
    if (bytes != (size_t)Lx * Ly) return fail(SPINMC_E_INVALID, "set_state: wrong byte count");
    const uint8_t* src = (const uint8_t*)host;
    std::vector<uint8_t> planes((size_t)Lx * Ly);
    for (int y = 0; y < Ly; ++y)
        for (int x = 0; x < Lx; ++x) {
            const int8_t v = (int8_t)src[(size_t)y * Lx + x];
            uint8_t u;
            if (h.dev.model == SPINMC_ISING) {
                if (v != 1 && v != -1)
                    return fail(SPINMC_E_INVALID, "set_state: Ising spins must be +-1");
                u = v > 0 ? 1 : 0;
            } else {
                u = (uint8_t)v;
                if ((int)u >= h.dev.q)
                    return fail(SPINMC_E_INVALID, "set_state: Potts label out of range");
            }
            planes[(size_t)((x + y) & 1) * Ly * W + (size_t)y * W + (x >> 1)] = u;
        }
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess)
        e = hipMemcpy(c->d_lat + h.dev.lat_off, planes.data(), planes.size(), hipMemcpyHostToDevice);
    return check_dev(c, e, "set_state");
}

int spinmc_get_state(spinmc_ctx* c, int32_t r, void* host, size_t bytes) {
    if (!c || !host) return fail(SPINMC_E_INVALID, "get_state: null argument");
    if (c->poisoned) return fail(SPINMC_E_DEVICE, "get_state: context poisoned");
    if (r < 0 || r >= c->R) return fail(SPINMC_E_INVALID, "get_state: replica out of range");
    if (c->cpm) return cpm_get_state(c, r, host, bytes);
    if (c->msc) {
        if (r >= (int)c->reps.size()) return fail(SPINMC_E_INVALID, "get_state: group out of range");
        const HostRep& h = c->reps[r];
        if (bytes != h.lat_bytes) return fail(SPINMC_E_INVALID, "get_state: wrong byte count");
        std::vector<uint32_t> planes((size_t)h.dev.Lx * h.dev.Ly);
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess)
            e = hipMemcpy(planes.data(), c->d_lat + h.dev.lat_off, bytes, hipMemcpyDeviceToHost);
        if (e == hipSuccess) msc_permute(h.dev.Lx, h.dev.Ly, planes.data(), (uint32_t*)host, false);
        return check_dev(c, e, "get_state");
    }
    if (c->tri) return tri_get_state(c, r, host, bytes);
    const HostRep& h = c->reps[r];
    const int Lx = h.dev.Lx, Ly = h.dev.Ly, W = h.dev.W;
    if (bytes != (size_t)Lx * Ly) return fail(SPINMC_E_INVALID, "get_state: wrong byte count");
    if (int rc = persist_check(c)) return rc;
    std::vector<uint8_t> planes((size_t)Lx * Ly);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess)
        e = hipMemcpy(planes.data(), c->d_lat + h.dev.lat_off, planes.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return check_dev(c, e, "get_state");
    uint8_t* dst = (uint8_t*)host;
    for (int y = 0; y < Ly; ++y)
        for (int x = 0; x < Lx; ++x) {
            const uint8_t u = planes[(size_t)((x + y) & 1) * Ly * W + (size_t)y * W + (x >> 1)];
            dst[(size_t)y * Lx + x] =
                h.dev.model == SPINMC_ISING ? (uint8_t)(int8_t)(u ? 1 : -1) : u;
        }
    return SPINMC_OK;
}

int spinmc_thresholds(const spinmc_ctx* c, int32_t r, uint64_t* T, int32_t cap, int32_t* n_out,
                      int64_t* aux) {
    if (!c || !n_out) return fail(SPINMC_E_INVALID, "thresholds: null argument");
    if (r < 0 || r >= (int)c->reps.size())
        return fail(SPINMC_E_INVALID, "thresholds: replica out of range");
    const HostRep& h = c->reps[r];
    *n_out = (int32_t)h.T.size();
    if (aux) *aux = h.aux;
    if (T) {
        if (cap < (int32_t)h.T.size()) return fail(SPINMC_E_INVALID, "thresholds: capacity");
        std::copy(h.T.begin(), h.T.end(), T);
    }
    return SPINMC_OK;
}

int spinmc_schedule_sites(const spinmc_ctx* c, int64_t streamed[3], int64_t resident[3]) {
    if (!c || !streamed || !resident) return fail(SPINMC_E_INVALID, "schedule_sites: null argument");
    for (int m = 0; m < 3; ++m) streamed[m] = resident[m] = 0;
    if (c->cpm) {
        for (const HostRep& h : c->reps) streamed[kModelCpm] += (int64_t)h.dev.Lx * h.dev.Ly;
    } else if (c->msc) {  // 32 replicas per site, counted with the Ising lattices
        for (const HostRep& h : c->reps) streamed[kModelIsing] += 32 * (int64_t)h.dev.Lx * h.dev.Ly;
    } else if (c->tri) {  // counted with the Ising lattices
        for (const HostRep& h : c->reps) streamed[kModelIsing] += (int64_t)h.lat_bytes;
    } else {
        const int mode = effective_mode(c);
        for (const HostRep& h : c->reps) {
            const bool res = (mode == 1) || !h.chunk || (mode == 3 && h.resident);
            (res ? resident : streamed)[h.dev.model] += (int64_t)h.dev.Lx * h.dev.Ly;
        }
    }
    return SPINMC_OK;
}

int spinmc_get_schedule(const spinmc_ctx* c, spinmc_schedule* s) {
    if (!c || !s) return fail(SPINMC_E_INVALID, "get_schedule: null argument");
    *s = c->sched;
    return SPINMC_OK;
}

int spinmc_set_schedule(spinmc_ctx* c, const spinmc_schedule* s) {
    if (!c || !s) return fail(SPINMC_E_INVALID, "set_schedule: null argument");
    if (s->mode < 0 || s->mode > 3)
        return fail(SPINMC_E_INVALID, "set_schedule: mode %d not available", s->mode);
    if (s->tile_rows < 0 || (s->tile_rows & 1))
        return fail(SPINMC_E_INVALID, "set_schedule: tile_rows must be even and >= 0");
    if (s->wg_threads != 0 && s->wg_threads != 256 && s->wg_threads != 512)
        return fail(SPINMC_E_INVALID, "set_schedule: wg_threads must be 256 or 512");
    if (s->rpb != 0 && s->rpb != 1 && s->rpb != 2 && s->rpb != 4 && s->rpb != 8)
        return fail(SPINMC_E_INVALID, "set_schedule: rpb must be 0, 1, 2, 4 or 8");
    if ((s->flags & ~(SPINMC_SCHED_NT_ON | SPINMC_SCHED_NT_OFF | SPINMC_SCHED_PERSIST)) != 0 ||
        (s->flags & (SPINMC_SCHED_NT_ON | SPINMC_SCHED_NT_OFF)) ==
            (SPINMC_SCHED_NT_ON | SPINMC_SCHED_NT_OFF))
        return fail(SPINMC_E_INVALID,
                    "set_schedule: flags must be 0, NT_ON or NT_OFF, optionally with PERSIST");
    if ((s->flags & SPINMC_SCHED_PERSIST) && (c->tri || c->msc || (c->cpm && c->cpm_range != 1)))
        return fail(SPINMC_E_UNSUPPORTED,
                    "set_schedule: persistent passes serve square-lattice Ising, Potts and the "
                    "3x3 CPM only");
    if (s->mode == 1 && !c->cpm)
        for (const HostRep& h : c->reps)
            if (!h.resident)
                return fail(SPINMC_E_INVALID, "set_schedule: a lattice exceeds the resident LDS budget");
    c->sched = *s;
    c->prepared = false;  // new tiles, resident lists and graphs on the next sweep
    return SPINMC_OK;
}

int spinmc_sweep(spinmc_ctx* c, int32_t n, int32_t re, void* dev_stats) {
    if (!c) return fail(SPINMC_E_INVALID, "sweep: null context");
    if (c->poisoned) return fail(SPINMC_E_DEVICE, "sweep: context poisoned");
    if (n < 0 || re < 0) return fail(SPINMC_E_INVALID, "sweep: negative count");
    if (re > 0 && !dev_stats) return fail(SPINMC_E_INVALID, "sweep: recording needs dev_stats");
    // Philox counter word 1 carries the pass p = n_col t + c: every pass of
    // the call must fit 32 bits, i.e. (t + n) n_col <= 2^32, or later passes
    // would reuse the random words of earlier ones.
    const uint64_t n_col = c->cpm ? (c->cpm_range == 2 ? 9u : 4u)
                           : (c->tri && !c->reps.empty() &&
                              c->reps[0].d.model == SPINMC_ISING_TRI) ? 3u : 2u;
    if (((uint64_t)c->t + (uint64_t)n) * n_col > ((uint64_t)1 << 32))
        return fail(SPINMC_E_INVALID, "sweep: pass counter %llu (t + n) x %llu colours exceeds 2^32",
                    (unsigned long long)(c->t + (uint64_t)n), (unsigned long long)n_col);
    if (n == 0) return SPINMC_OK;
    int rc = c->cpm   ? cpm_sweep(c, n, re, (int32_t*)dev_stats)
             : c->msc ? msc_sweep(c, n, re, (int32_t*)dev_stats)
             : c->tri ? tri_sweep(c, n, re, (int32_t*)dev_stats)
                      : enqueue_sweep(c, n, re, (int32_t*)dev_stats);
    if (rc == SPINMC_OK) c->t += (uint64_t)n;
    return rc;
}

int spinmc_measure(spinmc_ctx* c, void* dev_stats, void* dev_obs) {
    if (!c || !dev_stats) return fail(SPINMC_E_INVALID, "measure: null argument");
    if (c->poisoned) return fail(SPINMC_E_DEVICE, "measure: context poisoned");
    int32_t* st = (int32_t*)dev_stats;
    if (c->cpm) return cpm_measure(c, st, (double*)dev_obs);
    if (c->msc) return msc_measure(c, st, (double*)dev_obs);
    if (c->tri) return tri_measure(c, st, (double*)dev_obs);
    hipError_t e = launch_fill_i32(st, (size_t)c->R * c->width, 0, c->stream);
    SweepArgs a{};
    a.reps = c->d_reps;
    a.stats = st;
    a.hist = c->d_hist;
    a.R = c->R;
    a.width = c->width;
    if (e == hipSuccess)
        e = launch_measure(c->d_reps, c->d_lists + c->off_all, c->R, c->max_sites, c->d_lat, st,
                           c->d_hist, c->width, c->stream);
    if (e == hipSuccess && !c->potts_list.empty())
        e = launch_potts_hist_finalize(a, c->d_lists + c->off_potts, (int)c->potts_list.size(), 0,
                                       c->stream);
    if (e == hipSuccess && dev_obs)
        e = launch_observables(c->d_reps, c->R, st, c->width, (double*)dev_obs, c->stream);
    return check_dev(c, e, "measure");
}

}  // extern "C"

namespace {

// Argument checks shared by spinmc_grad and spinmc_grad_noalloc.
int grad_check(spinmc_ctx* c, const void* dev_stats, int32_t n_rec, int32_t burn_in,
               const void* gout, void* dtheta, const char* who) {
    if (!c || !dev_stats) return fail(SPINMC_E_INVALID, "%s: null argument", who);
    if (c->poisoned) return fail(SPINMC_E_DEVICE, "%s: context poisoned", who);
    for (const HostRep& h : c->reps)
        if (h.dev.model != SPINMC_ISING) return fail(SPINMC_E_UNSUPPORTED, "%s: Ising contexts only", who);
    if (n_rec < 1 || burn_in < 0 || burn_in >= n_rec)
        return fail(SPINMC_E_INVALID, "%s: need 0 <= burn_in < n_rec", who);
    if (dtheta && !gout) return fail(SPINMC_E_INVALID, "%s: dtheta needs grad_out", who);
    const int n = n_rec - burn_in;
    // The moment sums are exact int64: |M|, |Bx|, |By| <= N (sites per
    // lattice) bound every product by N^2 and a sum over n samples by n N^2.
    for (const HostRep& h : c->reps) {
        const unsigned __int128 N = (unsigned __int128)h.dev.Lx * (unsigned)h.dev.Ly;
        if ((unsigned __int128)n * N * N >= ((unsigned __int128)1 << 63))
            return fail(SPINMC_E_INVALID,
                        "%s: %d samples of a %d x %d lattice overflow the int64 moment sums", who,
                        n, h.dev.Lx, h.dev.Ly);
    }
    return SPINMC_OK;
}

}  // namespace

extern "C" {

int spinmc_grad(spinmc_ctx* c, const void* dev_stats, int32_t n_rec, int32_t burn_in,
                const void* gout, void* means, void* grads, void* dtheta) {
    int rc = grad_check(c, dev_stats, n_rec, burn_in, gout, dtheta, "grad");
    if (rc) return rc;
    const int n = n_rec - burn_in;
    const bool split = n >= kCovSplitMin && (n + kCovChunk - 1) / kCovChunk <= 65535;
    hipError_t e = hipSuccess;
    if (split) {
        const size_t need = cov_partial_entries(c->R, n);
        if (need > c->cov_part_n) {  // grown on demand; hipFree waits for the device
            hipFree(c->d_cov_part);
            c->d_cov_part = nullptr;
            c->cov_part_n = 0;
            if (hipMalloc((void**)&c->d_cov_part, need * sizeof(long long)) != hipSuccess) {
                (void)hipGetLastError();
                c->d_cov_part = nullptr;
                return fail(SPINMC_E_NOMEM, "grad: %zu bytes of chunk sums", need * sizeof(long long));
            }
            c->cov_part_n = need;
        }
        e = launch_cov_grad_split(c->d_reps, c->R, (const int32_t*)dev_stats, n_rec, burn_in,
                                  c->width, (const double*)gout, (double*)means, (double*)grads,
                                  (double*)dtheta, c->d_cov_part, c->stream);
    } else {
        e = launch_cov_grad(c->d_reps, c->R, (const int32_t*)dev_stats, n_rec, burn_in, c->width,
                            (const double*)gout, (double*)means, (double*)grads, (double*)dtheta,
                            c->stream);
    }
    return check_dev(c, e, "grad");
}

int spinmc_grad_noalloc(spinmc_ctx* c, const void* dev_stats, int32_t n_rec, int32_t burn_in,
                        const void* gout, void* means, void* grads, void* dtheta) {
    int rc = grad_check(c, dev_stats, n_rec, burn_in, gout, dtheta, "grad_noalloc");
    if (rc) return rc;
    const int n = n_rec - burn_in;
    const size_t need = cov_partial_entries(c->R, n);
    if (need > kCovScratchEntries)
        return fail(SPINMC_E_INVALID,
                    "grad_noalloc: %d replicas x %d samples need %zu bytes of chunk sums, above "
                    "the %zu bytes of the static scratch array (use spinmc_grad)",
                    c->R, n, need * sizeof(long long), kCovScratchEntries * sizeof(long long));
    long long* part = nullptr;
    hipError_t e = cov_scratch(c->device, &part);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SPINMC_E_DEVICE, "grad_noalloc: device address of the scratch array on "
                                     "device %d (%s; that device must be current)",
                    c->device, hipGetErrorString(e));
    }
    e = launch_cov_grad_split(c->d_reps, c->R, (const int32_t*)dev_stats, n_rec, burn_in, c->width,
                              (const double*)gout, (double*)means, (double*)grads,
                              (double*)dtheta, part, c->stream);
    return check_dev(c, e, "grad_noalloc");
}

int spinmc_profile(spinmc_ctx* c, int32_t enable) {
    if (!c) return fail(SPINMC_E_INVALID, "profile: null context");
    if (enable) {
        hipStreamSynchronize(c->stream);
        c->prof_recs.clear();
        c->ev_used = 0;
    }
    c->prof = enable != 0;
    return SPINMC_OK;
}

int spinmc_profile_read(spinmc_ctx* c, int32_t kind, double* ms, int64_t* launches) {
    if (!c || !ms || !launches) return fail(SPINMC_E_INVALID, "profile_read: null argument");
    double tot = 0.0;
    int64_t n = 0;
    for (auto& r : c->prof_recs) {
        if (std::get<0>(r) != kind) continue;
        hipError_t e = hipEventSynchronize(std::get<2>(r));
        float m = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&m, std::get<1>(r), std::get<2>(r));
        if (e != hipSuccess) return check_dev(c, e, "profile_read");
        tot += m;
        ++n;
    }
    *ms = tot;
    *launches = n;
    return SPINMC_OK;
}

}  // extern "C"

namespace {

// Per-process cache of autotuned schedules (optionally mirrored in the file
// named by SPINMC_AUTOTUNE_CACHE), keyed by device architecture, compute-unit
// count and the context's shape signature.
std::mutex g_tune_mu;
std::map<std::string, spinmc_schedule> g_tune;
bool g_tune_loaded = false;

std::string tune_key(const spinmc_ctx* c, int mode_filter) {
    std::ostringstream k;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess)
        k << prop.gcnArchName << "/" << prop.multiProcessorCount;
    else
        k << "?";
    k << "|m" << mode_filter << "|";
    std::map<std::tuple<int, int, int, int, int, int>, int> shapes;
    for (const HostRep& h : c->reps)
        ++shapes[std::make_tuple(h.d.model, h.d.Lx, h.d.Ly, h.d.model == SPINMC_ISING ? 2 : h.d.q,
                                 h.d.Lz, c->cpm ? c->cpm_range : 0)];
    for (const auto& kv : shapes)
        k << std::get<0>(kv.first) << "," << std::get<1>(kv.first) << "," << std::get<2>(kv.first)
          << "," << std::get<3>(kv.first) << "," << std::get<4>(kv.first) << ","
          << std::get<5>(kv.first) << "*" << kv.second << ";";
    return k.str();
}

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = std::getenv("SPINMC_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t tab = line.find('\t');
        if (tab == std::string::npos) continue;
        std::istringstream v(line.substr(tab + 1));
        spinmc_schedule sc{};
        if (v >> sc.mode >> sc.tile_rows >> sc.wg_threads >> sc.flags >> sc.rpb)
            g_tune[line.substr(0, tab)] = sc;
    }
}

void tune_store(const std::string& key, const spinmc_schedule& sc) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_load_locked();
    g_tune[key] = sc;
    const char* path = std::getenv("SPINMC_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    std::ofstream f(path, std::ios::app);
    if (f) f << key << '\t' << sc.mode << ' ' << sc.tile_rows << ' ' << sc.wg_threads << ' '
             << sc.flags << ' ' << sc.rpb << '\n';
}

}  // namespace

extern "C" {

int spinmc_autotune(spinmc_ctx* c, int32_t trial_sweeps, spinmc_schedule* chosen, double* rates,
                    int32_t cap, int32_t* n_tried) {
    if (!c) return fail(SPINMC_E_INVALID, "autotune: null context");
    if (c->poisoned) return fail(SPINMC_E_DEVICE, "autotune: context poisoned");
    if (trial_sweeps < 1) return fail(SPINMC_E_INVALID, "autotune: trial_sweeps must be >= 1");
    if (c->tri || c->msc) {  // one kernel shape: nothing to choose
        if (chosen) *chosen = c->sched;
        if (n_tried) *n_tried = 0;
        return SPINMC_OK;
    }
    const bool use_cache = !(chosen && chosen->mode == -1);
    const int mode_filter = chosen && chosen->mode > 0 ? chosen->mode : 0;
    const std::string key = tune_key(c, mode_filter);
    if (use_cache) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        tune_load_locked();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            c->sched = it->second;
            c->prepared = false;
            if (chosen) *chosen = it->second;
            if (n_tried) *n_tried = 0;
            return SPINMC_OK;
        }
    }
    // candidate schedules
    std::vector<spinmc_schedule> cand;
    if (c->cpm) {
        // resident where the lattices fit (else the default streamed passes),
        // then streamed passes over several tile heights
        cand.push_back(spinmc_schedule{0, 0, 0, 0});
        for (int tr : {0, 2, 4, 8, 16}) cand.push_back(spinmc_schedule{2, tr, 256, 0});
        if (c->cpm_range == 1 && c->cpm_quad) {  // one site per lane
            for (int tr : {0, 8, 32}) cand.push_back(spinmc_schedule{2, tr, 0, 0});
            for (int tr : {0, 8}) cand.push_back(spinmc_schedule{2, tr, 512, 0});
        }
        // tiled persistent passes (where they apply), tiles of 64 and 32 rows
        int TH = 0, TW = 0, nb = 0;
        if (cpm_tiled_plan(c, &TH, &TW, &nb))
            for (int tr : {0, 32}) cand.push_back(spinmc_schedule{2, tr, 256, SPINMC_SCHED_PERSIST});
    } else {
        bool all_res = true, any_res_chunk = false, any_stream = false;
        int min_def = 1 << 30;
        for (const HostRep& h : c->reps) {
            all_res = all_res && h.resident;
            any_res_chunk = any_res_chunk || (h.resident && h.chunk);
            any_stream = any_stream || h.chunk;
            if (h.chunk) min_def = std::min(min_def, default_tile_rows(h));
        }
        if (all_res)
            for (int th : {256, 512}) cand.push_back(spinmc_schedule{1, 0, th, 0});
        if (any_stream) {
            std::vector<int> trs = {0};
            if (min_def >= 8) trs.push_back(std::max(2, (min_def / 2) & ~1));
            trs.push_back(min_def * 2);
            for (int mode : {2, 3}) {
                if (mode == 3 && !any_res_chunk) continue;
                for (int tr : trs)
                    for (int th : {256, 512}) cand.push_back(spinmc_schedule{mode, tr, th, 0});
                // persistent passes: slabs sized by the chip's occupancy, and
                // slabs of four default tiles
                cand.push_back(spinmc_schedule{mode, 0, 256, SPINMC_SCHED_PERSIST});
                cand.push_back(spinmc_schedule{mode, min_def * 4, 256, SPINMC_SCHED_PERSIST});
            }
        }
    }
    if (mode_filter > 0) {
        std::vector<spinmc_schedule> keep;
        for (const auto& k : cand)
            if (k.mode == mode_filter) keep.push_back(k);
        cand.swap(keep);
    }
    if (cand.empty()) return fail(SPINMC_E_UNSUPPORTED, "autotune: no candidate schedule");
    if (c->cpm) {  // current areas before they are saved
        if (int rc = cpm_recount_if_dirty(c)) return rc;
    }
    const spinmc_schedule saved_sched = c->sched;
    const uint64_t saved_t = c->t;
    // scratch copy of the state (lattices, sweep counter, CPM areas)
    uint8_t* lat_copy = nullptr;
    int32_t* area_copy = nullptr;
    uint64_t dt_saved = 0;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMalloc((void**)&lat_copy, c->lat_bytes);
    if (e == hipSuccess && c->cpm) e = hipMalloc((void**)&area_copy, sizeof(int32_t) * c->total_cells);
    if (e != hipSuccess) {
        hipFree(lat_copy);
        hipGetLastError();
        return fail(SPINMC_E_NOMEM, "autotune: no memory for the state copy");
    }
    e = hipMemcpy(lat_copy, c->d_lat, c->lat_bytes, hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipMemcpy(&dt_saved, c->d_t, sizeof dt_saved, hipMemcpyDeviceToHost);
    if (e == hipSuccess && c->cpm)
        e = hipMemcpy(area_copy, c->d_area, sizeof(int32_t) * c->total_cells,
                      hipMemcpyDeviceToDevice);
    auto restore = [&]() -> hipError_t {
        hipError_t r = hipStreamSynchronize(c->stream);
        if (r == hipSuccess) r = hipMemcpy(c->d_lat, lat_copy, c->lat_bytes, hipMemcpyDeviceToDevice);
        if (r == hipSuccess) r = hipMemcpy(c->d_t, &dt_saved, sizeof dt_saved, hipMemcpyHostToDevice);
        if (r == hipSuccess && c->cpm) {
            r = hipMemcpy(c->d_area, area_copy, sizeof(int32_t) * c->total_cells,
                          hipMemcpyDeviceToDevice);
            if (r == hipSuccess) r = hipMemcpy(c->d_snap, area_copy, sizeof(int32_t) * c->total_cells,
                                               hipMemcpyDeviceToDevice);
        }
        c->t = saved_t;
        return r;
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    double sites = 0;
    for (const HostRep& h : c->reps) sites += (double)h.dev.Lx * h.dev.Ly;
    int best = -1;
    double best_rate = 0;
    int tried = 0;
    // one timed run of trial_sweeps * mult sweeps under schedule sc (after a
    // warm-up that builds tiles and graphs), the state restored after it;
    // recorded in rates for the first round of candidates
    auto timed_run = [&](const spinmc_schedule& sc, int mult, bool record) -> double {
        const int n = trial_sweeps * mult;
        c->sched = sc;
        c->prepared = false;
        int rc = c->cpm ? cpm_sweep(c, 1, 0, nullptr) : enqueue_sweep(c, 1, 0, nullptr);
        if (rc == SPINMC_OK) rc = c->cpm ? cpm_sweep(c, n, 0, nullptr)
                                         : enqueue_sweep(c, n, 0, nullptr);
        if (rc != SPINMC_OK) {
            e = hipErrorUnknown;
            return 0.0;
        }
        e = restore();
        if (e != hipSuccess) return 0.0;
        e = hipEventRecord(e0, c->stream);
        rc = c->cpm ? cpm_sweep(c, n, 0, nullptr) : enqueue_sweep(c, n, 0, nullptr);
        if (rc != SPINMC_OK) {
            e = hipErrorUnknown;
            return 0.0;
        }
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        const double rate = ms > 0 ? sites * n / (ms * 1e6) : 0.0;
        if (record) {
            if (rates && tried < cap) rates[tried] = rate;
            ++tried;
        }
        if (e == hipSuccess) e = restore();
        return rate;
    };
    std::vector<double> cand_rate;
    auto trial = [&](const spinmc_schedule& sc) -> double {
        const double r = timed_run(sc, 1, true);
        cand_rate.push_back(r);
        return r;
    };
    for (size_t k = 0; k < cand.size() && e == hipSuccess; ++k) {
        const double rate = trial(cand[k]);
        if (e == hipSuccess && rate > best_rate) {
            best_rate = rate;
            best = (int)k;
        }
    }
    // the best streaming schedule with nontemporal own-plane access forced
    // on and off (candidates so far use the size rule)
    if (e == hipSuccess && best >= 0 && !c->cpm && cand[best].mode >= 2) {
        const size_t nb = cand.size();
        for (int f : {SPINMC_SCHED_NT_ON, SPINMC_SCHED_NT_OFF}) {
            spinmc_schedule sc = cand[best];
            sc.flags = (sc.flags & SPINMC_SCHED_PERSIST) | f;
            cand.push_back(sc);
        }
        for (size_t k = nb; k < cand.size() && e == hipSuccess; ++k) {
            const double rate = trial(cand[k]);
            if (e == hipSuccess && rate > best_rate) {
                best_rate = rate;
                best = (int)k;
            }
        }
    }
    // replicas per resident workgroup for the best candidate with resident
    // groups (the packing rule's choice is the baseline already measured)
    if (e == hipSuccess && best >= 0 && !c->cpm && cand[best].mode != 2 && cand[best].rpb == 0) {
        bool any_res = false;
        for (const HostRep& h : c->reps) any_res = any_res || h.resident;
        if (any_res) {
            const size_t nb = cand.size();
            for (int r : {1, 2, 4, 8}) {
                spinmc_schedule sc = cand[best];
                sc.rpb = r;
                cand.push_back(sc);
            }
            for (size_t k = nb; k < cand.size() && e == hipSuccess; ++k) {
                const double rate = trial(cand[k]);
                if (e == hipSuccess && rate > best_rate) {
                    best_rate = rate;
                    best = (int)k;
                }
            }
        }
    }
    // run-off: short trials of close candidates differ by noise, so the three
    // fastest run again four times as long, twice each, and the best of
    // those runs decides (not recorded in rates)
    if (e == hipSuccess && cand.size() > 1 && cand_rate.size() == cand.size()) {
        std::vector<int> order(cand.size());
        for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
        std::sort(order.begin(), order.end(),
                  [&](int x, int y) { return cand_rate[x] > cand_rate[y]; });
        double run_best = 0;
        for (int k = 0; k < 3 && k < (int)order.size() && e == hipSuccess; ++k) {
            for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
                const double r = timed_run(cand[order[k]], 4, false);
                if (e == hipSuccess && r > run_best) {
                    run_best = r;
                    best = order[k];
                }
            }
        }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (e == hipSuccess && persist_check(c) != SPINMC_OK) {
        hipFree(lat_copy);
        hipFree(area_copy);
        return SPINMC_E_DEVICE;
    }
    hipError_t er = restore();
    hipFree(lat_copy);
    hipFree(area_copy);
    if (e != hipSuccess || er != hipSuccess || best < 0) {
        c->sched = saved_sched;
        c->prepared = false;
        if (c->poisoned) return SPINMC_E_DEVICE;
        return check_dev(c, e != hipSuccess ? e : er, "autotune");
    }
    c->sched = cand[best];
    c->prepared = false;
    tune_store(key, cand[best]);
    if (chosen) *chosen = cand[best];
    if (n_tried) *n_tried = tried;
    return SPINMC_OK;
}

}  // extern "C"

namespace {

// Resolve mode 0: everything resident when every lattice fits the LDS
// budget, else the hybrid (resident where it fits, streamed otherwise).
int effective_mode(const spinmc_ctx* c) {
    if (c->sched.mode != 0) return c->sched.mode;
    for (const HostRep& h : c->reps)
        if (!h.resident) return 3;
    return 1;
}

int default_tile_rows(const HostRep& h) {
    // ~16 KiB of one plane per unit
    int rows = std::max(2, 16384 / std::max(1, h.dev.W));
    rows &= ~1;
    return std::min(rows, h.dev.Ly);
}

void drop_graphs(spinmc_ctx* c) {
    for (auto& kv : c->graphs) hipGraphExecDestroy(kv.second);
    c->graphs.clear();
}

// Work items of the persistent streamed passes of one model.  Replicas are
// cut into row slabs of about `target` sites (tile_rows rows when the
// schedule names a height); a replica of one slab is a whole item, and whole
// items are packed longest first into bins of about `target` sites (at most
// items_cap per bin); each slab gets a workgroup of its own.  The slab
// workgroups come first and, since they wait on one another, their number
// stays within the occupancy of the chip (cap): otherwise the slabs grow.
int plan_model(const spinmc_ctx* c, const std::vector<int>& reps, int tile_rows, int cap,
               int items_cap, int flag0, std::vector<PersistItem>& items,
               std::vector<int32_t>& wg_items, int* n_slabs_out) {
    double total = 0;
    int max_ly = 2;
    for (int i : reps) {
        total += (double)c->reps[i].dev.Lx * c->reps[i].dev.Ly;
        max_ly = std::max(max_ly, c->reps[i].dev.Ly);
    }
    double target = std::max(1.0, total / std::max(cap, 1));
    int rows_fixed = tile_rows;
    for (int attempt = 0; attempt < 64; ++attempt) {
        items.clear();
        wg_items.clear();
        std::vector<std::pair<double, int>> whole;  // (sites, replica)
        int n_slabs = 0;
        for (int i : reps) {
            const RepDev& d = c->reps[i].dev;
            int rows;
            if (rows_fixed > 0) {
                rows = std::min(rows_fixed, d.Ly);
            } else {
                const int S = std::max(1, (int)std::ceil((double)d.Lx * d.Ly / target - 1e-9));
                rows = std::min(d.Ly, ((d.Ly + S - 1) / S + 1) & ~1);
            }
            const int S = (d.Ly + rows - 1) / rows;
            if (S == 1) {
                whole.push_back({(double)d.Lx * d.Ly, i});
                continue;
            }
            const int f0 = flag0 + n_slabs;
            for (int k = 0; k < S; ++k) {
                const int y0 = k * rows;
                PersistItem it{};
                it.rep = i;
                it.y0 = y0;
                it.rows = std::min(rows, d.Ly - y0);
                it.slab = f0 + k;
                it.up = f0 + (k + S - 1) % S;
                it.down = f0 + (k + 1) % S;
                items.push_back(it);
                wg_items.push_back(1);
            }
            n_slabs += S;
        }
        if (n_slabs > cap) {
            // too many slab workgroups to be resident together: larger slabs
            if (rows_fixed > 0) {
                if (rows_fixed >= max_ly) return fail(SPINMC_E_UNSUPPORTED, "persistent plan");
                rows_fixed = std::min(max_ly, rows_fixed * 2);
            } else {
                target *= 1.25;
            }
            continue;
        }
        if (!whole.empty()) {
            std::sort(whole.begin(), whole.end(),
                      [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
                          return a.first > b.first || (a.first == b.first && a.second < b.second);
                      });
            double wsum = 0;
            for (const auto& w : whole) wsum += w.first;
            const double bin_target = std::max(target, whole[0].first);
            int n_bins = (int)std::ceil(wsum / bin_target - 1e-9);
            n_bins = std::max(n_bins, ((int)whole.size() + items_cap - 1) / items_cap);
            n_bins = std::max(1, std::min(n_bins, (int)whole.size()));
            std::vector<double> load(n_bins, 0.0);
            std::vector<std::vector<int>> bin(n_bins);
            for (const auto& w : whole) {
                int best = -1;
                for (int b = 0; b < n_bins; ++b)
                    if ((int)bin[b].size() < items_cap && (best < 0 || load[b] < load[best])) best = b;
                bin[best].push_back(w.second);
                load[best] += w.first;
            }
            for (int b = 0; b < n_bins; ++b) {
                std::sort(bin[b].begin(), bin[b].end());
                for (int i : bin[b]) {
                    PersistItem it{};
                    it.rep = i;
                    it.y0 = 0;
                    it.rows = c->reps[i].dev.Ly;
                    it.slab = it.up = it.down = -1;
                    items.push_back(it);
                }
                wg_items.push_back((int)bin[b].size());
            }
        }
        *n_slabs_out = n_slabs;
        return SPINMC_OK;
    }
    return fail(SPINMC_E_UNSUPPORTED, "persistent plan: no slab size fits the chip");
}

int plan_persist(spinmc_ctx* c, int mode) {
    std::vector<int> by_model[2];
    for (int i = 0; i < c->R; ++i) {
        const HostRep& h = c->reps[i];
        const bool resident = (mode == 1) || !h.chunk || (mode == 3 && h.resident);
        if (!resident) by_model[h.dev.model == SPINMC_ISING ? 0 : 1].push_back(i);
    }
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess ||
        n_cu < 1)
        return fail(SPINMC_E_DEVICE, "persistent plan: compute-unit count");
    std::vector<PersistItem> all_items;
    std::vector<int32_t> offs{0};
    int n_flags = 0;
    size_t lds_max = 0;
    for (int m = 0; m < 2; ++m) {
        auto& P = c->pplan[m];
        P = spinmc_ctx::PersistPlan{};
        if (by_model[m].empty()) continue;
        P.slot_words = (int)align_up((size_t)2 * c->max_tab_n + 18, 4);
        const int items_cap = std::max(1, std::min(16, 8192 / (4 * P.slot_words)));
        P.lds = (size_t)items_cap * P.slot_words * 4;
        const bool nt = m == 0 ? c->nt_ising : c->nt_potts;
        int per_cu = 0;
        if (persist_occupancy(m == 0 ? kModelIsing : kModelPotts, nt, P.lds, &per_cu) != hipSuccess ||
            per_cu < 1) {
            (void)hipGetLastError();
            return fail(SPINMC_E_DEVICE, "persistent plan: occupancy query");
        }
        std::vector<PersistItem> items;
        std::vector<int32_t> wg_items;
        int rc = plan_model(c, by_model[m], c->sched.tile_rows, per_cu * n_cu, items_cap, n_flags,
                            items, wg_items, &P.n_slabs);
        if (rc) return rc;
        P.n_wg = (int)wg_items.size();
        P.off0 = (int)offs.size() - 1;
        const int base = (int)all_items.size();
        int acc = 0;
        for (int k : wg_items) {
            acc += k;
            offs.push_back(base + acc);
        }
        all_items.insert(all_items.end(), items.begin(), items.end());
        n_flags += P.n_slabs;
        lds_max = std::max(lds_max, P.lds);
    }
    hipError_t e = hipSuccess;
    hipFree(c->d_pitems);
    hipFree(c->d_poff);
    c->d_pitems = nullptr;
    c->d_poff = nullptr;
    e = hipMalloc((void**)&c->d_pitems, sizeof(PersistItem) * std::max<size_t>(all_items.size(), 1));
    if (e == hipSuccess) e = hipMalloc((void**)&c->d_poff, sizeof(int32_t) * offs.size());
    if (e == hipSuccess && !all_items.empty())
        e = hipMemcpy(c->d_pitems, all_items.data(), sizeof(PersistItem) * all_items.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(c->d_poff, offs.data(), sizeof(int32_t) * offs.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && (n_flags > c->n_pflags || !c->d_pflags)) {
        // word 0 is the abort word, which survives re-planning; flags follow
        uint32_t abort_word = 0;
        if (c->d_pflags)
            e = hipMemcpy(&abort_word, c->d_pflags, sizeof abort_word, hipMemcpyDeviceToHost);
        hipFree(c->d_pflags);
        c->d_pflags = nullptr;
        if (e == hipSuccess) e = hipMalloc((void**)&c->d_pflags, sizeof(uint32_t) * (n_flags + 1));
        if (e == hipSuccess) e = hipMemset(c->d_pflags, 0, sizeof(uint32_t) * (n_flags + 1));
        if (e == hipSuccess)
            e = hipMemcpy(c->d_pflags, &abort_word, sizeof abort_word, hipMemcpyHostToDevice);
        if (e == hipSuccess) c->n_pflags = n_flags;
    }
    c->n_pflags_used = n_flags;
    if (e == hipSuccess) e = persist_reserve_lds(std::max<size_t>(lds_max, 1024));
    return check_dev(c, e, "persistent plan");
}

// A persistent launch whose wait ran past its bound leaves the state
// undefined: report it (synchronising) and poison the context.
int persist_check(spinmc_ctx* c) {
    if (!c->persist_used || !c->d_pflags) return SPINMC_OK;
    uint32_t abort_word = 0;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess)
        e = hipMemcpy(&abort_word, c->d_pflags, sizeof abort_word, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return check_dev(c, e, "persistent check");
    if (abort_word != 0) {
        c->poisoned = true;
        return fail(SPINMC_E_DEVICE, "persistent passes: a workgroup waited past its bound "
                                     "(slab workgroups not resident together); state undefined");
    }
    return SPINMC_OK;
}

// (Re)build the tile table and the resident lists for a schedule.
//   mode 1: every replica resident;
//   mode 2: every replica with the chunk layout streamed (others resident);
//   mode 3: resident if it fits the LDS budget, streamed otherwise.
int prepare(spinmc_ctx* c, int mode) {
    const int tr = c->sched.tile_rows;
    const long key = ((long)mode << 56) | ((long)c->sched.rpb << 48) |
                     ((long)(c->sched.wg_threads >> 8) << 40) | ((long)c->sched.flags << 32) |
                     (long)(unsigned)tr;
    if (c->prepared && c->prepared_key == key) return SPINMC_OK;
    std::vector<int32_t> res_chunk, res_gen, spotts;
    std::vector<TileDev> tiles, ptiles;  // Ising tiles first, then Potts tiles
    for (int i = 0; i < c->R; ++i) {
        const HostRep& h = c->reps[i];
        const bool resident = (mode == 1) || !h.chunk || (mode == 3 && h.resident);
        if (resident) {
            (h.chunk ? res_chunk : res_gen).push_back(i);
            continue;
        }
        if (h.dev.model == SPINMC_POTTS) spotts.push_back(i);
        const int rows = tr > 0 ? std::min(tr, h.dev.Ly) : default_tile_rows(h);
        std::vector<TileDev>& dst = h.dev.model == SPINMC_ISING ? tiles : ptiles;
        for (int y0 = 0; y0 < h.dev.Ly; y0 += rows)
            dst.push_back(TileDev{i, y0, std::min(rows, h.dev.Ly - y0), 0});
    }
    c->n_tiles_ising = (int)tiles.size();
    tiles.insert(tiles.end(), ptiles.begin(), ptiles.end());
    {
        size_t bi = 0, bp = 0;
        for (int i = 0; i < c->R; ++i) {
            const HostRep& h = c->reps[i];
            const bool resident = (mode == 1) || !h.chunk || (mode == 3 && h.resident);
            if (!resident) (h.dev.model == SPINMC_ISING ? bi : bp) += h.lat_bytes;
        }
        const int f = c->sched.flags & (SPINMC_SCHED_NT_ON | SPINMC_SCHED_NT_OFF);
        c->nt_ising = f == SPINMC_SCHED_NT_ON || (f == 0 && bi > kNtAutoBytes);
        c->nt_potts = f == SPINMC_SCHED_NT_ON || (f == 0 && bp > kNtAutoBytes);
    }
    hipError_t e = hipStreamSynchronize(c->stream);
    drop_graphs(c);
    c->res_chunk = res_chunk;
    c->res_gen = res_gen;
    c->stream_potts = spotts;
    // Resident groups: replicas of one shape, packed rpb per workgroup so
    // that the workgroup's threads cover about one 16-byte chunk (chunk
    // path) or one site (per-site path) each per pass, while keeping at
    // least two workgroups per CU when there are enough replicas.
    c->res_groups.clear();
    std::vector<int32_t> buf;
    const int tmax = c->sched.wg_threads > 0 ? c->sched.wg_threads : 512;
    for (int pass = 0; pass < 2; ++pass) {
        const std::vector<int32_t>& L = pass == 0 ? res_chunk : res_gen;
        // chunk groups: one model and shape each; per-site groups: one shape
        std::map<std::tuple<int, int, int>, std::vector<int32_t>> shapes;
        for (int i : L) {
            const RepDev& d = c->reps[i].dev;
            shapes[std::make_tuple(pass == 0 ? d.model : 0, d.Lx, d.Ly)].push_back(i);
        }
        for (auto& kv : shapes) {
            const HostRep& h = c->reps[kv.second[0]];
            const int items = pass == 0 ? (h.dev.Ly / 2) * (h.dev.W / 16) : h.dev.Ly * h.dev.W;
            const size_t slot = align_up((size_t)8 * c->max_tab_n, 16) + align_up(h.lat_bytes, 16);
            const int n = (int)kv.second.size();
            int P = 1;
            if (c->sched.rpb > 0) {
                // forced packing: at most rpb, within the LDS budget, one
                // wave per replica at least, and no more than the group holds
                while (P * 2 <= c->sched.rpb && P * 2 <= kMaxRpb && P * 2 * 64 <= tmax &&
                       (size_t)(P * 2) * slot <= kResidentLdsBudget && P * 2 <= n)
                    P *= 2;
            } else {
                while (P * 2 <= kMaxRpb && P * 2 * items <= tmax &&
                       (size_t)(P * 2) * slot <= kResidentLdsBudget && n / (P * 2) >= 512)
                    P *= 2;
            }
            // forced packing gives every replica a wave at least (64 P <= tmax)
            int threads = c->sched.rpb > 0 ? 64 * P : 64;
            while (threads < tmax && threads < P * items) threads *= 2;
            c->res_groups.push_back({(int)buf.size(), n, P, threads, std::get<0>(kv.first),
                                     pass == 0, slot});
            buf.insert(buf.end(), kv.second.begin(), kv.second.end());
        }
    }
    // buf holds every resident replica once (at most R entries): the region
    // [off_res_chunk, off_res_chunk + R) of the list buffer
    if (e == hipSuccess && !buf.empty())
        e = hipMemcpy(c->d_lists + c->off_res_chunk, buf.data(), sizeof(int32_t) * buf.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && !spotts.empty())
        e = hipMemcpy(c->d_lists + c->off_rest, spotts.data(), sizeof(int32_t) * spotts.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && (int)tiles.size() != c->n_tiles) {
        hipFree(c->d_tiles);
        c->d_tiles = nullptr;
        c->n_tiles = 0;
        if (!tiles.empty()) e = hipMalloc((void**)&c->d_tiles, sizeof(TileDev) * tiles.size());
    }
    if (e == hipSuccess && !tiles.empty())
        e = hipMemcpy(c->d_tiles, tiles.data(), sizeof(TileDev) * tiles.size(),
                      hipMemcpyHostToDevice);
    c->n_tiles = (int)tiles.size();
    if (e == hipSuccess && !buf.empty()) {
        size_t lds = 0;
        for (const auto& g : c->res_groups) lds = std::max(lds, g.slot * g.rpb);
        e = resident_reserve_lds(lds);
    }
    if (e != hipSuccess) return check_dev(c, e, "prepare schedule");
    c->persist = (c->sched.flags & SPINMC_SCHED_PERSIST) != 0 && mode != 1 && !tiles.empty();
    if (c->persist) {
        int rc = plan_persist(c, mode);
        if (rc) return rc;
    }
    c->prepared = true;
    c->prepared_key = key;
    return SPINMC_OK;
}

SweepArgs sweep_args(spinmc_ctx* c, int n, int re, int32_t* stats) {
    SweepArgs a{};
    a.reps = c->d_reps;
    a.tiles = c->d_tiles;
    a.tab = c->d_tab;
    a.lat = c->d_lat;
    a.t_base = c->d_t;
    a.stats = stats;
    a.hist = c->d_hist;
    a.key0 = (uint32_t)(c->seed & 0xffffffffu);
    a.key1 = (uint32_t)(c->seed >> 32);
    a.R = c->R;
    a.width = c->width;
    a.n_sweeps = n;
    a.record_every = re;
    a.n_units = c->n_tiles;
    a.tab_lds_bytes = (int)align_up((size_t)8 * c->max_tab_n, 16);
    return a;
}

int ensure_side_streams(spinmc_ctx* c);

// Resident kernels for the call's sweeps: each group on its own side stream,
// forked from and joined back into stream s (so they overlap one another and
// whatever s runs meanwhile).  With join = false the caller joins later via
// join_resident.
hipError_t enqueue_resident(spinmc_ctx* c, SweepArgs a, hipStream_t s) {
    if (c->res_groups.empty()) return hipSuccess;
    if (ensure_side_streams(c) != SPINMC_OK) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(c->cap_ev[0], s);
    for (size_t k = 0; k < c->res_groups.size() && e == hipSuccess; ++k) {
        const auto& g = c->res_groups[k];
        hipStream_t side = c->cap[1 + k % kSide];
        if (k < (size_t)kSide) e = hipStreamWaitEvent(side, c->cap_ev[0], 0);
        if (e != hipSuccess) break;
        a.rep_list = c->d_lists + c->off_res_chunk + g.off;
        a.n_list = g.count;
        a.rpb = g.rpb;
        a.res_slot_bytes = (int)g.slot;
        e = timed(c, SPINMC_K_RESIDENT, [&] {
            return launch_resident(a, g.count, g.model, g.chunk, g.threads, g.slot * g.rpb, side);
        }, side);
    }
    return e;
}

hipError_t join_resident(spinmc_ctx* c, hipStream_t s) {
    hipError_t e = hipSuccess;
    const size_t used = std::min(c->res_groups.size(), (size_t)kSide);
    for (size_t k = 0; k < used && e == hipSuccess; ++k) {
        e = hipEventRecord(c->cap_ev[1 + k], c->cap[1 + k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, c->cap_ev[1 + k], 0);
    }
    return e;
}

// Streamed colour passes for sweeps [i0, i0 + n) of the call on stream s.
hipError_t enqueue_stream(spinmc_ctx* c, const SweepArgs& a, int i0, int n, int re,
                          hipStream_t s) {
    hipError_t e = hipSuccess;
    const int threads = c->sched.wg_threads > 0 ? std::min(c->sched.wg_threads, 512) : 256;
    for (int i = i0; i < i0 + n && e == hipSuccess; ++i) {
        const bool rec = re > 0 && ((i + 1) % re) == 0;
        const int row = rec ? (i + 1) / re - 1 : -1;
        const int ni = c->n_tiles_ising, np = c->n_tiles - c->n_tiles_ising;
        for (int col = 0; col < 2 && e == hipSuccess; ++col) {
            const int rr = col == 1 ? row : -1;
            if (ni > 0)
                e = timed(c, SPINMC_K_STREAM_ISING, [&] {
                    return launch_stream_pass(a, SPINMC_ISING, 0, ni, col, i, rr, threads,
                                              a.tab_lds_bytes, c->nt_ising, s);
                }, s);
            if (e == hipSuccess && np > 0)
                e = timed(c, SPINMC_K_STREAM_POTTS, [&] {
                    return launch_stream_pass(a, SPINMC_POTTS, ni, np, col, i, rr, threads,
                                              a.tab_lds_bytes, c->nt_potts, s);
                }, s);
        }
        if (e == hipSuccess && rec && !c->stream_potts.empty())
            e = launch_potts_hist_finalize(a, c->d_lists + c->off_rest,
                                           (int)c->stream_potts.size(), row, s);
    }
    return e;
}

// Persistent streamed passes for n unrecorded sweeps from sweep a.sweep_off
// of the call on stream s: the slab flags cleared by a fill kernel (no memset
// node in captured graphs), then one launch per model.
hipError_t enqueue_persist(spinmc_ctx* c, SweepArgs a, int n, hipStream_t s) {
    a.n_sweeps = n;
    hipError_t e = hipSuccess;
    uint32_t* abort_flag = c->d_pflags;
    uint32_t* flags = c->d_pflags + 1;
    if (c->n_pflags_used > 0) e = launch_fill_i32((int32_t*)flags, (size_t)c->n_pflags_used, 0, s);
    for (int m = 0; m < 2 && e == hipSuccess; ++m) {
        const auto& P = c->pplan[m];
        if (P.n_wg == 0) continue;
        const bool nt = m == 0 ? c->nt_ising : c->nt_potts;
        e = timed(c, m == 0 ? SPINMC_K_PERSIST_ISING : SPINMC_K_PERSIST_POTTS, [&] {
            return launch_persist(a, m == 0 ? kModelIsing : kModelPotts, c->d_pitems,
                                  c->d_poff + P.off0, P.n_wg, flags, abort_flag, P.slot_words,
                                  P.lds, nt, s);
        }, s);
    }
    c->persist_used = true;
    return e;
}

int ensure_side_streams(spinmc_ctx* c) {
    if (c->cap[0]) return SPINMC_OK;
    for (int k = 0; k < 1 + kSide; ++k) {
        if (hipStreamCreateWithFlags(&c->cap[k], hipStreamNonBlocking) != hipSuccess)
            return fail(SPINMC_E_DEVICE, "side stream creation failed");
        if (hipEventCreateWithFlags(&c->cap_ev[k], hipEventDisableTiming) != hipSuccess)
            return fail(SPINMC_E_DEVICE, "event creation failed");
    }
    return SPINMC_OK;
}

// One graph for a chunk of G unrecorded sweeps: the streamed passes (2G
// launches, or one persistent launch per model) and, unless stream_only,
// the resident kernels on forked branches; the device sweep counter
// advances by G at the end.
int chunk_graph(spinmc_ctx* c, int G, bool stream_only, hipGraphExec_t* out) {
    const int key = stream_only ? -G : G;
    auto it = c->graphs.find(key);
    if (it != c->graphs.end()) {
        *out = it->second;
        return SPINMC_OK;
    }
    int rc0 = ensure_side_streams(c);
    if (rc0) return rc0;
    SweepArgs a = sweep_args(c, G, 0, nullptr);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(c->cap[0], hipStreamCaptureModeRelaxed);
    const bool prof = c->prof;
    c->prof = false;
    if (e == hipSuccess && !stream_only) e = enqueue_resident(c, a, c->cap[0]);
    if (e == hipSuccess && c->n_tiles > 0)
        e = c->persist ? enqueue_persist(c, a, G, c->cap[0]) : enqueue_stream(c, a, 0, G, 0, c->cap[0]);
    if (e == hipSuccess && !stream_only) e = join_resident(c, c->cap[0]);
    c->prof = prof;
    if (e == hipSuccess) e = launch_advance(c->d_t, (uint64_t)G, c->cap[0]);
    hipError_t e2 = hipStreamEndCapture(c->cap[0], &g);
    if (e == hipSuccess) e = e2;
    hipGraphExec_t ex = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (g) hipGraphDestroy(g);
    if (e != hipSuccess) return check_dev(c, e, "graph capture");
    c->graphs[key] = ex;
    *out = ex;
    return SPINMC_OK;
}

int enqueue_sweep(spinmc_ctx* c, int n, int re, int32_t* stats) {
    const int mode = effective_mode(c);
    int rc = prepare(c, mode);
    if (rc) return rc;
    hipError_t e = hipSuccess;
    // Unrecorded, untimed calls replay cached graphs of whole chunks.  When
    // both resident groups and streamed tiles exist, the resident kernels
    // run outside the graphs, one launch per group for all n sweeps on side
    // streams forked from the call's stream (their start counter copied to
    // d_t[1] first, since the graphs advance d_t[0] meanwhile), so that they
    // overlap the streamed graph replays for the whole call rather than
    // meeting them at every chunk boundary.
    if (re == 0 && !c->prof && c->use_graphs) {
        const bool split = c->n_tiles > 0 && !c->res_groups.empty();
        const int G = std::min(n, kGraphChunk);
        const int full = n / G, rest = n - full * G;
        hipGraphExec_t ex = nullptr, ex_rest = nullptr;
        rc = chunk_graph(c, G, split, &ex);
        if (rc) return rc;
        if (rest > 0) {
            rc = chunk_graph(c, rest, split, &ex_rest);
            if (rc) return rc;
        }
        if (split) {
            e = launch_copy_counter(c->d_t, c->stream);
            SweepArgs ar = sweep_args(c, n, 0, nullptr);
            ar.t_base = c->d_t + 1;
            if (e == hipSuccess) e = enqueue_resident(c, ar, c->stream);
        }
        for (int k = 0; k < full && e == hipSuccess; ++k) e = hipGraphLaunch(ex, c->stream);
        if (e == hipSuccess && rest > 0) e = hipGraphLaunch(ex_rest, c->stream);
        if (e == hipSuccess && split) e = join_resident(c, c->stream);
        return check_dev(c, e, "sweep (graph)");
    }
    SweepArgs a = sweep_args(c, n, re, stats);
    const int n_rec = re > 0 ? n / re : 0;
    if (n_rec > 0 && c->n_tiles > 0) {
        // stream-pass statistics accumulate with atomics: clear their rows
        // first (resident replicas overwrite theirs)
        e = launch_fill_i32(stats, (size_t)n_rec * c->R * c->width, 0, c->stream);
    }
    // resident groups on side streams, one launch per group for all n
    // sweeps, concurrent with the streamed passes (as in the graph replays;
    // the device counter does not move before the end of the call);
    // persistent streamed launches in chunks of the graph's length
    if (e == hipSuccess) e = enqueue_resident(c, a, c->stream);
    if (e == hipSuccess && c->n_tiles > 0) {
        if (c->persist && re == 0) {
            for (int j0 = 0; j0 < n && e == hipSuccess; j0 += kGraphChunk) {
                SweepArgs aj = a;
                aj.sweep_off = j0;
                e = enqueue_persist(c, aj, std::min(kGraphChunk, n - j0), c->stream);
            }
        } else {
            e = enqueue_stream(c, a, 0, n, re, c->stream);
        }
    }
    if (e == hipSuccess) e = join_resident(c, c->stream);
    if (e == hipSuccess) e = launch_advance(c->d_t, (uint64_t)n, c->stream);
    return check_dev(c, e, "sweep");
}

}  // namespace

// =========================================================== Cellular Potts
namespace {

CpmArgs cpm_args(spinmc_ctx* c, int32_t* stats) {
    CpmArgs a{};
    a.reps = c->d_reps;
    a.tiles = c->d_tiles;
    a.tab = c->d_tab;
    a.lat = reinterpret_cast<int32_t*>(c->d_lat);
    a.ctype = c->d_ctype;
    a.target = c->d_target;
    a.area = c->d_area;
    a.snap = c->d_snap;
    a.sbuf = c->d_sbuf;
    a.dbuf = c->d_dbuf;
    a.total_cells = c->total_cells;
    a.js = c->d_js;
    a.t_base = c->d_t;
    a.stats = stats;
    a.key0 = (uint32_t)(c->seed & 0xffffffffu);
    a.key1 = (uint32_t)(c->seed >> 32);
    a.R = c->R;
    a.width = c->width;
    a.range = c->cpm_range;
    return a;
}

// Threads of a streamed CPM pass: the quad pass one site per lane in
// workgroups of 1024 (wg_threads 0) or 512, one quad per lane at 256; the
// other passes at most 256.
int cpm_pass_threads(const spinmc_ctx* c) {
    const int w = c->sched.wg_threads;
    if (c->cpm_range == 1 && c->cpm_quad) return w == 0 ? 1024 : w;
    return w > 0 ? std::min(w, 256) : 256;
}

// Row tiles: whole periods of the colouring (2 rows for the 2x2 sublattice,
// 6 for the 3x3 one, which also keeps them even); by default about 4096
// sites a tile, 8192 for the one-site-per-lane quad pass.
int cpm_build_tiles(spinmc_ctx* c) {
    // captured graphs refer to the tile buffer and its count
    for (auto& kv : c->graphs) hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    std::vector<TileDev> tiles;
    const int period = c->cpm_range == 2 ? 6 : 2;
    for (int i = 0; i < c->R; ++i) {
        const RepDev& r = c->reps[i].dev;
        const int per = cpm_pass_threads(c) > 256 ? 8192 : 4096;
        int rows = c->sched.tile_rows > 0 ? c->sched.tile_rows : per / r.Lx;
        rows -= rows % period;
        rows = std::max(period, std::min(rows, r.Ly));
        for (int y0 = 0; y0 < r.Ly; y0 += rows)
            tiles.push_back(TileDev{i, y0, std::min(rows, r.Ly - y0), 0});
    }
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess && (int)tiles.size() != c->n_tiles) {
        hipFree(c->d_tiles);
        c->d_tiles = nullptr;
        e = hipMalloc((void**)&c->d_tiles, sizeof(TileDev) * tiles.size());
    }
    if (e == hipSuccess)
        e = hipMemcpy(c->d_tiles, tiles.data(), sizeof(TileDev) * tiles.size(),
                      hipMemcpyHostToDevice);
    c->n_tiles = (int)tiles.size();
    c->tiles_rows = c->sched.tile_rows;
    c->tiles_threads = cpm_pass_threads(c);
    return check_dev(c, e, "CPM tiles");
}

int create_cpm(const spinmc_replica_desc* d, int n, uint64_t seed, void* stream,
               spinmc_ctx** out) {
    spinmc_ctx* c = new spinmc_ctx();
    hipGetDevice(&c->device);
    c->stream = (hipStream_t)stream;
    c->seed = seed;
    c->R = n;
    c->width = 16;
    c->cpm = true;
    c->reps.resize(n);
    size_t lat_off = 0, tab_off = 0, cell_off = 0, js_off = 0;
    std::vector<uint32_t> tab;
    std::vector<int8_t> ctype;
    std::vector<int32_t> target, js;
    for (int i = 0; i < n; ++i) {
        HostRep& h = c->reps[i];
        CpmFixed f;
        int rc = cpm_fixed_point(d[i], i, f);
        if (rc) {
            delete c;
            return rc;
        }
        h.d = d[i];
        h.d.adhesion = nullptr;
        h.d.cell_type = nullptr;
        h.d.target_area = nullptr;
        h.adh.assign(d[i].adhesion, d[i].adhesion + d[i].n_types * d[i].n_types);
        h.ctype.assign(d[i].cell_type, d[i].cell_type + d[i].q + 1);
        h.target.assign(d[i].target_area, d[i].target_area + d[i].q + 1);
        h.T = f.T;
        h.aux = f.K0;
        RepDev& r = h.dev;
        r.model = SPINMC_CPM;
        r.Lx = d[i].Lx;
        r.Ly = d[i].Ly;
        r.W = d[i].Lx / 2;
        r.q = d[i].q;
        r.rid = d[i].rid;
        r.n_types = d[i].n_types;
        r.S = f.S;
        r.LS = f.LS;
        r.K1 = f.K1;
        r.K0 = f.K0;
        h.lat_bytes = (size_t)r.Lx * r.Ly * 4;
        r.lat_off = (int64_t)(lat_off / 4);  // int32 elements
        lat_off = align_up(lat_off + h.lat_bytes, kAlign);
        r.tab_n = (int)f.T.size();
        r.tab_off = (int)tab_off;
        tab.resize(tab_off + 2 * f.T.size());
        for (size_t k = 0; k < f.T.size(); ++k) {
            tab[tab_off + k] = (uint32_t)(f.T[k] >> 16);
            tab[tab_off + f.T.size() + k] = (uint32_t)(f.T[k] & 0xFFFFu);
        }
        tab_off += 2 * f.T.size();
        c->max_tab_n = std::max(c->max_tab_n, r.tab_n);
        r.cell_off = (int)cell_off;
        ctype.insert(ctype.end(), h.ctype.begin(), h.ctype.end());
        target.insert(target.end(), h.target.begin(), h.target.end());
        cell_off += (size_t)r.q + 1;
        r.js_off = (int)js_off;
        js.insert(js.end(), f.JS.begin(), f.JS.end());
        js_off += f.JS.size();
        c->max_sites = std::max(c->max_sites, r.Lx * r.Ly);
    }
    c->total_cells = (int)cell_off;
    c->lat_bytes = lat_off + 64;
    c->cpm_range = d[0].cpm_range == 2 ? 2 : 1;  // shared by every replica (checked)
    {
        int cap = 0;
        bool quad = c->cpm_range == 1;
        for (int i = 0; i < n; ++i) {
            cap = std::max(cap, c->reps[i].dev.q + 1);
            quad = quad && (c->reps[i].dev.Lx % 8 == 0);
        }
        c->cpm_cell_cap = (int)align_up((size_t)cap, 16);
        const size_t tab_lds = align_up((size_t)8 * std::max(c->max_tab_n, 1), 16);
        c->cpm_quad = quad && c->cpm_cell_cap <= kCpmLdsCells &&
                      cpm_quad_lds_bytes((int)tab_lds, c->cpm_cell_cap) <= kCpmQuadLdsMax;
    }
    std::vector<RepDev> rd(n);
    for (int i = 0; i < n; ++i) rd[i] = c->reps[i].dev;
    if (tab.empty()) tab.push_back(0);
    auto A = [&](void** p, size_t b) { return hipMalloc(p, std::max<size_t>(b, 16)); };
    hipError_t e = hipSuccess;
    if ((e = A((void**)&c->d_lat, c->lat_bytes)) || (e = A((void**)&c->d_reps, sizeof(RepDev) * n)) ||
        (e = A((void**)&c->d_tab, sizeof(uint32_t) * tab.size())) ||
        (e = A((void**)&c->d_t, sizeof(uint64_t))) ||
        (e = A((void**)&c->d_ctype, ctype.size())) ||
        (e = A((void**)&c->d_target, sizeof(int32_t) * target.size())) ||
        (e = A((void**)&c->d_area, sizeof(int32_t) * cell_off)) ||
        (e = A((void**)&c->d_snap, sizeof(int32_t) * cell_off)) ||
        (e = A((void**)&c->d_sbuf, sizeof(int32_t) * 2 * cell_off)) ||
        (e = A((void**)&c->d_dbuf, sizeof(int32_t) * 3 * cell_off)) ||
        (e = A((void**)&c->d_js, sizeof(int32_t) * js.size()))) {
        free_all(c);
        delete c;
        hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? SPINMC_E_NOMEM : SPINMC_E_DEVICE,
                    "create: device allocation failed: %s", hipGetErrorString(e));
    }
    const uint64_t zero = 0;
    if ((e = hipMemcpy(c->d_reps, rd.data(), sizeof(RepDev) * n, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(c->d_tab, tab.data(), sizeof(uint32_t) * tab.size(),
                       hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(c->d_t, &zero, sizeof zero, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(c->d_ctype, ctype.data(), ctype.size(), hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(c->d_target, target.data(), sizeof(int32_t) * target.size(),
                       hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(c->d_js, js.data(), sizeof(int32_t) * js.size(), hipMemcpyHostToDevice)) ||
        (e = hipMemset(c->d_lat, 0, c->lat_bytes))) {
        free_all(c);
        delete c;
        return fail(SPINMC_E_DEVICE, "create: upload failed: %s", hipGetErrorString(e));
    }
    int rc = cpm_build_tiles(c);
    if (rc == SPINMC_OK) {
        CpmArgs a = cpm_args(c, nullptr);
        e = launch_cpm_area_recount(a, c->n_tiles, c->total_cells, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        rc = check_dev(c, e, "create: area count");
    }
    if (rc) {
        free_all(c);
        delete c;
        return rc;
    }
    *out = c;
    return SPINMC_OK;
}

int cpm_set_state(spinmc_ctx* c, int r, const void* host, size_t bytes) {
    const HostRep& h = c->reps[r];
    const size_t n = (size_t)h.dev.Lx * h.dev.Ly;
    if (bytes != n * 4) return fail(SPINMC_E_INVALID, "set_state: wrong byte count");
    const int32_t* v = (const int32_t*)host;
    for (size_t i = 0; i < n; ++i)
        if (v[i] < 0 || v[i] > h.dev.q)
            return fail(SPINMC_E_INVALID, "set_state: cell id out of range");
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess)
        e = hipMemcpy(reinterpret_cast<int32_t*>(c->d_lat) + h.dev.lat_off, host, bytes,
                      hipMemcpyHostToDevice);
    // the areas are recounted once before the next sweep or measurement, so
    // that setting every replica's state costs one count, not one per call
    c->cpm_areas_dirty = true;
    return check_dev(c, e, "set_state");
}

int cpm_recount_if_dirty(spinmc_ctx* c) {
    if (!c->cpm_areas_dirty) return SPINMC_OK;
    CpmArgs a = cpm_args(c, nullptr);
    hipError_t e = launch_cpm_area_recount(a, c->n_tiles, c->total_cells, c->stream);
    if (e == hipSuccess) c->cpm_areas_dirty = false;
    return check_dev(c, e, "area count");
}

// A tiled persistent launch whose barrier wait ran past its bound leaves the
// state undefined: report it (synchronising) and poison the context.
int cpm_tiled_check(spinmc_ctx* c) {
    if (!c->cpm_tiled_used || !c->d_cpm_bar) return SPINMC_OK;
    uint32_t abort_word = 0;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess)
        e = hipMemcpy(&abort_word, c->d_cpm_bar, sizeof abort_word, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return check_dev(c, e, "CPM tiled check");
    if (abort_word != 0) {
        c->poisoned = true;
        return fail(SPINMC_E_DEVICE, "CPM tiled passes: a workgroup waited past its bound "
                                     "(tile workgroups not resident together); state undefined");
    }
    return SPINMC_OK;
}

// Tiles of the tiled persistent passes for the context, or false when they
// do not apply: range 1, four-site quads, every replica of one shape, tiles
// dividing the lattice, and all tile workgroups resident at once.
bool cpm_tiled_plan(spinmc_ctx* c, int* TH, int* TW, int* n_blocks) {
    if (c->cpm_range != 1 || !c->cpm_quad) return false;
    const int Lx = c->reps[0].dev.Lx, Ly = c->reps[0].dev.Ly;
    for (const HostRep& h : c->reps)
        if (h.dev.Lx != Lx || h.dev.Ly != Ly) return false;
    int tw = 0;
    for (int cand : {64, 32, 16, 8})
        if (Lx % cand == 0) {
            tw = cand;
            break;
        }
    int th = c->sched.tile_rows > 0 ? c->sched.tile_rows : 64;
    th = std::min(th, Ly) & ~1;
    while (th >= 2 && Ly % th != 0) th -= 2;
    if (tw == 0 || th < 2) return false;
    const long blocks = (long)c->R * (Lx / tw) * (Ly / th);
    const size_t tab_bytes = align_up((size_t)8 * std::max(c->max_tab_n, 1), 16);
    int per_cu = 0, n_cu = 0;
    if (cpm_tiled_occupancy((int)tab_bytes, c->cpm_cell_cap, th, tw, &per_cu) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, c->device) !=
            hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (per_cu < 1 || blocks > (long)per_cu * n_cu) return false;
    *TH = th;
    *TW = tw;
    *n_blocks = (int)blocks;
    return true;
}

int cpm_get_state(spinmc_ctx* c, int r, void* host, size_t bytes) {
    const HostRep& h = c->reps[r];
    if (bytes != (size_t)h.dev.Lx * h.dev.Ly * 4)
        return fail(SPINMC_E_INVALID, "get_state: wrong byte count");
    if (int rc = cpm_tiled_check(c)) return rc;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess)
        e = hipMemcpy(host, reinterpret_cast<int32_t*>(c->d_lat) + h.dev.lat_off, bytes,
                      hipMemcpyDeviceToHost);
    return check_dev(c, e, "get_state");
}

// The colour pass `col` of sweep `i` of a call.
hipError_t cpm_enqueue_pass(spinmc_ctx* c, const CpmArgs& a, int i, int col, hipStream_t s) {
    const size_t tab_bytes = align_up((size_t)8 * std::max(c->max_tab_n, 1), 16);
    const int threads = cpm_pass_threads(c);
    return timed(c, SPINMC_K_CPM_PASS, [&] {
        if (c->cpm_range == 2)
            return launch_cpm_pass5(a, c->n_tiles, col, i, threads, tab_bytes, s);
        if (c->cpm_quad)
            return launch_cpm_pass_quad(a, c->n_tiles, col, i, threads, (int)tab_bytes,
                                        c->cpm_cell_cap, s);
        return launch_cpm_pass(a, c->n_tiles, col, i, threads, tab_bytes, s);
    }, s);
}

// One graph for a chunk of G unrecorded Monte Carlo steps (their n_col G
// colour passes; the device step counter advances by G at its end), replayed
// instead of the direct launches.
int cpm_chunk_graph(spinmc_ctx* c, int G, hipGraphExec_t* out) {
    auto it = c->graphs.find(G);
    if (it != c->graphs.end()) {
        *out = it->second;
        return SPINMC_OK;
    }
    int rc0 = ensure_side_streams(c);
    if (rc0) return rc0;
    CpmArgs a = cpm_args(c, nullptr);
    const int n_col = c->cpm_range == 2 ? 9 : 4;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(c->cap[0], hipStreamCaptureModeRelaxed);
    const bool prof = c->prof;
    c->prof = false;
    for (int i = 0; i < G && e == hipSuccess; ++i)
        for (int col = 0; col < n_col && e == hipSuccess; ++col)
            e = cpm_enqueue_pass(c, a, i, col, c->cap[0]);
    c->prof = prof;
    if (e == hipSuccess) e = launch_advance(c->d_t, (uint64_t)G, c->cap[0]);
    hipError_t e2 = hipStreamEndCapture(c->cap[0], &g);
    if (e == hipSuccess) e = e2;
    hipGraphExec_t ex = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (g) hipGraphDestroy(g);
    if (e != hipSuccess) return check_dev(c, e, "CPM graph capture");
    c->graphs[G] = ex;
    *out = ex;
    return SPINMC_OK;
}

int cpm_sweep(spinmc_ctx* c, int n, int re, int32_t* stats) {
    if (c->tiles_rows != c->sched.tile_rows || c->tiles_threads != cpm_pass_threads(c)) {
        int rc = cpm_build_tiles(c);
        if (rc) return rc;
    }
    if (int rc = cpm_recount_if_dirty(c)) return rc;
    CpmArgs a = cpm_args(c, stats);
    const size_t tab_bytes = align_up((size_t)8 * std::max(c->max_tab_n, 1), 16);
    if (c->cpm_quad && !c->cpm_lds_reserved) {
        hipError_t er = cpm_reserve_lds(cpm_quad_lds_bytes((int)tab_bytes, c->cpm_cell_cap));
        if (er != hipSuccess) return check_dev(c, er, "CPM LDS reservation");
        c->cpm_lds_reserved = true;
    }
    hipError_t e = hipSuccess;
    // unrecorded steps of lattices whose ids and tables fit 64 KiB of LDS (the
    // 3x3 neighbourhood with every Lx % 8 == 0, or the 5x5 one): the resident
    // kernel, one launch per chunk of at most 500 steps (the step counter
    // advances after each), unless streamed passes are requested
    if (re == 0 && !c->prof && (c->cpm_quad || c->cpm_range == 2) && c->sched.mode != 2 &&
        cpm_resident_lds_bytes((int)tab_bytes, c->cpm_cell_cap, c->max_sites) <= 64 * 1024) {
        for (int done = 0; done < n && e == hipSuccess;) {
            const int k = std::min(500, n - done);
            e = launch_cpm_resident(a, k, (int)tab_bytes, c->cpm_cell_cap, c->max_sites,
                                    c->stream);
            if (e == hipSuccess) e = launch_advance(c->d_t, (uint64_t)k, c->stream);
            done += k;
        }
        return check_dev(c, e, "sweep (resident)");
    }
    if (n == 0) return SPINMC_OK;
    // tiled persistent passes (schedule flag SPINMC_SCHED_PERSIST): one
    // launch per chunk of up to 500 steps, barriers cleared before each
    int TH = 0, TW = 0, n_blocks = 0;
    if (re == 0 && (c->sched.flags & SPINMC_SCHED_PERSIST) && cpm_tiled_plan(c, &TH, &TW, &n_blocks)) {
        if (!c->d_cpm_bar) {
            if (hipMalloc((void**)&c->d_cpm_bar, sizeof(uint32_t) * (c->R + 1)) != hipSuccess ||
                hipMemset(c->d_cpm_bar, 0, sizeof(uint32_t) * (c->R + 1)) != hipSuccess) {
                (void)hipGetLastError();
                return fail(SPINMC_E_NOMEM, "sweep: CPM barrier words");
            }
        }
        e = launch_cpm_pass_init(a, 0, c->stream);
        for (int done = 0; done < n && e == hipSuccess;) {
            const int k = std::min(500, n - done);
            e = launch_fill_i32(reinterpret_cast<int32_t*>(c->d_cpm_bar + 1), (size_t)c->R, 0,
                                c->stream);
            if (e == hipSuccess)
                e = timed(c, SPINMC_K_CPM_TILED, [&] {
                    return launch_cpm_tiled(a, k, TH, TW, (int)tab_bytes, c->cpm_cell_cap,
                                            n_blocks, c->d_cpm_bar + 1, c->d_cpm_bar, c->stream);
                }, c->stream);
            if (e == hipSuccess) e = launch_advance(c->d_t, (uint64_t)k, c->stream);
            done += k;
        }
        if (e == hipSuccess) e = launch_cpm_pass_final(a, 0, c->stream);
        c->cpm_tiled_used = true;
        return check_dev(c, e, "sweep (tiled)");
    }
    // the streamed passes keep their snapshots in rotating buffers seeded
    // from the areas here and folded back into them at the end of the call
    // (and before recorded statistics)
    if (re == 0 && !c->prof && c->use_graphs) {
        const int G = std::min(n, kGraphChunk);
        const int full = n / G, rest = n - full * G;
        hipGraphExec_t ex = nullptr;
        int rc = cpm_chunk_graph(c, G, &ex);
        if (rc) return rc;
        hipGraphExec_t ex_rest = nullptr;
        if (rest > 0) {
            rc = cpm_chunk_graph(c, rest, &ex_rest);
            if (rc) return rc;
        }
        e = launch_cpm_pass_init(a, 0, c->stream);
        for (int k = 0; k < full && e == hipSuccess; ++k) e = hipGraphLaunch(ex, c->stream);
        if (e == hipSuccess && rest > 0) e = hipGraphLaunch(ex_rest, c->stream);
        if (e == hipSuccess) e = launch_cpm_pass_final(a, 0, c->stream);
        return check_dev(c, e, "sweep (graph)");
    }
    const int n_rec = re > 0 ? n / re : 0;
    if (n_rec > 0) e = launch_fill_i32(stats, (size_t)n_rec * c->R * c->width, 0, c->stream);
    const int n_col = c->cpm_range == 2 ? 9 : 4;
    if (e == hipSuccess) e = launch_cpm_pass_init(a, 0, c->stream);
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        for (int col = 0; col < n_col && e == hipSuccess; ++col)
            e = cpm_enqueue_pass(c, a, i, col, c->stream);
        if (e == hipSuccess && re > 0 && ((i + 1) % re) == 0) {
            e = launch_cpm_pass_final(a, i + 1, c->stream);
            if (e == hipSuccess) e = launch_cpm_stats(a, c->n_tiles, (i + 1) / re - 1, c->stream);
        }
    }
    if (e == hipSuccess) e = launch_cpm_pass_final(a, n, c->stream);
    if (e == hipSuccess) e = launch_advance(c->d_t, (uint64_t)n, c->stream);
    return check_dev(c, e, "sweep");
}

int cpm_measure(spinmc_ctx* c, int32_t* stats, double* obs) {
    if (int rc = cpm_recount_if_dirty(c)) return rc;
    CpmArgs a = cpm_args(c, stats);
    hipError_t e = launch_fill_i32(stats, (size_t)c->R * c->width, 0, c->stream);
    if (e == hipSuccess) e = launch_cpm_stats(a, c->n_tiles, 0, c->stream);
    if (e == hipSuccess && obs)
        e = launch_observables(c->d_reps, c->R, stats, c->width, obs, c->stream);
    return check_dev(c, e, "measure");
}

// ============================================================ triangular Ising
// Thresholds of the flip for idx = 7 [s > 0] + (S6 + 6) / 2 in FP64 (the
// Algorithm-1 test; T = 2^32 accepts always).
void tri_thresholds(const spinmc_replica_desc& d, std::vector<uint64_t>& T) {
    T.resize(kTriClasses);
    for (int si = 0; si < 2; ++si)
        for (int a = 0; a < 7; ++a) {
            const double s = si ? 1.0 : -1.0;
            double u = (double)d.Jx * (double)(2 * a - 6);
            u = u + (double)d.h;
            const double dE = 2.0 * s * u;
            T[7 * si + a] = dE <= 0.0 ? ((uint64_t)1 << 32)
                                      : (uint64_t)std::ceil(std::ldexp(std::exp(-d.beta * dE), 32));
        }
}

TriArgs tri_args(spinmc_ctx* c, int32_t* stats) {
    TriArgs a{};
    a.reps = c->d_reps;
    a.lat = reinterpret_cast<int8_t*>(c->d_lat);
    a.tab = c->d_tab64;
    a.t_base = c->d_t;
    a.stats = stats;
    a.key0 = (uint32_t)(c->seed & 0xffffffffu);
    a.key1 = (uint32_t)(c->seed >> 32);
    a.R = c->R;
    a.width = c->width;
    int mb = 0;
    bool l12 = true, l8 = true;
    a.model = c->reps[0].dev.model;
    for (const HostRep& h : c->reps) {
        l8 = l8 && h.dev.Lx % 8 == 0;
        if (a.model == kModelIsingHC)
            mb = std::max(mb, (h.dev.Lx * h.dev.Ly * h.dev.q / 2 + 3) / 4);
        else
            mb = std::max(mb, (h.dev.Lx * h.dev.Ly / 3 + 3) / 4);
        l12 = l12 && h.dev.Lx % 12 == 0;
    }
    a.max_blocks = mb;
    a.all_lx12 = l12 ? 1 : 0;
    a.all_lx8 = l8 ? 1 : 0;
    a.max_sites = c->max_sites;
    return a;
}

int create_tri(const spinmc_replica_desc* d, int n, uint64_t seed, int init, void* stream,
               spinmc_ctx** out) {
    spinmc_ctx* c = new spinmc_ctx();
    hipGetDevice(&c->device);
    c->stream = (hipStream_t)stream;
    c->seed = seed;
    c->R = n;
    c->width = 8;
    c->tri = true;
    c->reps.resize(n);
    std::vector<uint64_t> tab((size_t)n * kTriClasses);
    std::vector<RepDev> rd(n);
    size_t lat_off = 0;
    for (int i = 0; i < n; ++i) {
        HostRep& h = c->reps[i];
        h.d = d[i];
        tri_thresholds(d[i], h.T);
        std::copy(h.T.begin(), h.T.end(), tab.begin() + (size_t)i * kTriClasses);
        RepDev& r = h.dev;
        r.model = d[i].model == SPINMC_ISING_HC ? kModelIsingHC : kModelIsingTri;
        r.Lx = d[i].Lx;
        r.Ly = d[i].Ly;
        r.q = d[i].model == SPINMC_ISING_HC && d[i].Lz > 1 ? d[i].Lz : 1;  // Lz
        r.W = d[i].Lx;
        r.rid = d[i].rid;
        r.Jx = d[i].Jx;
        r.Jy = d[i].Jy;
        r.h = d[i].h;
        r.beta = d[i].beta;
        h.lat_bytes = (size_t)r.Lx * r.Ly * r.q;
        r.lat_off = (int64_t)lat_off;
        lat_off = align_up(lat_off + h.lat_bytes, kAlign);
        rd[i] = r;
        c->max_sites = std::max(c->max_sites, r.Lx * r.Ly * r.q);
    }
    c->lat_bytes = lat_off + 64;
    auto A = [&](void** p, size_t b) { return hipMalloc(p, std::max<size_t>(b, 16)); };
    hipError_t e = hipSuccess;
    if ((e = A((void**)&c->d_lat, c->lat_bytes)) || (e = A((void**)&c->d_reps, sizeof(RepDev) * n)) ||
        (e = A((void**)&c->d_tab64, sizeof(uint64_t) * tab.size())) ||
        (e = A((void**)&c->d_t, sizeof(uint64_t)))) {
        free_all(c);
        delete c;
        hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? SPINMC_E_NOMEM : SPINMC_E_DEVICE,
                    "create: device allocation failed: %s", hipGetErrorString(e));
    }
    const uint64_t zero = 0;
    if ((e = hipMemcpy(c->d_reps, rd.data(), sizeof(RepDev) * n, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(c->d_tab64, tab.data(), sizeof(uint64_t) * tab.size(),
                       hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(c->d_t, &zero, sizeof zero, hipMemcpyHostToDevice))) {
        free_all(c);
        delete c;
        return fail(SPINMC_E_DEVICE, "create: upload failed: %s", hipGetErrorString(e));
    }
    // init = 0: every spin -1 (as for the square lattice); init = 1: the init stream
    e = hipMemset(c->d_lat, 0xFF, c->lat_bytes);
    if (e == hipSuccess && init) {
        TriArgs a = tri_args(c, nullptr);
        e = launch_tri_init(a, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    if (e != hipSuccess) {
        free_all(c);
        delete c;
        return fail(SPINMC_E_DEVICE, "create: init failed: %s", hipGetErrorString(e));
    }
    *out = c;
    return SPINMC_OK;
}

// Chain / square / cubic spins between the natural order (z Ly + y) Lx + x
// of host buffers and the device's colour planes (site (z, y, x) at byte
// (z Ly + y, x >> 1) of plane (x + y + z) & 1, planes of Ly Lz rows by Lx / 2).
static void hc_permute(const RepDev& d, const int8_t* src, int8_t* dst, bool to_planes) {
    const size_t W = (size_t)d.Lx / 2, psz = (size_t)d.Ly * d.q * W;
    for (int z = 0; z < d.q; ++z)
        for (int y = 0; y < d.Ly; ++y)
            for (int x = 0; x < d.Lx; ++x) {
                const size_t row = (size_t)z * d.Ly + y;
                const size_t nat = row * d.Lx + x;
                const size_t pl = (size_t)((x + y + z) & 1) * psz + row * W + (x >> 1);
                if (to_planes)
                    dst[pl] = src[nat];
                else
                    dst[nat] = src[pl];
            }
}

// Triangular spins between the natural order y Lx + x and the device's three
// colour planes (site (y, x) at byte (y, x / 3) of plane (x + 2y) mod 3,
// planes of Ly rows by Lx / 3).
static void tri_permute(const RepDev& d, const int8_t* src, int8_t* dst, bool to_planes) {
    const size_t W3 = (size_t)d.Lx / 3, psz = (size_t)d.Ly * W3;
    for (int y = 0; y < d.Ly; ++y)
        for (int x = 0; x < d.Lx; ++x) {
            const size_t nat = (size_t)y * d.Lx + x;
            const size_t pl = (size_t)((x + 2 * y) % 3) * psz + (size_t)y * W3 + (size_t)(x / 3);
            if (to_planes)
                dst[pl] = src[nat];
            else
                dst[nat] = src[pl];
        }
}

int tri_set_state(spinmc_ctx* c, int r, const void* host, size_t bytes) {
    const HostRep& h = c->reps[r];
    if (bytes != h.lat_bytes) return fail(SPINMC_E_INVALID, "set_state: wrong byte count");
    const int8_t* v = (const int8_t*)host;
    for (size_t i = 0; i < bytes; ++i)
        if (v[i] != 1 && v[i] != -1) return fail(SPINMC_E_INVALID, "set_state: Ising spins must be +-1");
    std::vector<int8_t> planes(bytes);
    if (h.dev.model == kModelIsingHC)
        hc_permute(h.dev, v, planes.data(), true);
    else
        tri_permute(h.dev, v, planes.data(), true);
    v = planes.data();
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemcpy(c->d_lat + h.dev.lat_off, v, bytes, hipMemcpyHostToDevice);
    return check_dev(c, e, "set_state");
}

int tri_get_state(spinmc_ctx* c, int r, void* host, size_t bytes) {
    const HostRep& h = c->reps[r];
    if (bytes != h.lat_bytes) return fail(SPINMC_E_INVALID, "get_state: wrong byte count");
    hipError_t e = hipStreamSynchronize(c->stream);
    std::vector<int8_t> planes(bytes);
    if (e == hipSuccess)
        e = hipMemcpy(planes.data(), c->d_lat + h.dev.lat_off, bytes, hipMemcpyDeviceToHost);
    if (e == hipSuccess) {
        if (h.dev.model == kModelIsingHC)
            hc_permute(h.dev, planes.data(), (int8_t*)host, false);
        else
            tri_permute(h.dev, planes.data(), (int8_t*)host, false);
    }
    return check_dev(c, e, "get_state");
}

// Resident schedule (recorded sweeps too): every lattice in LDS (<= 64 KiB,
// so that two workgroups fit a compute unit) and the span alignment.
bool tri_resident_ok(const spinmc_ctx* c, const TriArgs& a, int* lds) {
    if (c->sched.mode == 2) return false;  // streamed passes requested
    size_t mx = 0;
    for (const HostRep& h : c->reps) {
        mx = std::max(mx, h.lat_bytes);
        if (a.model == kModelIsingHC ? h.dev.Lx % 8 : h.dev.Lx % 12) return false;
        if (h.lat_bytes % 4) return false;
    }
    if (mx > 64 * 1024) return false;
    *lds = (int)align_up(mx, 16);
    return true;
}

int tri_sweep(spinmc_ctx* c, int n, int re, int32_t* stats) {
    TriArgs a = tri_args(c, stats);
    hipError_t e = hipSuccess;
    int lds = 0;
    const int n_rec = re > 0 ? n / re : 0;
    if (n_rec > 0) e = launch_fill_i32(stats, (size_t)n_rec * c->R * c->width, 0, c->stream);
    if (tri_resident_ok(c, a, &lds)) {
        // chunks of at most 1000 sweeps per launch (statistics recorded inside);
        // the counter advances after each
        for (int done = 0; done < n && e == hipSuccess;) {
            const int k = std::min(1000, n - done);
            // the launch's recorded rows (16 B each) gather in LDS behind the lattice
            const int rows = re > 0 ? (done + k) / re - done / re : 0;
            const int lds_k = lds + 16 * rows;
            e = timed(c, SPINMC_K_RESIDENT,
                      [&] { return launch_nat_resident(a, k, done, re, lds_k, c->stream); },
                      c->stream);
            if (e == hipSuccess) e = launch_advance(c->d_t, (uint64_t)k, c->stream);
            done += k;
        }
        return check_dev(c, e, "sweep");
    }
    const bool hc = a.model == kModelIsingHC;
    const int n_col = hc ? 2 : 3;
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        for (int col = 0; col < n_col && e == hipSuccess; ++col)
            e = timed(c, hc ? SPINMC_K_HC_PASS : SPINMC_K_TRI_PASS,
                      [&] { return launch_tri_pass(a, col, i, c->stream); }, c->stream);
        if (e == hipSuccess && re > 0 && ((i + 1) % re) == 0)
            e = launch_tri_stats(a, (i + 1) / re - 1, c->stream);
    }
    if (e == hipSuccess) e = launch_advance(c->d_t, (uint64_t)n, c->stream);
    return check_dev(c, e, "sweep");
}

int tri_measure(spinmc_ctx* c, int32_t* stats, double* obs) {
    TriArgs a = tri_args(c, stats);
    hipError_t e = launch_fill_i32(stats, (size_t)c->R * c->width, 0, c->stream);
    if (e == hipSuccess) e = launch_tri_stats(a, 0, c->stream);
    if (e == hipSuccess && obs) e = launch_tri_observables(a, obs, c->stream);
    return check_dev(c, e, "measure");
}

// ================================================= multispin-coded Ising
// The square lattice's 18 classes idx = 9 [s > 0] + 3 (Sx/2 + 1) + (Sy/2 + 1)
// in FP64 (dE = 2 s (Jx Sx + Jy Sy + h); T = 2^32 accepts always).
void msc_thresholds(const spinmc_replica_desc& d, std::vector<uint64_t>& T) {
    T.resize(kMscClasses);
    for (int si = 0; si < 2; ++si)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                const double s = si ? 1.0 : -1.0;
                double u = (double)d.Jx * (2.0 * a - 2.0);
                u = u + (double)d.Jy * (2.0 * b - 2.0);
                u = u + (double)d.h;
                const double dE = 2.0 * s * u;
                T[9 * si + 3 * a + b] =
                    dE <= 0.0 ? ((uint64_t)1 << 32)
                              : (uint64_t)std::ceil(std::ldexp(std::exp(-d.beta * dE), 32));
            }
}

MscArgs msc_args(spinmc_ctx* c, int32_t* stats) {
    MscArgs a{};
    a.reps = c->d_reps;
    a.lat = reinterpret_cast<uint32_t*>(c->d_lat);
    a.tab = c->d_tab64;
    a.t_base = c->d_t;
    a.stats = stats;
    a.key0 = (uint32_t)(c->seed & 0xffffffffu);
    a.key1 = (uint32_t)(c->seed >> 32);
    a.G = (int)c->reps.size();
    a.width = c->width;
    int mb = 0;
    for (const HostRep& h : c->reps) mb = std::max(mb, h.dev.Lx * h.dev.Ly / 8);
    a.max_blocks = mb;
    a.max_sites = c->max_sites;
    return a;
}

int create_msc(const spinmc_replica_desc* d, int n, uint64_t seed, int init, void* stream,
               spinmc_ctx** out) {
    spinmc_ctx* c = new spinmc_ctx();
    hipGetDevice(&c->device);
    c->stream = (hipStream_t)stream;
    c->seed = seed;
    c->R = 32 * n;
    c->width = 8;
    c->msc = true;
    c->reps.resize(n);
    std::vector<uint64_t> tab((size_t)n * kMscClasses);
    std::vector<RepDev> rd(n), robs((size_t)32 * n);
    size_t lat_off = 0;
    for (int i = 0; i < n; ++i) {
        HostRep& h = c->reps[i];
        h.d = d[i];
        msc_thresholds(d[i], h.T);
        std::copy(h.T.begin(), h.T.end(), tab.begin() + (size_t)i * kMscClasses);
        RepDev& r = h.dev;
        r.model = kModelIsingMsc;
        r.Lx = d[i].Lx;
        r.Ly = d[i].Ly;
        r.W = d[i].Lx;
        r.rid = d[i].rid;
        r.Jx = d[i].Jx;
        r.Jy = d[i].Jy;
        r.h = d[i].h;
        r.beta = d[i].beta;
        h.lat_bytes = (size_t)r.Lx * r.Ly * 4;
        r.lat_off = (int64_t)lat_off;
        lat_off = align_up(lat_off + h.lat_bytes, kAlign);
        rd[i] = r;
        for (int b = 0; b < 32; ++b) {  // observables: square-lattice Ising entries
            RepDev o = r;
            o.model = kModelIsing;
            robs[(size_t)32 * i + b] = o;
        }
        c->max_sites = std::max(c->max_sites, r.Lx * r.Ly);
    }
    c->lat_bytes = lat_off + 64;
    auto A = [&](void** p, size_t b) { return hipMalloc(p, std::max<size_t>(b, 16)); };
    hipError_t e = hipSuccess;
    if ((e = A((void**)&c->d_lat, c->lat_bytes)) || (e = A((void**)&c->d_reps, sizeof(RepDev) * n)) ||
        (e = A((void**)&c->d_reps_obs, sizeof(RepDev) * robs.size())) ||
        (e = A((void**)&c->d_tab64, sizeof(uint64_t) * tab.size())) ||
        (e = A((void**)&c->d_t, sizeof(uint64_t)))) {
        free_all(c);
        delete c;
        hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? SPINMC_E_NOMEM : SPINMC_E_DEVICE,
                    "create: device allocation failed: %s", hipGetErrorString(e));
    }
    const uint64_t zero = 0;
    if ((e = hipMemcpy(c->d_reps, rd.data(), sizeof(RepDev) * n, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(c->d_reps_obs, robs.data(), sizeof(RepDev) * robs.size(),
                       hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(c->d_tab64, tab.data(), sizeof(uint64_t) * tab.size(),
                       hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(c->d_t, &zero, sizeof zero, hipMemcpyHostToDevice))) {
        free_all(c);
        delete c;
        return fail(SPINMC_E_DEVICE, "create: upload failed: %s", hipGetErrorString(e));
    }
    // init = 0: every spin -1 (all bits 0); init = 1: the init stream per bit
    e = hipMemset(c->d_lat, 0, c->lat_bytes);
    if (e == hipSuccess && init) {
        MscArgs a = msc_args(c, nullptr);
        e = launch_msc_init(a, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    if (e != hipSuccess) {
        free_all(c);
        delete c;
        return fail(SPINMC_E_DEVICE, "create: init failed: %s", hipGetErrorString(e));
    }
    *out = c;
    return SPINMC_OK;
}

int msc_sweep(spinmc_ctx* c, int n, int re, int32_t* stats) {
    MscArgs a = msc_args(c, stats);
    hipError_t e = hipSuccess;
    const int n_rec = re > 0 ? n / re : 0;
    if (n_rec > 0) e = launch_fill_i32(stats, (size_t)n_rec * c->R * c->width, 0, c->stream);
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        for (int col = 0; col < 2 && e == hipSuccess; ++col)
            e = timed(c, SPINMC_K_MSC_PASS, [&] { return launch_msc_pass(a, col, i, c->stream); },
                      c->stream);
        if (e == hipSuccess && re > 0 && ((i + 1) % re) == 0)
            e = launch_msc_stats(a, (i + 1) / re - 1, c->stream);
    }
    if (e == hipSuccess) e = launch_advance(c->d_t, (uint64_t)n, c->stream);
    return check_dev(c, e, "sweep");
}

int msc_measure(spinmc_ctx* c, int32_t* stats, double* obs) {
    MscArgs a = msc_args(c, stats);
    hipError_t e = launch_fill_i32(stats, (size_t)c->R * c->width, 0, c->stream);
    if (e == hipSuccess) e = launch_msc_stats(a, 0, c->stream);
    if (e == hipSuccess && obs)
        e = launch_observables(c->d_reps_obs, c->R, stats, c->width, obs, c->stream);
    return check_dev(c, e, "measure");
}

}  // namespace
