/*
 * spinmc.h -- C ABI of libspinmc, the MI355X (gfx950) checkerboard
 * Metropolis-Hastings sampler for the Ising, q-state Potts and Cellular
 * Potts models of "A differentiable programming framework for spin models"
 * (Farias, Schultz, Mombach, Maziero).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every function returns a spinmc_status (0 = OK, < 0 = error).  On error
 *   nothing is enqueued and no state changes; spinmc_last_error() returns a
 *   thread-local message.  After a device fault a context is poisoned: every
 *   call but spinmc_destroy returns SPINMC_E_DEVICE.
 * - "dev" pointers are device memory owned by the caller (for example torch
 *   tensors); "host" pointers are host memory.  Device work is enqueued on the
 *   HIP stream given to spinmc_create (NULL = the null stream) and runs
 *   asynchronously unless stated otherwise.
 * - Lattices are periodic, Ly rows by Lx columns, Lx and Ly even.  Site
 *   (y, x) has colour (x + y) & 1 for Ising/Potts (Related Work, checkerboard
 *   decomposition, Fig. 1) and 2 (y & 1) + (x & 1) for the Cellular Potts
 *   model, whose Moore neighbourhood needs four colours.
 * - A sweep (Ising/Potts) is the colour-0 pass then the colour-1 pass; a
 *   Cellular Potts Monte Carlo step is the four colour passes in order.  The
 *   global sweep counter t (persisted in the context) numbers the passes
 *   p = 2t + c (CPM: 4t + c), which key the Philox4x32-10 streams together
 *   with the seed and the replica id.  Results depend only on (seed, rid,
 *   t, state), never on batching, tiling or the schedule.
 * - A context is not thread-safe; separate contexts are independent.
 */
#ifndef SPINMC_H
#define SPINMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spinmc_ctx spinmc_ctx;

enum spinmc_model {
    SPINMC_ISING = 0,
    SPINMC_POTTS = 1,
    SPINMC_CPM = 2,
    SPINMC_ISING_TRI = 3,   /* triangular lattice                                  */
    SPINMC_ISING_HC = 4,    /* chain / square / simple cubic, natural layout (Lz)  */
    SPINMC_ISING_MSC = 5    /* multispin-coded square lattice: 32 replicas a word */
};

enum spinmc_status {
    SPINMC_OK = 0,
    SPINMC_E_INVALID = -1,          /* bad argument (shape, range, NULL, NaN)          */
    SPINMC_E_UNSUPPORTED = -2,      /* valid but not implemented by this library        */
    SPINMC_E_NOMEM = -3,            /* device allocation failed; nothing leaked         */
    SPINMC_E_DEVICE = -4,           /* no usable GPU, or a device fault (ctx poisoned)  */
    SPINMC_E_NOT_REPRESENTABLE = -5,/* CPM energies not exact in the fixed-point scale */
    SPINMC_E_STATE = -6             /* call not valid in the current state              */
};

/* Integer statistics recorded per replica and per recorded sweep
 * (spinmc_stats_width() int32 entries, 8 or 16):
 *   Ising  [M, Bx, By, 0...]   M = sum s, Bx = sum s(y,x) s(y,x+1),
 *                              By = sum s(y,x) s(y+1,x)        (Eq. (1))
 *   Potts  [Nx, Ny, S, nmax, 0...]  equal horizontal / vertical bonds, sum
 *                              of labels, population of the largest state
 *                              (Eq. (2))
 *   Chain / cubic Ising (SPINMC_ISING_HC) [M, Bx, By, Bz, 0...] bond sums
 *                              along x, y, z (0 for an absent dimension)
 *   Triangular Ising [M, Bh, Bv, Bd, 0...]  Bh = sum s(y,x) s(y,x+1),
 *                              Bv = sum s(y,x) s(y+1,x), Bd = sum s(y,x)
 *                              s(y+1,x-1)
 *   CPM    [b0..b9, Hlo, Hhi, 0...] von Neumann bonds between different ids
 *                              by unordered type pair (a <= b, index
 *                              a*n_types - a(a-1)/2 + (b - a)), and the
 *                              energy of Eq. (3) (adhesion over the pairs
 *                              of the replica's neighbourhood) times the
 *                              fixed-point scale S as an int64 split in two
 *                              int32 words.                                 */

/* Triangular-lattice Ising (the triangular kernels of the Methods;
 * SPINMC_ISING_TRI): spins on an Ly x Lx array, neighbours (y, x+-1),
 * (y+-1, x), (y-1, x+1), (y+1, x-1), periodic; one coupling J = Jx (Jy must
 * equal Jx) for every bond, H = -J sum s s' - h sum s.  Three colours
 * c = (x + 2y) mod 3, passes p = 3t + c per sweep; the sites of colour c with
 * within-colour index k = y Lx/3 + x/3 take word k & 3 of Philox block
 * (k >> 2, p, rid, 0) whole as W and flip iff W < ceil(2^32 exp(-beta dE)),
 * dE = 2 s (J S6 + h) (always when dE <= 0).  Initial state as for Ising.
 * A context holds only triangular replicas.  Sweeps, recorded or not, run
 * resident in LDS (one workgroup per replica) when every lattice holds at
 * most 64 KiB and every Lx is a multiple of 12, unless the schedule's mode
 * is 2 (streamed passes); tile_rows and wg_threads are ignored, and
 * spinmc_autotune returns the schedule unchanged.  spinmc_grad is not
 * available.
 *
 * Chain, square and simple-cubic Ising in one natural layout (the 1D, 2D and
 * 3D convolutions of the Methods; SPINMC_ISING_HC): an Lz x Ly x Lx array,
 * n = (z Ly + y) Lx + x; Lx even >= 2, Ly and Lz each 1 (absent) or even
 * >= 2; neighbours x +- 1 and, where present, y +- 1, z +- 1 (periodic); one
 * coupling J = Jx (Jy must equal Jx).  Two colours c = (x + y + z) & 1,
 * p = 2t + c; the colour-c site of the pair (2k, 2k + 1) takes word k & 3 of
 * Philox block (k >> 2, p, rid, 0) whole as W; flip iff
 * W < ceil(2^32 exp(-beta 2 s (J S + h))), S the neighbour sum.  States are
 * int8 [Lz][Ly][Lx]; contexts as for the triangular lattice (resident when
 * every lattice holds at most 64 KiB and every Lx is a multiple of 8).
 *
 * Multispin-coded square-lattice Ising (1-bit spins; SPINMC_ISING_MSC): one
 * descriptor is a group of 32 replicas with its Lx (a multiple of 8), Ly
 * (even), Jx, Jy, h, beta and rid, packed bit by bit in one uint32 per site
 * (bit b = 1: s = +1 in replica b; natural layout y Lx + x).  The 32 replicas
 * share the random numbers: in pass p = 2t + c each site of colour
 * c = (x + y) & 1 with within-colour index k = n >> 1 takes W = word k & 3
 * of Philox block (k >> 2, p, rid, 0) whole, and every bit whose
 * square-lattice class (as for SPINMC_ISING) has W < T flips.  Initial bit
 * b of site n: 1 iff word n & 3 of block (n >> 2, b, rid, 2) is < 2^31.
 * The replicas are correlated through the shared draws; each one alone is
 * a Metropolis chain.  A context of G groups reports 32 G replicas to
 * spinmc_num_replicas / sweep / measure (replica 32 g + b, statistics
 * [M, Bx, By] as for SPINMC_ISING); spinmc_get_state / set_state move the
 * uint32 words of group g (Ly Lx * 4 bytes).  Only groups in a context.     */

/* Hamiltonian parameters of one replica (Eq. (1), Eq. (2), Eq. (3)).
 * Signs: Ising H = -Jx sum_h s s' - Jy sum_v s s' - h sum s with s = +-1;
 * Potts H = -Jx sum delta(s, s') - h sum s with labels 0..q-1 (Jy must equal
 * Jx); both count every nearest-neighbour bond once, so J > 0 is
 * ferromagnetic (the paper writes the same model with J = -1).
 * CPM H = sum over unordered Moore pairs J[type][type'] [id != id']
 *         + lambda sum over cells (a - A)^2 (no area term for id 0, the
 *         medium).  The descriptor is deep-copied by spinmc_create.          */
typedef struct spinmc_replica_desc {
    int32_t model;               /* enum spinmc_model                              */
    int32_t Lx, Ly;              /* even, >= 2 (triangular: multiples of 3, >= 3)    */
    int32_t q;                   /* Potts: 2..255; CPM: number of cells n (ids 0..n); Ising: ignored */
    float Jx, Jy, h;             /* couplings and field (Ising, Potts)              */
    double beta;                 /* inverse temperature (Ising, Potts), >= 0         */
    uint32_t rid;                /* replica id: selects the random streams          */
    /* Cellular Potts only */
    int32_t n_types;             /* 1..4, type 0 = medium                           */
    const float *adhesion;       /* host [n_types * n_types], symmetric             */
    const int8_t *cell_type;     /* host [q + 1], cell_type[0] = 0                  */
    const int32_t *target_area;  /* host [q + 1] (entry 0 unused)                   */
    float lambda_area;           /* >= 0                                            */
    double temperature;          /* > 0                                             */
    int32_t cpm_range;           /* neighbourhood of the adhesion sum and of the
                                    copy source: 0 or 1 = Moore 3x3 (2x2
                                    sublattice, 4 passes per step, neighbour =
                                    bits 0..2 of the main word); 2 = 5x5, the
                                    second shell added (3x3 sublattice, 9 passes
                                    c = 3 (y % 3) + x % 3 per step, p = 9t + c,
                                    k = (y/3) Lx/3 + x/3, neighbour j of 24 in
                                    row-major order by (u 24) >> 16 of the low 16
                                    bits u, or (f1 24) >> 32 with f1 word 1 of
                                    the fallback block when (u 24) mod 2^16 < 16;
                                    Lx, Ly multiples of 6).  One value for every
                                    replica of a context.                        */
    int32_t Lz;                  /* SPINMC_ISING_HC: third extent (0 or 1 = none) */
} spinmc_replica_desc;

/* Create a batch of n replicas (Methods, batched tensors: one context runs
 * many lattices or temperatures at once; Ising and Potts may be mixed; a CPM
 * context holds only CPM replicas).  Builds the FP64 Metropolis thresholds
 * T = ceil(2^32 exp(-beta dE)) of Algorithm 1 on the host, allocates the
 * lattices, and if init = 1 draws the initial state from the Philox init
 * stream (Ising: s = +1 iff the word < 2^31; Potts: floor(word q / 2^32)).
 * init = 0 leaves zeros (Ising all -1, Potts all 0, CPM all medium); CPM
 * states are set with spinmc_set_state.  hip_stream: a hipStream_t or NULL.
 * Errors: SPINMC_E_INVALID (shape, ranges, n < 1, duplicate rid),
 * SPINMC_E_NOT_REPRESENTABLE (CPM J or lambda not exact at S <= 256 below
 * 2^20), SPINMC_E_NOMEM, SPINMC_E_DEVICE (no GPU).  *out receives the
 * context, owned by the caller until spinmc_destroy.                        */
int spinmc_create(const spinmc_replica_desc *d, int32_t n, uint64_t seed, int32_t init,
                  void *hip_stream, spinmc_ctx **out);

/* Free every device buffer of the context.  Waits for its stream.  NULL is a
 * no-op.                                                                     */
int spinmc_destroy(spinmc_ctx *ctx);

/* Copy one replica's lattice from / to host memory, natural row-major:
 * Ising int8 in {-1, +1}, Potts uint8 in [0, q), CPM int32 in [0, n].
 * bytes must equal Lx*Ly*elem_size.  Synchronous (waits for the stream).
 * set_state validates every value first (SPINMC_E_INVALID leaves the state
 * unchanged); for CPM it also recomputes the cell areas.                    */
int spinmc_set_state(spinmc_ctx *ctx, int32_t replica, const void *host_buf, size_t bytes);
int spinmc_get_state(spinmc_ctx *ctx, int32_t replica, void *host_buf, size_t bytes);

/* Run n_sweeps sweeps (CPM: Monte Carlo steps) of every replica
 * (Algorithm 1 with the checkerboard colouring).  If record_every > 0 the
 * integer statistics after sweeps k*record_every (k = 1, 2, ...) are written
 * to dev_stats as int32 [n_sweeps / record_every][n_replicas][width], row
 * k-1.  dev_stats may be NULL only when record_every == 0.  Advances the
 * sweep counter by n_sweeps.  Asynchronous.  The work runs in the schedule
 * chosen by spinmc_set_schedule / spinmc_autotune; every schedule produces
 * the same bits.                                                            */
int spinmc_sweep(spinmc_ctx *ctx, int32_t n_sweeps, int32_t record_every, void *dev_stats);

/* Integer statistics of the current state into dev_stats int32 [n][width]
 * and, if dev_obs is not NULL, FP64 observables into dev_obs [n][4]:
 *   Ising (e, |m|, m^2, m) with e = -(Jx Bx + Jy By + h M)/N, m = M/N;
 *   Potts (e, m_P, S/N, 0) with e = -(Jx (Nx+Ny) + h S)/N and
 *         m_P = (q nmax / N - 1)/(q - 1);
 *   CPM   (H, 0, 0, 0) with H = (H*S)/S.   Asynchronous.                    */
int spinmc_measure(spinmc_ctx *ctx, void *dev_stats, void *dev_obs);

/* Fluctuation (covariance) estimator of the gradients of equilibrium Ising
 * observables; it replaces the logistic relaxation of Algorithm 2 (Methods)
 * with the exact identity d<O>/dtheta = <dO/dtheta> - beta Cov(O, dH/dtheta).
 * dev_stats: int32 [n_rec][n][width] as written by spinmc_sweep; samples
 * k >= burn_in are used.  Observables O = (e, |m|); parameters
 * theta = (Jx, Jy, h), dH/dJx = -Bx, dH/dJy = -By, dH/dh = -M.
 * Outputs (device FP64, any may be NULL): dev_means [n][4] =
 * (<e>, <|m|>, <m^2>, chi) with chi = beta N (<m^2> - <|m|>^2);
 * dev_grads [n][2][3] = d<O_o>/dtheta_j; dev_dtheta [n][3] =
 * sum_o dev_grad_out[n][o] * d<O_o>/dtheta (dev_grad_out FP64 [n][2],
 * required when dev_dtheta is set).  Moments are exact int64 sums combined
 * in FP64, so the result does not depend on how the sums are split.  From
 * 512 samples on, the context keeps a device buffer of chunk sums,
 * 104 B x n x ceil((n_rec - burn_in) / 64), allocated on the first call
 * that needs it (SPINMC_E_NOMEM if that fails) and kept for later calls.
 * Ising-only contexts.  Asynchronous.                                       */
int spinmc_grad(spinmc_ctx *ctx, const void *dev_stats, int32_t n_rec, int32_t burn_in,
                const void *dev_grad_out, void *dev_means, void *dev_grads, void *dev_dtheta);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * outputs as spinmc_grad, bit for bit, with the chunk sums in a static
 * per-device array of 4 MiB instead of a buffer the context allocates.  The
 * call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine); the array's device address is resolved once per device, at
 * spinmc_create or at the first call, with the context's device current.
 * Every record length takes the split form (chunks of 64 samples), so
 * n x ceil((n_rec - burn_in) / 64) x 104 B must not exceed 4 MiB
 * (SPINMC_E_INVALID otherwise; spinmc_grad has no such limit).  Each call
 * rewrites every entry it reads, so no state carries over between calls, but
 * all calls on one device share the array: calls that overlap in time on one
 * device (different streams or host threads) race and must be serialised by
 * the caller.  Arguments, outputs and errors otherwise as spinmc_grad.
 * Asynchronous.                                                             */
int spinmc_grad_noalloc(spinmc_ctx *ctx, const void *dev_stats, int32_t n_rec, int32_t burn_in,
                        const void *dev_grad_out, void *dev_means, void *dev_grads,
                        void *dev_dtheta);

/* Global sweep counter t (host mirror of the device counter).               */
int spinmc_sweep_counter(const spinmc_ctx *ctx, uint64_t *t);

/* int32 entries per replica in a statistics row (8 or 16).                 */
int spinmc_stats_width(const spinmc_ctx *ctx);

/* Number of replicas.                                                      */
int spinmc_num_replicas(const spinmc_ctx *ctx);

/* Copy replica r's Metropolis thresholds to host memory as uint64 values
 * T in [0, 2^32] (accept iff the uniform word W < T): Ising 18 entries
 * (index 9[s>0] + 3(Sx/2+1) + (Sy/2+1)), Potts 9(2q-1) (index
 * (dn+4)(2q-1) + (s'-s+q-1)), CPM K1 entries for k = 1..K1 (k >= K1 gives
 * T = 1 up to the first k with T = 0, reported in *aux).  *n_out receives
 * the entry count; cap is the capacity of host_T.                          */
int spinmc_thresholds(const spinmc_ctx *ctx, int32_t replica, uint64_t *host_T, int32_t cap,
                      int32_t *n_out, int64_t *aux);

/* Execution schedule of spinmc_sweep (the batched scheduler).
 * mode 1 resident: one persistent launch per group of replicas (one model
 *   and shape) for all sweeps of the call; each workgroup owns 1 to 16
 *   replicas whose lattices live in LDS for the whole call (lattices up to
 *   128 KiB); groups run concurrently on side streams.
 * mode 2 stream: one launch per colour pass over (replica, row-tile) units of
 *   every replica whose Lx/2 is a multiple of 16 (others go resident).
 * mode 3 hybrid: resident where the lattice fits the LDS budget, streamed
 *   otherwise; both run concurrently.
 * mode 0 auto: resident if every lattice fits, else hybrid.
 * Calls without recording replay cached hipGraphs of 50-sweep chunks of
 * the streamed passes; resident groups run one launch per group for all
 * sweeps of a call on side streams forked from and joined into the call's
 * stream, concurrently with the streamed work.
 * tile_rows: rows of a plane per streamed unit (even; 0 = about 16 KiB);
 * wg_threads: 256 or 512 (0 = default);
 * flags: 0, SPINMC_SCHED_NT_ON or SPINMC_SCHED_NT_OFF: streamed passes load
 *   and store their own colour plane with nontemporal hints (bypassing the
 *   caches, for lattice sets that do not fit the 256 MB last-level cache).
 *   0 decides per model: on when that model's streamed lattices exceed
 *   192 MiB.  The chain is the same either way.
 * SPINMC_SCHED_PERSIST (or-ed with the NT setting; modes 2 and 3 of Ising
 *   and Potts contexts, else SPINMC_E_UNSUPPORTED): unrecorded sweeps run
 *   the streamed replicas of each model in ONE launch per chunk instead of
 *   one per colour pass: an occupancy-sized grid of 256-thread workgroups,
 *   each owning whole replicas or one row slab of a replica cut into slabs
 *   (tile_rows rows, or 0 = slabs sized so that the slab workgroups fill the
 *   chip once); a slab starts a pass once the slabs above and below it have
 *   published the previous one (per-slab pass counters, no grid barrier).
 *   Recorded sweeps keep one launch per pass.  A wait that runs past its
 *   bound (which only a slab workgroup that never became resident could
 *   cause) ends the launch early; the next spinmc_get_state then returns
 *   SPINMC_E_DEVICE and poisons the context.
 * CPM contexts with the 3x3 neighbourhood: SPINMC_SCHED_PERSIST runs the
 *   unrecorded steps of replicas of one shape (Lx a multiple of 8) as tiled
 *   persistent passes: one launch per chunk of up to 500 steps, a workgroup
 *   per tile (tile_rows rows, or 64, by up to 64 columns) holding its ids in
 *   LDS, neighbouring tiles exchanging their border cells through the
 *   lattice at a per-replica barrier after every pass; when the tiles do not
 *   divide the lattice or cannot all be resident at once, the streamed passes
 *   run instead.  A barrier wait past its bound poisons the context as above.
 * Invalid values return SPINMC_E_INVALID.  CPM contexts: mode 2 keeps every
 * step on streamed passes; any other mode lets the unrecorded steps of
 * lattices whose ids and tables fit 64 KiB of LDS run resident (one
 * workgroup per replica).  tile_rows is rounded down to whole periods of
 * the colouring (2 rows, or 6 with the 5x5 neighbourhood).  wg_threads of
 * a streamed 3x3 pass where every Lx is a multiple of 8: 0 = one site per
 * lane in workgroups of 1024 (tiles of about 8192 sites by default), 512 =
 * the same in workgroups of 512, 256 = four same-colour sites per lane in
 * workgroups of 256 (tiles of about 4096 sites); the same decisions either
 * way.  Other CPM passes use at most 256 threads.  spinmc_autotune tries
 * both forms of the 3x3 pass, and for Ising and Potts contexts also the
 * best streaming schedule with NT forced on and off.                        */
enum { SPINMC_SCHED_NT_ON = 1, SPINMC_SCHED_NT_OFF = 2, SPINMC_SCHED_PERSIST = 4 };
typedef struct spinmc_schedule {
    int32_t mode;
    int32_t tile_rows;
    int32_t wg_threads;
    int32_t flags;
    int32_t rpb;     /* replicas per resident workgroup: 0 = packing rule, else a
                      * power of two up to 8 (capped by the LDS budget, by one
                      * wave per replica and by the group's size)              */
} spinmc_schedule;

int spinmc_set_schedule(spinmc_ctx *ctx, const spinmc_schedule *s);
int spinmc_get_schedule(const spinmc_ctx *ctx, spinmc_schedule *s);

/* Sites per sweep that the current schedule streams through colour-pass
 * launches and that it keeps resident in LDS, per model: streamed[m] and
 * resident[m] for m = SPINMC_ISING, SPINMC_POTTS, SPINMC_CPM (host arrays of
 * 3 entries each, written in full).                                         */
int spinmc_schedule_sites(const spinmc_ctx *ctx, int64_t streamed[3], int64_t resident[3]);

/* Time candidate schedules for trial_sweeps sweeps each on a scratch copy of
 * the state (the context's state and counter are restored afterwards), pick
 * the fastest, store it, and return it in *chosen (may be NULL) with the
 * measured attempts per ns of every candidate in host_rates (capacity cap,
 * may be NULL; *n_tried receives the count).  If chosen is not NULL and
 * chosen->mode > 0 on entry, only candidates of that mode are tried.
 * The candidates: modes, tile heights, workgroup sizes, persistent passes,
 * then nontemporal access forced on and off for the best streaming
 * candidate and replicas per resident workgroup 1, 2, 4 and 8 for the best
 * candidate with resident groups.  The three fastest then run again, twice
 * each for 4 trial_sweeps sweeps (not reported in host_rates), and the best
 * of those runs is chosen: short trials of close candidates differ by
 * timing noise.  Choices are cached per process, keyed by
 * the device's architecture and compute-unit count and the context's shape
 * signature (model, Lx, Ly, q and the multiplicity of every shape, CPM
 * neighbourhood range): a later call for an equal signature returns the
 * cached schedule without trials (*n_tried = 0) unless chosen->mode is -1 on
 * entry.  With the environment variable SPINMC_AUTOTUNE_CACHE naming a file,
 * the cache is also read from and appended to that file (one line per
 * choice).  Synchronous.                                                     */
int spinmc_autotune(spinmc_ctx *ctx, int32_t trial_sweeps, spinmc_schedule *chosen,
                    double *host_rates, int32_t cap, int32_t *n_tried);

const char *spinmc_last_error(void);

/* Kernel timing with HIP events, for benchmarks.  spinmc_profile(ctx, 1)
 * clears the record and brackets every following sweep-kernel launch with a
 * pair of events on the stream it is launched on (sweeps then run without
 * graph replay); spinmc_profile(ctx, 0) stops.  spinmc_profile_read waits
 * for the recorded events and returns, for one kernel class, the summed
 * elapsed milliseconds and the launch count.                                */
enum spinmc_kernel_kind {
    SPINMC_K_STREAM_ISING = 0,  /* streamed Ising colour pass                 */
    SPINMC_K_RESIDENT = 1,      /* resident multi-sweep kernel (all groups)   */
    SPINMC_K_CPM_PASS = 3,      /* CPM colour pass                            */
    SPINMC_K_STREAM_POTTS = 4,  /* streamed Potts colour pass                 */
    SPINMC_K_TRI_PASS = 5,      /* triangular-lattice Ising colour pass       */
    SPINMC_K_HC_PASS = 6,       /* chain / cubic Ising colour pass            */
    SPINMC_K_MSC_PASS = 7,      /* multispin-coded Ising colour pass          */
    SPINMC_K_PERSIST_ISING = 8, /* persistent streamed Ising chunk            */
    SPINMC_K_PERSIST_POTTS = 9, /* persistent streamed Potts chunk            */
    SPINMC_K_CPM_TILED = 10     /* tiled persistent CPM chunk                 */
};
int spinmc_profile(spinmc_ctx *ctx, int32_t enable);
int spinmc_profile_read(spinmc_ctx *ctx, int32_t kind, double *ms_total, int64_t *launches);

/* ------------------------------------------------------------------------
 * Surrogate MLP 4-128-128-3 (SiLU), BF16 weights and activations with FP32
 * accumulation on MFMA.  Maps normalised (beta, Jx, Jy, h) to normalised
 * (<e>, <|m|>, chi).  Parameters live in one caller-owned FP32 device buffer
 * of spinmc_mlp_num_params() floats (layout: W1[128][4], b1[128],
 * W2[128][128], b2[128], W3[3][128], b3[3]); the BF16 copies used by the
 * matrix cores are rounded from it (round to nearest even) by every call.
 * Adam follows the paper's optimiser settings by default (Results,
 * optimisation: learning rate 1e-3, betas 0.9 / 0.999).                    */
int spinmc_mlp_num_params(void);

/* y[B][3] = MLP(x[B][4]) (device FP32).  dev_act may be NULL; otherwise it
 * receives the pre-activations the backward pass needs, FP32
 * [B][256] = spinmc_mlp_act_floats(B) floats.  B >= 1.                     */
int spinmc_mlp_act_floats(int32_t B);
int spinmc_mlp_forward(const void *dev_params, const void *dev_x, int32_t B, void *dev_y,
                       void *dev_act, void *hip_stream);

/* Gradients of L = (1/B) sum_b sum_j w_j (y_bj - t_bj)^2 with respect to the
 * parameters (dev_grad, FP32, same layout as the parameters) and optionally
 * the inputs (dev_dx [B][4], may be NULL).  dev_act from the forward call of
 * the same x.  dev_loss (FP32 scalar, may be NULL) receives L.  Per-output
 * weights dev_w [3] (FP32).  dev_workspace: FP32
 * [spinmc_mlp_workspace_floats(B)] of per-workgroup partial sums, reduced in
 * a fixed order (deterministic).                                            */
int spinmc_mlp_workspace_floats(int32_t B);
int spinmc_mlp_backward(const void *dev_params, const void *dev_x, const void *dev_act,
                        const void *dev_t, const void *dev_w, int32_t B, void *dev_grad,
                        void *dev_dx, void *dev_loss, void *dev_workspace, void *hip_stream);

/* One training step in one call: spinmc_mlp_forward (pre-activations into
 * dev_act, [B][256] FP32), spinmc_mlp_backward (no input gradient) and
 * spinmc_mlp_adam, with the fixed-order reduction of the partial gradients
 * and the Adam update fused into one kernel: the same arithmetic in the same
 * order as the three calls, so the parameters, moments, dev_grad (may be
 * NULL) and dev_loss (may be NULL) equal theirs bit for bit.  Arguments as
 * in those calls.                                                           */
int spinmc_mlp_train_step(void *dev_params, const void *dev_x, const void *dev_t,
                          const void *dev_w, int32_t B, void *dev_grad, void *dev_m,
                          void *dev_v, int32_t step, float lr, float beta1, float beta2,
                          float eps, void *dev_loss, void *dev_act, void *dev_workspace,
                          void *hip_stream);

/* One Adam step on the FP32 parameters: m, v (FP32, same size) are the
 * moment buffers, step >= 1 the 1-based step number.                        */
int spinmc_mlp_adam(void *dev_params, const void *dev_grad, void *dev_m, void *dev_v,
                    int32_t step, float lr, float beta1, float beta2, float eps,
                    void *hip_stream);

/* One Adam step on n FP32 parameters (any buffer): m, v the moment buffers
 * of the same size, step >= 1 the 1-based step number.  Used by the
 * optimisation experiments (Results: Adam, learning rate 1e-3).            */
int spinmc_adam(void *dev_params, const void *dev_grad, void *dev_m, void *dev_v, int64_t n,
                int32_t step, float lr, float beta1, float beta2, float eps, void *hip_stream);

/* ------------------------------------------------------------------------
 * Differentiable Monte Carlo (Methods, Algorithm 2) for the Ising model:
 * the relaxed checkerboard chain on continuous spins s in [-1, 1] with one
 * coupling per bond, and its reverse-mode gradient.  Per colour pass
 * (colour c = (x+y) & 1 first c = 0, pass p = 2t + c), every site of colour c:
 *   hloc = Jx[y][x] s(y,x+1) + Jx[y][x-1] s(y,x-1) + Jy[y][x] s(y+1,x)
 *          + Jy[y-1][x] s(y-1,x) + h                     (periodic),
 *   P = exp(min(-beta * 2 s hloc, 80))   (energy change of the flip
 *       proposal; past the cap q is exactly 1 either way),
 *   q = 1 / (1 + exp(-alpha (P - r))),   s <- q (-s) + (1 - q) s,
 * r = (w >> 8) 2^-24 with w word k & 3 of Philox4x32-10 counter
 * (k >> 2, p, rid0 + replica, 3), key (seed lo, seed hi), k = y Lx/2 + x>>1.
 * alpha -> infinity recovers the Metropolis chain.  FP32 arithmetic.
 * Buffers (caller-owned device memory, row-major [R][Ly][Lx] FP32): spins,
 * Jx (bond (y,x)-(y,x+1)), Jy (bond (y,x)-(y+1,x)).  Invalid arguments
 * return SPINMC_E_INVALID before anything is enqueued.                      */
typedef struct spinmc_dmc_params {
    int32_t R, Lx, Ly, n_sweeps;   /* replicas, even Lx and Ly >= 2, sweeps >= 0 */
    float beta, alpha, h, reserved; /* alpha >= 0                                 */
    uint64_t seed, t0;              /* Philox key, first sweep counter            */
    uint32_t rid0, reserved2;       /* replica ids rid0 .. rid0 + R - 1           */
} spinmc_dmc_params;

/* Sizes (floats) of the forward's save buffer (pre-pass spins of the
 * updated colour, 2 n_sweeps R Ly Lx/2) and of the backward's work buffer
 * (dL/dhloc of two consecutive passes, 2 R Ly Lx/2); negative on invalid
 * parameters.  Buffers with 16-byte aligned addresses and Lx a multiple of
 * 8 take the vectorised kernels; any other case takes per-site kernels with
 * the same results.                                                         */
int64_t spinmc_dmc_save_floats(const spinmc_dmc_params *p);
int64_t spinmc_dmc_work_floats(const spinmc_dmc_params *p);

/* n_sweeps relaxed sweeps of dev_s in place; dev_save receives what the
 * backward replay needs.                                                    */
int spinmc_dmc_forward(const spinmc_dmc_params *p, void *dev_s, const void *dev_Jx,
                       const void *dev_Jy, void *dev_save, void *hip_stream);

/* Reverse replay of the forward call with the same parameters: on entry
 * dev_s holds the final spins and dev_gs = dL/ds_final; on exit dev_s holds
 * the initial spins and dev_gs = dL/ds_initial; dL/dJx and dL/dJy are added
 * to dev_gJx, dev_gJy.                                                      */
int spinmc_dmc_backward(const spinmc_dmc_params *p, void *dev_s, const void *dev_Jx,
                        const void *dev_Jy, const void *dev_save, void *dev_gs, void *dev_gJx,
                        void *dev_gJy, void *dev_work, void *hip_stream);

/* ------------------------------------------------------------------------
 * Spin-value optimisation (Results, optimisation of the spin values): the
 * energy the methods minimise and the quantised update.
 *
 * Energy of the spins dev_s with the couplings of p's layout (R, Lx, Ly;
 * field p->h; the other fields of p are not used):
 *   H = -sum_{y,x} s[y][x] (Jx[y][x] s[y][x+1] + Jy[y][x] s[y+1][x]) - h sum s
 * into dev_energy (double[R], summed in FP64 in a fixed order, so repeated
 * calls agree bit for bit) and, if dev_grad is not null, dH/ds =
 * -(local field of the relaxed chain) into dev_grad (FP32 [R][Ly][Lx]).   */
int spinmc_dmc_energy(const spinmc_dmc_params *p, const void *dev_s, const void *dev_Jx,
                      const void *dev_Jy, void *dev_energy, void *dev_grad, void *hip_stream);

/* The discretisation of Algorithm 2 after a gradient step on n FP32 values:
 * out = -1 where base - eta g < 0, +1 elsewhere (dev_g null: base alone).
 * dev_out may equal dev_base.  0 <= n <= 2^31, eta finite.                */
int spinmc_dmc_discretize(int64_t n, const void *dev_base, const void *dev_g, float eta,
                          void *dev_out, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* SPINMC_H */
