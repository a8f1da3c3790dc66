/*
 * pa.h -- C ABI of an MI355X (gfx950) library for population annealing (PA)
 * of the two-dimensional q-state Potts model.
 *
 * Method: Barash, Weigel, Shchur, Janke, "Exploring first-order phase
 * transitions with population annealing", arXiv:1704.01888.
 *   Sec. 2, steps 1-5 : the PA loop (initial population, resampling with the
 *                       relative Boltzmann weights, theta Metropolis rounds,
 *                       population averages, next temperature);
 *   Sec. 2, eq. (1)   : Poisson copy numbers, R_i = sum_j r_j;
 *   Sec. 2, eq. (2)   : free-energy estimator -beta_i F = ln Z_beta0 + sum ln Q_m;
 *   Sec. 3, eq. (3)   : H = -sum_<ij> delta(s_i, s_j), J = 1, periodic L x L;
 *   Sec. 3, eq. (4)   : population averages;
 *   Sec. 5, eq. (6)   : ground-state initial population (heating runs);
 *   Sec. 6, eq. (7)-(8): ln Z at beta -> infinity = ln q - beta E_0, E_0 = -2N.
 *
 * Conventions fixed by this library where the paper leaves a choice open
 * (all of them are also implemented, independently, by the CPU oracle):
 *   - spins are uint8 in 0..q-1, replica-major, row-major (site n = y*L + x);
 *   - random words: Philox4x32-10 keyed by (seed low 32 bits, seed high 32
 *     bits); the counter is (index within unit, slot, step, domain << 28 |
 *     sub-index), so every random number is a pure function of logical
 *     indices and never of threads, tiles or launches;
 *   - one Metropolis round = one checkerboard sweep: colour 0 ((x+y) even)
 *     then colour 1; proposal uniform over the q-1 other states; acceptance
 *     iff dE <= 0 or w < floor(2^32 exp(-beta dE));
 *   - Poisson resampling is drawn as R_i ~ Pois(R) (from the plan) followed by
 *     R_i multinomial draws with integer weights round(2^Kb exp(-|dbeta| d_j)),
 *     d_j = |E_j - E_ref|; this is the same joint law as eq. (1) because the
 *     Poisson means add up to R;
 *   - the new population is stored in ancestor order;
 *   - histogram widths (Sec. 4): bins of bin_e energy levels (bin_m levels of
 *     M~) counted from E = -2N (M~ = 0); the histogram is taken as the
 *     piecewise-linear curve through the bin counts (zero beyond both ends),
 *     and the width is the distance between its outermost crossings of half
 *     the largest count, converted to e = E/N or m = M/N units.
 *
 * Floating point: the device evaluates in FP64 only the ln Q_i terms and their
 * running sum -beta_i F (eq. (2)); the population averages (eq. (4)-(5)) and
 * the histogram widths are formed on the host from the exact integer sums and
 * histogram counts the device produces.
 *
 * Memory ownership: device memory belongs to the caller.  The library only
 * sub-allocates inside the workspace d_ws (device pointer, at least
 * pa_plan_info.workspace_bytes bytes, 256-byte aligned), which must stay
 * valid until pa_run_finish returns.  All host pointers passed in are read
 * during the call only; result buffers are caller-owned host memory.
 * "stream" is a hipStream_t (NULL = the null stream); all device work of a
 * run is ordered on it.
 *
 * Errors: every call returns pa_status; nothing throws across the ABI.
 * pa_last_error() gives a thread-local message for the last failure.
 * A device error (PA_ERR_DEVICE) leaves the run unusable; finish it.
 */
#ifndef PA_H
#define PA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PA_OK = 0,
    PA_ERR_INVALID = -1,   /* bad argument or description                          */
    PA_ERR_NOMEM = -2,     /* workspace smaller than pa_plan_info.workspace_bytes  */
    PA_ERR_DEVICE = -3,    /* HIP error or failed device-side consistency check    */
    PA_ERR_CAPACITY = -4,  /* the Poisson schedule drew R_i = 0 or R_i > 2^31      */
    PA_ERR_UNSUPPORTED = -5, /* valid for the method, outside this device path    */
    PA_ERR_BUSY = -6,      /* a server already runs on this context                */
    PA_ERR_CANCELLED = -7, /* request cancelled (pa_serve_cancel / pa_serve_stop)  */
    PA_ERR_TIMEOUT = -8    /* pa_serve_wait timed out; the request is still live   */
} pa_status;

typedef enum { PA_RESAMPLE_POISSON = 0, PA_RESAMPLE_MULTINOMIAL = 1, PA_RESAMPLE_NONE = 2 } pa_resample;
typedef enum { PA_INIT_RANDOM = 0, PA_INIT_GROUND = 1 } pa_init;

/* Output selection bits for pa_run_desc.outputs. */
enum {
    PA_OUT_HIST = 1,   /* per-step energy histograms, [K][2N+1] (and, with
                          PA_OUT_MAG, M~ histograms [K][N+1])              */
    PA_OUT_MAG = 2,    /* magnetisation, eq. (4)-(5): sum of M~ and M-bar   */
    PA_OUT_FINAL = 4,  /* final population, energies and last ancestors  */
    PA_OUT_WIDTHS = 8, /* full width at half maximum of the energy histogram
                          (and, with PA_OUT_MAG, of the magnetisation
                          histogram) at every step, Sec. 4              */
    PA_OUT_DIGEST = 16 /* a 64-bit digest of the whole population at every
                          step (see pa_result.digest)                   */
};

/* A PA run (Sec. 2): lattice L x L periodic (Sec. 3), q states, target
 * population R, inverse temperatures beta[0..K-1], theta sweeps per step. */
typedef struct {
    uint32_t L;          /* lattice side, even, 2 <= L <= 4096 on this device path, and
                            L <= 254 when L is not a multiple of 4 (L <= 256: replicas in
                            LDS, one wave per replica byte by byte when L = 2 mod 4; larger
                            L: tiled half-sweeps with the replicas in HBM and a third
                            population buffer in the workspace) */
    uint32_t q;          /* 2 <= q <= 255                                               */
    uint64_t R;          /* 1 <= R <= 2^31                                              */
    uint32_t K;          /* number of temperatures, K >= 1                              */
    const double *beta;  /* [K] host array, finite and >= 0; random init needs beta[0] == 0 */
    uint32_t theta;      /* Metropolis sweeps per step, < 2^27                          */
    uint64_t seed;       /* Philox key                                                  */
    int32_t resample;    /* pa_resample                                                 */
    int32_t init;        /* pa_init                                                     */
    uint32_t outputs;    /* PA_OUT_* bits                                               */
    uint32_t bin_e;      /* PA_OUT_WIDTHS: energy levels per histogram bin (0 means 1)  */
    uint32_t bin_m;      /* PA_OUT_WIDTHS: M~ levels per histogram bin (0 means 1)      */
} pa_run_desc;

/* Kernel kinds, for the optional per-kernel timing of pa_result. */
enum {
    PA_KERNEL_INIT = 0,     /* initial population + energies (step 1)               */
    PA_KERNEL_SWEEP = 1,    /* gather + theta sweeps + energies (eq. (1), step 3)   */
    PA_KERNEL_POST = 2,     /* sums, E_ref, ln Q (eq. (2), (4)) + weight scan (step 2) */
    PA_KERNEL_RESAMPLE = 3, /* multinomial draws + copy numbers -> ancestors (eq. (1)) */
    PA_KERNEL_KINDS = 4
};

/* Host result buffers, caller-allocated; arrays of length K unless noted. */
typedef struct {
    uint64_t *R_i;           /* population size after each step                    */
    int64_t  *E_sum;         /* exact integer sum of the energies                  */
    double   *E_mean;        /* eq. (4): E_sum / R_i                               */
    double   *lnQ;           /* ln Q_i of Sec. 2 step 2; lnQ[0] = 0                */
    double   *minus_beta_F;  /* eq. (2) with ln Z_beta0 (N ln q, or eq. (7)-(8))   */
    uint32_t *hist;          /* [K][2N+1], h[b] = #{j: E_j = b - 2N}; NULL unless PA_OUT_HIST */
    int64_t  *Mt_sum;        /* PA_OUT_MAG: exact sum over the population of M~ (eq. (5)) */
    double   *M_mean;        /* PA_OUT_MAG: eq. (4)-(5), M-bar = (q Mt_sum - N R_i) / ((q-1) R_i),
                                one rounding                                         */
    uint32_t *mhist;         /* [K][N+1], #{j: M~_j = m}; PA_OUT_MAG with PA_OUT_HIST */
    double   *width_e;       /* PA_OUT_WIDTHS: FWHM of the histogram of e = E/N       */
    double   *width_m;       /* PA_OUT_WIDTHS with PA_OUT_MAG: FWHM of the histogram of m = M/N */
    uint64_t *digest;        /* PA_OUT_DIGEST: sum over slots k < R_i and dwords n < N/4 of
                                r * d mod 2^64, d = spins 4n..4n+3 of slot k (little endian),
                                r = (w1 << 32 | w0) | 1 with w = Philox(n, k, i, 5 << 28);
                                equal populations in equal slots give equal digests, and any
                                single changed dword changes the digest              */
    uint8_t  *final_spins;   /* [R_{K-1}][N]; NULL unless PA_OUT_FINAL; the final_* and
                                last_anc buffers are written only by a run that has
                                reached its last temperature                          */
    int32_t  *final_E;       /* [R_{K-1}];     NULL unless PA_OUT_FINAL              */
    uint32_t *last_anc;      /* [R_{K-1}] ancestors of the last resampling (identity if K == 1) */
    double   *kernel_ms;     /* [PA_KERNEL_KINDS] summed HIP-event time per kernel kind, or NULL;
                                filled only when profiling is on (pa_ctx_set_profiling) */
    uint64_t *kernel_launches; /* [PA_KERNEL_KINDS] launches per kind, or NULL          */
} pa_result;

typedef struct {
    uint64_t R_cap;            /* largest population of the run                     */
    uint64_t R_final;          /* R_{K-1}                                           */
    uint64_t workspace_bytes;  /* device bytes pa_run / pa_run_begin need            */
    uint32_t Kb;               /* weight precision: 63 - ceil(log2 R_cap)           */
    uint32_t n_tables;         /* distinct |beta_i - beta_{i-1}| values             */
} pa_plan_info;

typedef struct pa_ctx pa_ctx;          /* device handle                           */
typedef struct pa_run_state pa_run_state; /* one run in flight                     */

/* Plan a run on the host (no device work): validates the description, draws
 * the population schedule (Sec. 2 eq. (1), see the header comment) and sizes
 * the workspace. */
pa_status pa_plan(const pa_run_desc *desc, pa_plan_info *info);

/* The plan's integer tables, for checking against an independent
 * implementation: T[K][4] Metropolis thresholds floor(2^32 exp(-beta_i dE)),
 * dE = 1..4 (Sec. 2 step 3); R_sched[K] population sizes (R_sched[0] = R).
 * Either pointer may be NULL. */
pa_status pa_plan_tables(const pa_run_desc *desc, uint64_t *T, uint64_t *R_sched);

/* Integer resampling weights W[d] = round(2^Kb exp(-|dbeta| d)), d = 0..2N, as
 * the library builds them; returns the table length D (first zero) in *D. */
pa_status pa_weight_table(double abs_dbeta, uint32_t Kb, uint32_t N, uint64_t *W, uint32_t *D);

/* Device handle on HIP device `device`. */
pa_status pa_ctx_create(int device, pa_ctx **out);
void pa_ctx_destroy(pa_ctx *ctx);
/* Bracket every kernel launch of later runs with HIP events on the run's
 * stream and report the summed durations in pa_result.kernel_ms. */
pa_status pa_ctx_set_profiling(pa_ctx *ctx, int enable);

/* Sweep kernel shape.  For L a power of two up to 256 and for L = 12, 20, 24,
 * 48, 96, 192 the sweep kernel exists for one or two lane counts per replica
 * (a divisor of 64: several replicas per wave; a multiple of 64: one replica
 * per workgroup; neither, at L = 12, 20, 24: replicas spanning waves, several
 * per workgroup); results do not depend on the choice.  Other L use one
 * generic shape.  pa_ctx_get_lanes reports the lanes later runs will use and
 * the candidates (0 lanes and no candidates for the tiled path, L > 256);
 * pa_ctx_set_lanes picks one (0 = default) for later runs.
 * pa_autotune times every candidate on a synthetic population of about 64 MB
 * (K = 3, theta = 4) in the caller's workspace (at least pa_plan's size for
 * it; 256 MB is enough for every L), keeps the fastest in the context and
 * returns it with its sweep rate. */
pa_status pa_ctx_set_lanes(pa_ctx *ctx, uint32_t L, uint32_t lanes);
pa_status pa_ctx_get_lanes(pa_ctx *ctx, uint32_t L, uint32_t *lanes, uint32_t *candidates /*[2]*/,
                           uint32_t *n_candidates);
pa_status pa_autotune(pa_ctx *ctx, uint32_t L, uint32_t q, void *d_ws, uint64_t ws_bytes, void *stream,
                      uint32_t *best_lanes, double *best_attempts_per_ns);

/* Tuned sweep shapes.  An entry gives, for lattice side L, a q class (q_large:
 * q above 128, the other form of the neighbour comparison) and a population
 * class (r_class: R_cap below 2^11, 2^14, 2^17, or above), the lanes per
 * replica and the waves per workgroup of the sweep kernel.  Later runs on the
 * context whose description falls in an entry's class sweep with its shape --
 * pa_run, pa_run_batch and the serving loop alike -- unless pa_ctx_set_lanes
 * fixed a lane count for L; results do not depend on the shape.  Lattices on
 * the tiled path (L > 256) have no shape.
 * pa_tune: times every shape of L (each lane count with a kernel for L; for
 *   each, the waves per workgroup that fit 1024 threads, 256 for L = 2 mod 4,
 *   and the LDS) on a synthetic run of R replicas (K = 3, theta = 10) in the
 *   caller's workspace (at least pa_plan's size for that run), keeps the
 *   fastest as the entry of (L, q, R)'s class and returns it with its rate;
 *   `timed` (may be NULL) receives up to timed_cap of the shapes with their
 *   rates, *n_timed the number of shapes timed.  Calls on the context must
 *   not overlap it.
 * pa_tune_set: installs an entry (PA_ERR_INVALID if it is not a shape of L).
 * pa_tune_get: the shape later runs of (L, q, R) will use (the entry, or the
 *   default with attempts_per_ns 0).
 * pa_tune_save / pa_tune_load: the context's entries as a text file, one JSON
 *   object per line with the keys arch, L, q_large, r_class, lanes,
 *   waves_per_block and attempts_per_ns; loading keeps the lines of this
 *   device's architecture (e.g. "gfx950") and refuses a file with a malformed
 *   line or a shape its lattice side does not have (nothing is installed
 *   then). */
typedef struct {
    uint32_t L, q_large, r_class;      /* the class */
    uint32_t lanes, waves_per_block;   /* its shape */
    double attempts_per_ns;            /* measured sweep rate (0 if not measured) */
} pa_tune_entry;
pa_status pa_tune(pa_ctx *ctx, uint32_t L, uint32_t q, uint64_t R, void *d_ws, uint64_t ws_bytes, void *stream,
                  pa_tune_entry *best, pa_tune_entry *timed, uint32_t timed_cap, uint32_t *n_timed);
pa_status pa_tune_set(pa_ctx *ctx, const pa_tune_entry *entry);
pa_status pa_tune_get(pa_ctx *ctx, uint32_t L, uint32_t q, uint64_t R, pa_tune_entry *entry);
pa_status pa_tune_save(pa_ctx *ctx, const char *path);
pa_status pa_tune_load(pa_ctx *ctx, const char *path, uint32_t *n_loaded);

/* Whole run, steps 1-5 of Sec. 2, enqueued on `stream`; returns when the
 * results are in `out`. */
pa_status pa_run(pa_ctx *ctx, const pa_run_desc *desc, void *d_ws, uint64_t ws_bytes,
                 void *stream, pa_result *out);

/* Allocation-free form of pa_run, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops that forbid allocation):
 * the workspace is a device array of PA_STATIC_SCRATCH_BYTES that the library
 * holds on every GPU it runs on until the process ends, so the call makes no
 * device allocation.  PA_ERR_NOMEM if the run's pa_plan workspace_bytes exceed
 * it.  Every call on one GPU uses that GPU's array, which keeps the previous
 * call's contents (a run clears what must start at zero): calls that overlap
 * on one GPU, from any thread or context, race.  Per-kernel timing
 * (pa_ctx_set_profiling) is not recorded by this call. */
#define PA_STATIC_SCRATCH_BYTES (64ull << 20)
pa_status pa_run_static(pa_ctx *ctx, const pa_run_desc *desc, void *stream, pa_result *out);

/* Stepwise form of pa_run.
 * pa_run_begin: plan, upload tables, create the initial population (step 0).
 * pa_run_advance: enqueue the next n steps (resampling + theta sweeps + stats).
 * pa_run_sync: wait for the enqueued work.
 * pa_run_read: synchronous copy of the current population (any pointer NULL
 *   to skip): spins[R_cur][N], E[R_cur], anc[R_cur] (ancestors of the last
 *   resampling), counts[R_prev] (copy numbers of the last resampling).
 * pa_run_read_free_energy: synchronous read of the current step and its
 *   -beta F (eq. (2), accumulated so far).
 * pa_run_load: replace the current population by host spins[R_cur][N] at step
 *   `step` with -beta F value minus_beta_F (resume from a checkpoint: the
 *   population and -beta F of pa_run_read and pa_run_read_free_energy at that
 *   step; the continuation is bit-identical, and pa_run_finish then reports
 *   the steps from `step` on).
 * pa_run_read_slots: see below.
 * pa_run_finish: wait, copy the per-step results into `out` (may be NULL) and
 *   release the run. */
pa_status pa_run_begin(pa_ctx *ctx, const pa_run_desc *desc, void *d_ws, uint64_t ws_bytes,
                       void *stream, pa_run_state **out);
pa_status pa_run_advance(pa_run_state *run, uint32_t n_steps);
pa_status pa_run_sync(pa_run_state *run);
pa_status pa_run_read(pa_run_state *run, uint32_t *step, uint64_t *R_cur, uint64_t *R_prev,
                      uint8_t *spins, int32_t *E, uint32_t *anc, uint32_t *counts);
pa_status pa_run_read_free_energy(pa_run_state *run, uint32_t *step, double *minus_beta_F);
pa_status pa_run_load(pa_run_state *run, uint32_t step, uint64_t R_cur, const uint8_t *spins,
                      double minus_beta_F);
/* Synchronous copy of n selected replicas: from the current population
 * (previous == 0) or from the population before the last step (previous == 1,
 * valid until the next pa_run_advance).  spins_out is [n][N]. */
pa_status pa_run_read_slots(pa_run_state *run, int previous, const uint32_t *slots, uint32_t n,
                            uint8_t *spins_out);
pa_status pa_run_finish(pa_run_state *run, pa_result *out);

/* Checkpoints.  A run's population at its current step, with -beta F of that
 * step (eq. (2), accumulated so far) and the run description, in a binary file
 * that a new run -- on this library or on any other implementation of the same
 * conventions -- continues bit-identically (every random number is a function
 * of logical indices; the weights, thresholds and population schedule follow
 * from the description).  Results of the continued run are valid from the
 * checkpoint's step on.
 *
 * File format (little-endian, 128-byte header, then beta, then the spins):
 *   offset  type    field
 *        0  char[8] magic "PACKPT01"
 *        8  u32     header size, 128
 *       12  u32     L        16  u32  q        20  u32  K
 *       24  u64     R        32  u32  theta    36  i32  resample (pa_resample)
 *       40  u64     seed     48  i32  init     52  u32  outputs
 *       56  u32     bin_e    60  u32  bin_m
 *       64  u32     step i of the population (0 <= i < K)
 *       68  u32     zero
 *       72  u64     R_i, replicas in the population
 *       80  f64     -beta_i F_i
 *       88  i64     sum of the energies of the population (eq. (3)), a check
 *       96  zero up to byte 128
 *      128  f64[K]  beta_0 .. beta_{K-1}
 *  128+8K  u8[R_i][L*L]  spins 0..q-1, replica-major, row-major (slot order)
 *
 * pa_checkpoint: write the run's current state to `path` (waits for the run's
 *   enqueued work).  PA_ERR_INVALID if the file cannot be written.
 * pa_checkpoint_info: the description of a checkpoint (desc->beta points to
 *   `beta` when beta_cap >= K, else NULL; PA_ERR_NOMEM if `beta` is given but
 *   shorter than K, with desc->K set), its step and population size -- enough
 *   to size the workspace with pa_plan before pa_resume.
 * pa_resume: a new run in d_ws continued from the checkpoint (like
 *   pa_run_begin followed by pa_run_load); PA_ERR_INVALID for a malformed or
 *   truncated file or when the energies recomputed from the spins do not add up
 *   to the stored sum. */
pa_status pa_checkpoint(pa_run_state *run, const char *path);
pa_status pa_checkpoint_info(const char *path, pa_run_desc *desc, double *beta, uint32_t beta_cap,
                             uint32_t *step, uint64_t *R_cur);
pa_status pa_resume(pa_ctx *ctx, const char *path, void *d_ws, uint64_t ws_bytes, void *stream,
                    pa_run_state **out);

/* Batched runs: n independent PA runs (any mix of L, q, R, K, theta, seeds,
 * resampling and init modes) advanced together, one set of segmented launches
 * per global step g for every run with K > g.  The runs start together (one
 * launch of fills and weight-table copies, one initial sweep launch per kernel
 * class, one launch of step-0 statistics) and their per-step results come back
 * through one gathering launch and one copy.  Results are identical to n
 * separate pa_run calls.  pa_plan_batch gives the workspace size (the runs'
 * workspaces, the descriptor tables of the start, the steps and the read-back,
 * and the gathering area); outs[n] as in pa_run. */
pa_status pa_plan_batch(const pa_run_desc *descs, uint32_t n, uint64_t *workspace_bytes);
/* With graphs enabled, pa_run_batch records its per-step launch sequence once
 * as a HIP graph (on a stream of the context, ordered after the caller's
 * stream by events) and replays it for later calls with the same
 * descriptions, workspace and kernel shapes (up to 8 cached graphs). */
pa_status pa_ctx_set_graphs(pa_ctx *ctx, int enable);
/* Batch modes.  PA_BATCH_SEGMENTED (the default): the launches above, one
 * set per global step.  PA_BATCH_TEAM: the runs whose every remaining step fits
 * one workgroup's sweep class, with populations up to 8192 replicas and no
 * 64-bit thresholds, go through all their steps in one cooperative launch per
 * sweep class and workgroup size -- each run a team of workgroups that meet
 * at one device-wide barrier per step: every sweeping workgroup redoes the
 * resampling of eq. (1) from the energies in its LDS and then claims blocks of
 * replicas to sweep; the statistics of Sec. 4 run in a workgroup of their own,
 * one step behind.  Other runs take the segmented launches (graphs on: all of
 * them).  Results are identical in both modes; the segmented form measured as
 * fast or faster on every batch tried. */
enum { PA_BATCH_TEAM = 0, PA_BATCH_SEGMENTED = 1 };
pa_status pa_ctx_set_batch_mode(pa_ctx *ctx, int mode);
/* How the last pa_run_batch on ctx went: the runs it finished in team
 * launches and the number of those launches (either may be NULL). */
pa_status pa_ctx_batch_info(pa_ctx *ctx, uint32_t *team_runs, uint32_t *team_launches);
/* Stops the pa_run_batch running on ctx (callable from any thread): a team
 * launch leaves its barrier waits and the call returns PA_ERR_CANCELLED; the
 * runs' results are then undefined, the context stays usable.  A barrier wait
 * that lasts longer than 10 s ends the same way with PA_ERR_DEVICE. */
pa_status pa_ctx_abort_batch(pa_ctx *ctx);
pa_status pa_run_batch(pa_ctx *ctx, const pa_run_desc *descs, uint32_t n, void *d_ws,
                       uint64_t ws_bytes, void *stream, pa_result *outs);

/* Serving: continuous batching of PA runs.  pa_serve_start runs a scheduler
 * thread on the context; it owns the caller's device arena (d_arena,
 * 256-byte aligned, valid until pa_serve_stop returns) and the stream.
 * Requests (pa_serve_submit; the description is copied, the result buffers are
 * the caller's and must stay valid until pa_serve_wait returns) wait in arrival
 * order and are admitted as soon as a run slot is free (max_slots) and their
 * workspace (pa_plan_info.workspace_bytes) fits the free arena, first fit; a
 * request that does not fit yet lets later ones pass.  Admitted runs stay
 * device-resident and advance together with the batched launches, several
 * steps per scheduling round; finished runs release slot and memory at once.
 * Every run's results equal those of pa_run for the same description.
 * pa_serve_wait blocks until the ticket finishes (timeout_us < 0: no limit),
 * fills the timing (microseconds since pa_serve_start) and consumes the
 * ticket.  pa_serve_cancel marks a ticket: a queued request is dropped, a
 * running one is released at the next round; its wait returns
 * PA_ERR_CANCELLED.  pa_serve_stop lets admitted runs finish, cancels queued
 * ones and joins the thread.  Submit, wait and cancel are thread-safe. */
typedef struct { double arrival_us, admit_us, done_us; uint64_t attempts; } pa_timing;
pa_status pa_serve_start(pa_ctx *ctx, void *d_arena, uint64_t arena_bytes, uint32_t max_slots,
                         void *stream);
pa_status pa_serve_submit(pa_ctx *ctx, const pa_run_desc *desc, pa_result *out, uint64_t *ticket);
pa_status pa_serve_wait(pa_ctx *ctx, uint64_t ticket, int64_t timeout_us, pa_timing *timing);
pa_status pa_serve_cancel(pa_ctx *ctx, uint64_t ticket);
pa_status pa_serve_stop(pa_ctx *ctx);
/* pa_serve_checkpoint: write the current state of a running ticket to `path`
 * in the format of pa_checkpoint, at the next step boundary of the serving
 * loop, and wait for it (the run goes on).  PA_ERR_BUSY for a ticket not
 * admitted yet or with a checkpoint in progress, PA_ERR_INVALID for an unknown
 * or finished ticket.  pa_serve_resume: submit a request that continues the run
 * of a checkpoint file (its results are valid from the checkpoint's step on);
 * otherwise as pa_serve_submit. */
pa_status pa_serve_checkpoint(pa_ctx *ctx, uint64_t ticket, const char *path);
pa_status pa_serve_resume(pa_ctx *ctx, const char *path, pa_result *out, uint64_t *ticket);


/* ---- Analysis of run outputs (host only, no device work) -------------------
 *
 * pa_width_maxima: the largest histogram width along a run (Sec. 4, Tables
 * I-III): width[0..K) (pa_result.width_e or width_m) at inverse temperatures
 * beta[0..K); returns the first index i_max attaining the maximum, w_max =
 * width[i_max] and T_max = 1 / beta[i_max] (infinite at beta = 0).  NaN
 * widths are invalid.
 *
 * pa_free_energy_crossing: inverse temperature where the -beta F estimates of
 * a cooling run and of a heating run from ground states cross (Sec. 6, eq. (2)
 * with eq. (7)-(8); the crossing locates the transition point).  beta[0..K)
 * strictly increasing; mbf_cool and mbf_heat are -beta F on that grid (the
 * heating run's pa_result.minus_beta_F reversed by the caller).  With d_i =
 * mbf_cool[i] - mbf_heat[i], the candidates are the intervals with d_i > 0 >=
 * d_{i+1} (the cooling estimate falls below the heating one); the one with the
 * largest d_i - d_{i+1} is taken and *beta_x is the zero of the straight line
 * through its end points.  PA_ERR_INVALID if there is no such interval. */
pa_status pa_width_maxima(const double *beta, const double *width, uint32_t K, uint32_t *i_max,
                          double *w_max, double *T_max);
pa_status pa_free_energy_crossing(const double *beta, const double *mbf_cool, const double *mbf_heat,
                                  uint32_t K, double *beta_x);

/* ---- Instruction issue-rate probes (measurement of the sweep's ceiling) ----
 *
 * The sweep kernel is bound by the issue of 32-bit integer vector
 * instructions, whose rates on gfx950 depend on the kind.  pa_issue_probe runs
 * a stream of one kind (eight independent chains per lane, 32 waves per
 * compute unit) on every compute unit of the context's device and returns the
 * rate in lane-instructions per second (the fastest of three timed launches
 * after a warm-up).  PA_PROBE_MIX is the sweep inner loop's mix of kinds per
 * pair update (18 multiply-adds, 19 three-input bitops, 4 each of perm, xad
 * and sad, 2 xor, 2 and, 2 compare-select pairs).  d_out is a device buffer of
 * at least 4 * 256 * 8 * (compute units) bytes (one word per probe thread,
 * overwritten); the launches are ordered on `stream` and the call waits for
 * them. */
enum {
    PA_PROBE_XOR = 0,     /* v_xor_b32                               */
    PA_PROBE_BITOP3 = 1,  /* v_bitop3_b32 (three-input bitwise op)   */
    PA_PROBE_MAD64 = 2,   /* v_mad_u64_u32 (32x32 -> 64 multiply-add) */
    PA_PROBE_PERM = 3,    /* v_perm_b32                              */
    PA_PROBE_SAD = 4,     /* v_sad_u8                                */
    PA_PROBE_XAD = 5,     /* v_xad_u32                               */
    PA_PROBE_MULHI = 6,   /* v_mul_hi_u32                            */
    PA_PROBE_CMPSEL = 7,  /* v_cmp_le_u32 to VCC + v_cndmask_b32     */
    PA_PROBE_MIX = 8,     /* the sweep's mix, see above              */
    PA_PROBE_KINDS = 9
};
pa_status pa_issue_probe(pa_ctx *ctx, uint32_t kind, void *d_out, uint64_t out_bytes, void *stream,
                         double *lane_instr_per_s);

const char *pa_status_str(pa_status s);
const char *pa_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
