// pa_device.h -- launch interface between the host runtime (pa_host.cpp) and
// the gfx950 kernels (pa_kernels.hip).  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pa {

enum SweepMode : uint32_t { SWEEP_UPDATE = 0, SWEEP_INIT_RANDOM = 1, SWEEP_INIT_GROUND = 2 };

// Philox domain tags (counter word 3, bits 28..31).
enum : uint32_t { DOM_INIT = 0, DOM_SWEEP = 1, DOM_RESAMPLE = 2, DOM_PLAN = 3, DOM_GROUND = 4,
                  DOM_DIGEST = 5 };

struct SweepArgs {
    const uint8_t *old_pop;   // [R_prev][N] (UPDATE mode)
    const uint32_t *anc;      // [R_new] ancestors, or nullptr for the identity
    uint8_t *new_pop;         // [R_new][N]
    int32_t *E_out;           // [R_new]
    uint32_t *Mt_out;         // [R_new] M~ of eq. (5), or nullptr
    uint64_t *H_out;          // [R_new] digest term of each replica, or nullptr
    uint64_t T[4];            // thresholds for dE = 1..4 (<= 2^32)
    uint32_t L, q, N;
    uint32_t R_new;
    uint32_t step;            // Philox counter word 2
    uint32_t theta;
    uint32_t mode;            // SweepMode
    uint32_t key0, key1;      // Philox key
    uint32_t G;               // lanes per replica: a power of two up to 64 (several replicas
                              // per wave) or a multiple of 64 (one replica per workgroup)
    uint32_t waves_per_block;
};

// The resampling into step `step` of a population small enough for one
// workgroup's LDS (Sec. 2 step 2, eq. (1)): the reference energy, the integer
// weights and their scan, the draws, the copy numbers and their scan, the
// slot map, all from the energies of step-1 -- the integer results of k_post's
// weights, k_sample and k_countfill.
struct SmallResample {
    const int32_t *E_prev;    // [R_prev] energies of step-1
    uint32_t *anc_out;        // [n_new] ancestors of the new slots
    uint32_t *counts_out;     // [R_prev] copy numbers
    uint64_t R_prev, n_new;
    const uint64_t *W;        // integer weights of the step, zero from D on
    uint32_t D;
    uint64_t w_const;         // nonzero: every weight equals it (dbeta = 0)
    uint32_t ref_max;         // E_ref = largest energy (dbeta < 0), else the smallest
    uint32_t resample;        // 0: resampling off (slot k keeps replica k)
    uint32_t step, key0, key1;
};
// Populations up to this size resample in one workgroup inside the post
// launch of the step before (R_cap; 12 bytes of LDS per replica).
constexpr uint64_t SMALL_RESAMPLE_MAX = 4096;

struct PostArgs {
    // population statistics of step i, from the energies E
    uint32_t *hist;           // [2N+1] energy histogram of step i (output; also the
                              // work area when the energies span more than the LDS window)
    uint32_t store_hist;      // write the full histograms of step i to hist / mhist
    uint32_t nbins;           // 2N+1
    int32_t two_n;
    uint64_t R_i;
    uint32_t step;            // i
    uint32_t has_next;        // i + 1 < K
    double dbeta_next;        // beta_{i+1} - beta_i
    double abs_dbeta_next;    // |beta_{i+1} - beta_i|
    int64_t *E_sum;           // [K]
    uint64_t *count;          // [K]   sum of the histogram (consistency check)
    double *lnQ;              // [K]
    double *mbF;              // [K]   -beta F
    int32_t *E_ref;           // [K]   reference energy used by step i+1
    // weights of the resampling to step i+1: workgroup 0 of a post launch
    // computes the statistics above, workgroups 1, 2, ... the inclusive scan
    // C over blocks of `wblock` replicas each
    uint32_t do_weights;
    uint32_t wblock;          // replicas per weight workgroup (scan_block(R_i))
    const int32_t *E;         // [R_i] energies of the population at step i
    const uint64_t *W;        // [D] fixed-point weights of step i+1 (zero from D on)
    uint32_t D;
    uint64_t w_const;         // nonzero: every weight equals it (dbeta = 0), W unused
    uint64_t *C;              // [R_i] inclusive prefix sums
    // magnetisation (eq. (4)-(5)) and histogram widths of step i
    const uint32_t *Mt;       // [R_i] M~ of the population at step i, or nullptr
    const uint64_t *H;        // [R_i] digest terms of the population, or nullptr
    uint64_t *digest;         // [K]
    uint32_t *mhist;          // [N+1] M~ histogram of step i (output / work area)
    uint32_t q, N;
    int64_t *Mt_sum;          // [K]
    uint32_t widths;          // integer parts of the FWHM of the histograms of step i
    uint32_t bin_e, bin_m;    // levels per histogram bin (>= 1)
    uint64_t *fw_e;           // [K][8]: H, jl, jr, h(jl-1), h(jl), h(jr), h(jr+1), unused
    uint64_t *fw_m;           // [K][8], M~ histogram (needs mhist)
    // a population of at most SMALL_RESAMPLE_MAX: one more workgroup does the
    // whole resampling into step i+1 (rs) in place of the weight workgroups
    uint32_t small;
    SmallResample rs;
};

struct SampleArgs {
    const uint64_t *C;        // [R_prev]
    uint64_t R_prev;
    uint64_t n_new;
    uint32_t step;
    uint32_t key0, key1;
    uint32_t *r;              // [R_prev] copy counts (zero on entry)
};

// Count scan and slot map, one workgroup per block of `block` ancestors.  The
// counts r of this step stay as they are (later workgroups read earlier
// blocks); the counts buffer of the other step parity, r_clear, is zeroed over
// [0, clear_n) for the next step's draws.
struct SlotmapArgs {
    const uint32_t *r;        // [R_prev] copy counts
    uint64_t R_prev;
    uint32_t *anc;            // [anc_cap]
    uint64_t anc_cap;         // capacity of anc (writes beyond it are dropped)
    uint32_t *counts_last;    // [R_prev] copy of the counts
    uint32_t block;           // ancestors per workgroup (scan_block(R_prev))
    uint32_t *r_clear;        // counts of the other parity
    uint64_t clear_n;
};

// Elements per workgroup of the multi-workgroup scans: rows of 4096 (four
// per thread), enough rows that at most 64 workgroups share a population.
// Each workgroup recomputes the sums before its block, so the work grows with
// the number of workgroups times the population.
__host__ __device__ inline uint32_t scan_block(uint64_t n) {
    const uint64_t row = 4096, max_blocks = 64;
    const uint64_t rows = (n + row * max_blocks - 1) / (row * max_blocks);
    return (uint32_t)(row * (rows ? rows : 1));
}
// Workgroups of a post launch: statistics, the weight blocks, and the
// resampling workgroup of a small population.
__host__ __device__ inline uint32_t post_blocks(const PostArgs &a) {
    return 1u + (a.do_weights ? (uint32_t)((a.R_i + a.wblock - 1) / a.wblock) : 0u) + (a.small ? 1u : 0u);
}
__host__ __device__ inline uint32_t countfill_blocks(const SlotmapArgs &m) {
    return (uint32_t)((m.R_prev + m.block - 1) / m.block);
}

// Lattices beyond one workgroup's LDS (L > 256): replicas stay in HBM; one
// launch per half-sweep over (replica, tile of `rows` rows).
struct TiledArgs {
    const uint8_t *src;       // [*][N] population read by a half-sweep or copy
    const uint32_t *anc;      // slot -> replica of src (ancestor), or nullptr for the identity
    uint8_t *dst;             // [R][N] population written
    uint64_t T[4];            // thresholds for dE = 1..4 (<= 2^32)
    uint32_t L, q, N, R;
    uint32_t rows, tiles;     // rows per tile, tiles per replica
    uint32_t step;            // Philox step
    uint32_t h0, halves;      // first half-sweep (sweep h/2, colour h%2) and count; 0: copy
    uint32_t key0, key1;
    uint32_t init;            // k_tiled_init: SWEEP_INIT_RANDOM or SWEEP_INIT_GROUND
    uint32_t *bonds;          // [R] equal-neighbour bond counts (measure; zero on entry)
    uint32_t *cnt;            // [R][q] per-state site counts, or nullptr (zero on entry)
    uint64_t *Hacc;           // [R] digest sums of the tiles, or nullptr (zero on entry)
    uint64_t *H_out;          // [R] digest term of each replica, or nullptr
    int32_t *E_out;           // [R]
    uint32_t *Mt_out;         // [R] or nullptr
};
bool tiled_path(uint32_t L);
uint32_t tiled_rows(uint32_t L);
uint32_t tiled_max_halves(uint32_t L);   // half-sweeps fused per tiled launch
hipError_t launch_tiled_half(const TiledArgs &a, hipStream_t s);
hipError_t launch_tiled_init(const TiledArgs &a, hipStream_t s);
// energies (eq. (3)) and M~ (eq. (5)) of dst; leaves bonds and cnt zeroed
hipError_t launch_tiled_measure(const TiledArgs &a, hipStream_t s);

hipError_t launch_sweep(const SweepArgs &a, hipStream_t s);
hipError_t launch_post(const PostArgs &a, hipStream_t s);
// multinomial draws (k_sample), then count scan + slot map (k_countfill)
hipError_t launch_resample(const SampleArgs &a, const SlotmapArgs &m, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s);

// One launch of many small fills and copies (a batch's start: zeroed
// histograms, counts and sums, weight tables; its end: the per-step result
// blocks gathered for one read-back).  Record r writes words [0, words) of
// dst: src[i] where src is set, else value; it owns workgroups
// start[r] .. start[r+1]-1, each PREP_CHUNK words.
struct PrepRec {
    uint32_t *dst;
    const uint32_t *src;
    uint64_t words;
    uint32_t value;
    uint32_t pad;
};
constexpr uint64_t PREP_CHUNK = 4096;
hipError_t launch_prep_batch(const PrepRec *recs, const uint32_t *start, uint32_t n, uint32_t blocks,
                             hipStream_t s);

// Batched forms: several runs per launch.  Sweep launches group runs of one
// kernel class (sweep_class); `start` [n+1] gives each run's first workgroup.
uint32_t sweep_class(uint32_t L, uint32_t q, bool t64, uint32_t G);
void *sweep_kernel(uint32_t cls, bool batch);
hipError_t launch_sweep_batch(uint32_t cls, const SweepArgs *runs, const uint32_t *start, uint32_t n,
                              uint32_t blocks, uint32_t threads, size_t lds, hipStream_t s);
// Post and count-scan launches: run r owns workgroups pstart[r] .. pstart[r+1]-1
// (post_blocks / countfill_blocks of its records).
hipError_t launch_post_batch(const PostArgs *runs, const uint32_t *pstart, uint32_t n, uint32_t blocks,
                             hipStream_t s);
hipError_t launch_resample_batch(const SampleArgs *sruns, const uint32_t *start, uint32_t n,
                                 uint32_t blocks, const SlotmapArgs *mruns, const uint32_t *mstart,
                                 uint32_t mblocks, hipStream_t s);

// Issue-rate probe of instruction kind `kind` (PA_PROBE_*): `blocks` workgroups
// of probe_threads() threads, `iters` iterations; out[blocks * probe_threads()].
hipError_t issue_probe(uint32_t kind, uint32_t blocks, uint32_t iters, uint32_t *out, hipStream_t s,
                       double *lane_instr_per_s, double *ms);
uint32_t probe_threads();

// Team kernel: small runs of one sweep class through all their steps in one
// cooperative launch (see k_team).  Per run and step i (first step of the
// launch i0 + 1): the resampling into i, the sweeps of i, the statistics of
// i - 1 (statistics of step i0 were formed before the launch).
struct TeamStep {
    SweepArgs w;              // sweeps of step i (each workgroup gathers from its own LDS
                              // ancestors and sweeps its own range of slots)
    PostArgs p;               // statistics of step i-1 (used when stats != 0)
    SmallResample r;          // the resampling into step i
    uint32_t stats;           // statistics of step i-1 due in this launch
};
struct TeamRun {
    uint32_t team0, team;     // first workgroup of the run's team, workgroups (>= 2)
    uint32_t rec0, n_steps;   // its TeamStep records
    uint32_t *barrier;        // the team's barrier counter (own 256 bytes, zero at launch)
    uint32_t *claims;         // [n_steps] sweep blocks claimed per step (zero at launch)
    PostArgs last;            // statistics of the last step, after the last sweeps
    uint32_t last_stats;
};
struct TeamCtl {
    uint32_t *abort;          // host-visible word: nonzero makes every barrier wait end
    uint64_t timeout_ticks;   // bound of one barrier wait (100 MHz real-time counter)
    uint32_t r_max;           // largest R_prev of the launch
    uint32_t anc_bytes;       // LDS for the ancestors of every new slot (16-byte multiple)
    uint32_t work_bytes;      // LDS after them: resampling, sweep groups or statistics
    uint32_t sub_lds;         // LDS of one sweep group (16-byte multiple)
};
// Kernel of a class for the team launch (null if the class has none), and its
// launch; team workgroups have 1024 threads.
void *team_kernel(uint32_t cls);
uint32_t team_threads();
// Workgroups of the team kernel of a class that fit the device at once with
// `lds` bytes of dynamic LDS each (0 if none).
uint32_t team_capacity(uint32_t cls, size_t lds, int device);
// Dynamic LDS of the statistics' histogram window (k_post).
constexpr size_t POST_LDS_BYTES = 14336 * 4;
hipError_t launch_team(uint32_t cls, const TeamRun *runs, uint32_t n_runs, const TeamStep *steps,
                       const TeamCtl &ctl, uint32_t blocks, size_t lds, hipStream_t s);

// Lanes-per-replica candidates for L (0 if L has no fixed-shape kernel).
uint32_t lane_candidates(uint32_t L, uint32_t *out /*[2]*/);
// Lanes per replica (log2) and waves per block for a lattice side L; `lanes`
// selects a candidate (anything else: the default).
void sweep_shape(uint32_t L, uint32_t lanes, uint32_t *G, uint32_t *waves_per_block);
// q_counters: q when the sweep counts states for M~ (eq. (5)), else 0
size_t sweep_lds_bytes(uint32_t N, uint32_t G, uint32_t waves_per_block, uint32_t q_counters);
uint64_t replicas_per_block(uint32_t G, uint32_t waves_per_block);
// index of L in the table of lattices with lane choices (-1: none), and its size
int lane_choice_index(uint32_t L);
constexpr int LANE_CHOICE_COUNT = 13;
// Device address of the fixed workspace array of pa_run_static on `device`
// (the current device), looked up once per device; null on failure.
void *static_scratch(int device, hipError_t *err);
// Largest dynamic LDS a workgroup may use on the current device.
size_t max_lds_per_block(int device);

}  // namespace pa
