/*
 * pa_oracle.h -- plain CPU oracle for population annealing of the 2D q-state
 * Potts model (Barash, Weigel, Shchur, Janke, "Exploring first-order phase
 * transitions with population annealing", arXiv:1704.01888).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no source with the GPU library: both sides implement the
 * same written conventions independently (Philox4x32-10 from its published
 * definition, the plan tables from their formulas, the update rule, the
 * resampler).
 *
 * Conventions where the paper is silent: spins are 0..q-1 (the paper's 1..q
 * shifted down by one), the lattice is L x L, periodic, row-major, site
 * n = y*L + x; the other choices (random-number counters, update order,
 * proposal, acceptance and resampling arithmetic) are stated at the functions
 * that make them.
 *
 * Every function returns 0 on success and a negative code on invalid input.
 */
#ifndef PA_ORACLE_H
#define PA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_RESAMPLE_POISSON = 0, ORC_RESAMPLE_MULTINOMIAL = 1, ORC_RESAMPLE_NONE = 2 };
enum { ORC_INIT_RANDOM = 0, ORC_INIT_GROUND = 1 };
enum { ORC_OK = 0, ORC_ERR_INVALID = -1, ORC_ERR_NOMEM = -2, ORC_ERR_CAPACITY = -4 };

/* Philox counter word 3 carries a domain tag in its top four bits. */
enum { ORC_DOM_INIT = 0, ORC_DOM_SWEEP = 1, ORC_DOM_RESAMPLE = 2, ORC_DOM_PLAN = 3,
       ORC_DOM_GROUND = 4, ORC_DOM_DIGEST = 5 };

typedef struct {
    uint32_t L, q;         /* lattice side (even, >= 2) and number of Potts states      */
    uint64_t R;            /* target population size R                                 */
    uint32_t K;            /* number of inverse temperatures beta_0 .. beta_{K-1}       */
    const double *beta;    /* [K] temperature protocol                                 */
    uint32_t theta;        /* Metropolis sweeps per temperature step                   */
    uint64_t seed;         /* Philox key = (low 32 bits, high 32 bits)                 */
    int32_t resample;      /* ORC_RESAMPLE_*                                           */
    int32_t init;          /* ORC_INIT_*                                               */
    uint32_t bin_e, bin_m; /* histogram widths: energy / M~ levels per bin (0 means 1)  */
} orc_desc;

/* Philox4x32-10 block: out = Philox(ctr, key). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Validate a run description. */
int orc_validate(const orc_desc *d);

/* Metropolis thresholds at inverse temperature beta: T[dE] for dE = 0..4 with
 * T[dE] = floor(2^32 * exp(-beta*dE)); T[0] = 2^32 (a move with dE <= 0 is
 * always accepted). */
void orc_thresholds(double beta, uint64_t T[5]);

/* Fixed-point resampling weights W[d] = round(2^Kb * exp(-|dbeta| d)) for
 * d = 0..2N; returns D = the first d with W[d] == 0 (or 2N+1). */
uint32_t orc_weights(double abs_dbeta, uint32_t Kb, uint32_t N, uint64_t *W);

/* One Poisson(lambda) draw by inversion of the uniform u in [0,1), visiting
 * the support in alternating order outward from the mode. */
uint64_t orc_poisson(double lambda, double u);

/* Plan: number of replicas after each step (R_sched[0] = R) and the capacity
 * R_cap = max_i R_sched[i] and the weight precision Kb = 63 - ceil(log2 R_cap). */
int orc_plan(const orc_desc *d, uint64_t *R_sched, uint64_t *R_cap, uint32_t *Kb);

/* Potts energy, eq. (3) with J = 1: E = -sum_n [d(s_n,s_right) + d(s_n,s_down)]. */
int32_t orc_energy(uint32_t L, const uint8_t *s);

/* Magnetisation, eq. (5): returns M~ = max_alpha #{k: s_k = alpha}. */
uint32_t orc_mtilde(uint32_t L, uint32_t q, const uint8_t *s);

/* Full width at half maximum of a histogram (Sec. 4), in levels: h[0..nb)
 * grouped into bins of B levels (bin j = levels jB .. jB+B-1), read as the
 * straight lines through the bin counts at the bin indices, zero beyond both
 * ends; the width is B times the distance between its outermost crossings of
 * half the largest count.  Returns 0 for an empty histogram. */
double orc_fwhm(const uint32_t *h, uint32_t nb, uint32_t B);

/* Digest of a population at step i: the sum, modulo 2^64, over slots k < R
 * and dwords n < N/4 of r * d, where d packs spins 4n..4n+3 of slot k
 * (little endian) and r = (w1 << 32 | w0) | 1 with w = Philox(n, k, i,
 * DIGEST << 28).  A checksum for comparing whole populations, not part of
 * the method. */
uint64_t orc_digest(const orc_desc *d, uint32_t i, const uint8_t *spins, uint64_t R);

/* Largest width along a run (Sec. 4, Tables I-III): first index of the
 * maximum of width[0..K), its value and T = 1/beta there. */
int orc_width_maxima(const double *beta, const double *width, uint32_t K, uint32_t *i_max,
                     double *w_max, double *T_max);

/* Crossing of the cooling and heating -beta F estimates (Sec. 6, Fig. 3) on an
 * increasing beta grid: over the intervals where the cooling estimate goes
 * from above the heating one to at or below it, the one with the largest
 * change of the difference; the crossing is linear between its end points. */
int orc_crossing(const double *beta, const double *f_cool, const double *f_heat, uint32_t K,
                 double *beta_x);

/* Initial configuration of slot k (random: uniform spins; ground: all equal). */
void orc_init_replica(const orc_desc *d, uint64_t k, uint8_t *s);

/* theta checkerboard Metropolis sweeps at beta_i (step i >= 1) on the replica in
 * slot k, in place. */
void orc_sweep_replica(const orc_desc *d, uint32_t i, uint64_t k, uint8_t *s);

/* One checkerboard Metropolis sweep number t at step i on slot k with the given
 * thresholds, in place (the building block of orc_sweep_replica). */
void orc_one_sweep(const orc_desc *d, uint32_t i, uint32_t t, uint64_t k,
                   const uint64_t T[5], uint8_t *s);

/* Resampling from beta_{i-1} to beta_i (step 2 of the algorithm, eq. (1)).
 * E[R_prev] are the energies of the current population; n_new draws are made.
 * Outputs the copy counts r[R_prev] and the ancestor of each new slot
 * anc[n_new] (ancestor-sorted).  *E_ref receives the reference energy. */
int orc_resample(const orc_desc *d, uint32_t i, uint32_t Kb, const int32_t *E,
                 uint64_t R_prev, uint64_t n_new, uint32_t *r, uint32_t *anc,
                 int32_t *E_ref);

/* ln Q_i (step 2, eq. (2)) from the energy histogram of the population at
 * beta_{i-1}: hist[b] = #{j: E_j = b - 2N}, b = 0..2N. */
double orc_lnQ(uint32_t N, double dbeta, const uint32_t *hist, uint64_t R_prev,
               int32_t *E_ref_out);

/* Results of a run: per-step arrays of length K unless stated. */
typedef struct {
    uint64_t *R_i;          /* population size at each beta                     */
    int64_t  *E_sum;        /* sum of energies                                  */
    double   *E_mean;       /* eq. (4)                                          */
    double   *lnQ;          /* ln Q_i, lnQ[0] = 0                               */
    double   *minus_beta_F; /* eq. (2) with ln Z_{beta_0}                       */
    double   *M_mean;       /* eq. (4)-(5) magnetisation mean, or NULL          */
    int64_t  *Mt_sum;       /* sum over the population of M~ (eq. (5)), or NULL */
    uint32_t *mhist;        /* [K][N+1] histogram of M~, or NULL                */
    double   *width_e;      /* FWHM of the histogram of e = E/N (Sec. 4), or NULL */
    double   *width_m;      /* FWHM of the histogram of m = M/N (Sec. 4), or NULL */
    uint64_t *digest;       /* population digest at each step (orc_digest), or NULL */
    uint32_t *hist;         /* [K][2N+1] energy histogram, or NULL              */
    uint8_t  *final_spins;  /* [R_{K-1}][N], or NULL                            */
    int32_t  *final_E;      /* [R_{K-1}], or NULL                               */
    uint32_t *last_anc;     /* ancestors of the last resampling [R_{K-1}], or NULL */
    int       n_threads;    /* threads used for the sweeps (output)             */
} orc_result;

/* Whole run (steps 1-5 of the algorithm). */
int orc_run(const orc_desc *d, orc_result *out);

/* Continuation of a run from a population at step `step` (R_cur replicas,
 * spins[R_cur][N], -beta F = minus_beta_F there): observes that population at
 * `step` (ln Q reported as 0 there) and runs steps step+1 .. K-1; the result
 * arrays are filled from index `step` on. */
int orc_run_from(const orc_desc *d, uint32_t step, uint64_t R_cur, const uint8_t *spins,
                 double minus_beta_F, orc_result *out);

/* A checkpoint file of the GPU library (128-byte little-endian header with the
 * run description, step, R_i, -beta F and energy sum; beta[K]; spins), read
 * into owned arrays; orc_free_checkpoint releases them. */
typedef struct {
    orc_desc desc;         /* desc.beta points to beta                 */
    double *beta;          /* [K]                                      */
    uint32_t step;
    uint64_t R_cur;
    double minus_beta_F;
    int64_t E_sum;
    uint8_t *spins;        /* [R_cur][L*L]                             */
} orc_checkpoint;
int orc_read_checkpoint(const char *path, orc_checkpoint *ck);
void orc_free_checkpoint(orc_checkpoint *ck);

/* Stepwise: advance a population from step i-1 to step i.
 * spins_old[R_prev][N], E_old[R_prev] in; spins_new[R_new][N], E_new[R_new],
 * anc[R_new] out (R_new = plan's R_sched[i]). */
int orc_step(const orc_desc *d, uint32_t i, uint32_t Kb, const uint8_t *spins_old,
             const int32_t *E_old, uint64_t R_prev, uint64_t R_new, uint8_t *spins_new,
             int32_t *E_new, uint32_t *anc);

#ifdef __cplusplus
}
#endif
#endif
