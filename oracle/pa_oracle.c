/*
 * pa_oracle.c -- plain, slow CPU oracle for population annealing (PA) of the
 * 2D q-state Potts model, arXiv:1704.01888.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the GPU library.  It shares no
 * source with the GPU library.
 *
 * Everything is written in the order the paper states the method:
 *   Sec. 2, steps 1-5  : initial population, resampling, Metropolis rounds,
 *                        population averages, loop over temperatures;
 *   Sec. 2, eq. (1)    : Poisson copy numbers, new population size R_i;
 *   Sec. 2, eq. (2)    : free-energy estimator -beta_i F = ln Z_beta0 + sum ln Q_m;
 *   Sec. 3, eq. (3)    : Potts Hamiltonian, J = 1, periodic square lattice;
 *   Sec. 3, eq. (4)-(5): population averages of E and M;
 *   Sec. 5, eq. (6)    : ground-state initial population for heating runs;
 *   Sec. 6, eq. (7)-(8): Z at beta -> infinity, q e^{-beta E_0}, E_0 = -2N.
 * Where the paper leaves a choice open (random-number generator, order of site
 * updates, proposal, acceptance arithmetic, resampling arithmetic) the reading
 * used here is stated next to the code.  Floating point is IEEE double.
 */
#include "pa_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplications by  */
/* fixed constants, the high halves xored with the other two counter words   */
/* and the round key; the key is advanced by two Weyl constants per round.   */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void philox_seeded(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                          uint32_t out[4])
{
    uint32_t ctr[4] = { c0, c1, c2, c3 };
    uint32_t key[2] = { (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    orc_philox4x32_10(ctr, key, out);
}

/* floor(w * n / 2^32): maps a uniform 32-bit word onto {0, .., n-1}. */
static uint32_t mulhi32(uint32_t w, uint32_t n)
{
    return (uint32_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

/* floor(x * S / 2^64) with a 128-bit product. */
static uint64_t mulhi64(uint64_t x, uint64_t S)
{
    return (uint64_t)(((unsigned __int128)x * (unsigned __int128)S) >> 64);
}

/* ------------------------------------------------------------------------ */
/* Validation of a run description.                                         */
/* ------------------------------------------------------------------------ */
int orc_validate(const orc_desc *d)
{
    if (!d || !d->beta) return ORC_ERR_INVALID;
    if (d->L < 2 || (d->L & 1u) || d->L > 4096) return ORC_ERR_INVALID;
    if (d->q < 2 || d->q > 255) return ORC_ERR_INVALID;
    if (d->R < 1 || d->R > (1ull << 31)) return ORC_ERR_INVALID;
    if (d->K < 1) return ORC_ERR_INVALID;
    if (d->theta >= (1u << 27)) return ORC_ERR_INVALID;
    if (d->resample < 0 || d->resample > 2) return ORC_ERR_INVALID;
    if (d->init < 0 || d->init > 1) return ORC_ERR_INVALID;
    for (uint32_t i = 0; i < d->K; ++i)
        if (!isfinite(d->beta[i]) || d->beta[i] < 0.0) return ORC_ERR_INVALID;
    /* A uniformly random population is in equilibrium only at beta = 0
     * (step 1 of the algorithm in Sec. 2). */
    if (d->init == ORC_INIT_RANDOM && d->beta[0] != 0.0) return ORC_ERR_INVALID;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Plan tables.                                                              */
/* ------------------------------------------------------------------------ */

/* Metropolis acceptance min(1, exp(-beta dE)) (Sec. 2 step 3, Sec. 3) as a
 * 32-bit integer threshold: a move with dE > 0 is accepted iff the uniform
 * word w satisfies w < T[dE].  T can reach 2^32 (beta = 0). */
void orc_thresholds(double beta, uint64_t T[5])
{
    T[0] = 1ull << 32;
    for (int dE = 1; dE <= 4; ++dE) {
        double x = beta * (double)dE;
        T[dE] = (uint64_t)floor(ldexp(exp(-x), 32));
    }
}

/* Relative Boltzmann weight exp(-(beta_i - beta_{i-1}) E_j) of Sec. 2 step 2,
 * written relative to the reference energy E_ref of the population so that
 * the weight of replica j is exp(-|dbeta| d_j) with d_j = |E_j - E_ref| >= 0,
 * in 2^-Kb fixed point. */
uint32_t orc_weights(double abs_dbeta, uint32_t Kb, uint32_t N, uint64_t *W)
{
    uint32_t D = 2 * N + 1;
    uint32_t first_zero = D;
    for (uint32_t dd = 0; dd < D; ++dd) {
        double x = abs_dbeta * (double)dd;
        double v = nearbyint(ldexp(exp(-x), (int)Kb));
        W[dd] = (uint64_t)v;
        if (W[dd] == 0 && first_zero == D) first_zero = dd;
    }
    for (uint32_t dd = first_zero; dd < D; ++dd) W[dd] = 0;
    return first_zero;
}

/* Poisson(lambda) by inversion: the support is visited in the order
 * m, m+1, m-1, m+2, m-2, ... (m = floor(lambda), the mode) and the first k at
 * which the accumulated probability exceeds u is returned.  The pmf is carried
 * by the ratios p(k+1) = p(k) lambda/(k+1) and p(k-1) = p(k) k/lambda from
 * p(m) = exp(-lambda + m ln lambda - lgamma(m+1)). */
uint64_t orc_poisson(double lambda, double u)
{
    double m = floor(lambda);
    double pm = exp(-lambda + m * log(lambda) - lgamma(m + 1.0));
    double acc = pm;
    if (u < acc) return (uint64_t)m;
    double hi = m, lo = m, phi = pm, plo = pm;
    for (;;) {
        hi = hi + 1.0;
        phi = phi * lambda / hi;
        acc = acc + phi;
        if (u < acc) return (uint64_t)hi;
        if (lo > 0.0) {
            plo = plo * lo / lambda;
            lo = lo - 1.0;
            acc = acc + plo;
            if (u < acc) return (uint64_t)lo;
        }
        /* All remaining mass has underflowed: u lies in the rounding gap just
         * below 1. */
        if (phi == 0.0 && (lo == 0.0 || plo == 0.0)) return (uint64_t)hi;
    }
}

static uint32_t ceil_log2_u64(uint64_t x)
{
    uint32_t b = 0;
    while ((1ull << b) < x) ++b;
    return b;
}

/* Population sizes per step.  The paper draws r_j ~ Pois((R/R_{i-1}) tau_i(E_j))
 * independently (eq. (1)).  Since sum_j tau_i(E_j) = R_{i-1}, the means add up
 * to R, so the same joint law is obtained by first drawing the new size
 * R_i ~ Pois(R) and then distributing R_i copies multinomially with
 * probabilities tau_i(E_j)/R_{i-1}.  R_i does not depend on the energies and is
 * drawn here up front, one uniform per step from the plan stream. */
int orc_plan(const orc_desc *d, uint64_t *R_sched, uint64_t *R_cap, uint32_t *Kb)
{
    int rc = orc_validate(d);
    if (rc) return rc;
    uint64_t cap = d->R;
    R_sched[0] = d->R;
    for (uint32_t i = 1; i < d->K; ++i) {
        uint64_t n;
        if (d->resample == ORC_RESAMPLE_POISSON) {
            uint32_t w[4];
            philox_seeded(d->seed, 0u, 0u, i, (uint32_t)ORC_DOM_PLAN << 28, w);
            uint64_t x = ((uint64_t)w[1] << 32) | (uint64_t)w[0];
            double u = ldexp((double)(x >> 11), -53);
            n = orc_poisson((double)d->R, u);
            if (n == 0) return ORC_ERR_CAPACITY;
            if (n > (1ull << 31)) return ORC_ERR_CAPACITY;
        } else {
            n = d->R;
        }
        R_sched[i] = n;
        if (n > cap) cap = n;
    }
    *R_cap = cap;
    *Kb = 63u - ceil_log2_u64(cap);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Model: eq. (3) and eq. (5).                                               */
/* ------------------------------------------------------------------------ */
static uint32_t kron(uint8_t a, uint8_t b) { return a == b ? 1u : 0u; }

int32_t orc_energy(uint32_t L, const uint8_t *s)
{
    /* Each nearest-neighbour bond of the periodic square lattice once: the
     * bond to the right and the bond below every site (2N bonds). */
    int64_t sum = 0;
    for (uint32_t y = 0; y < L; ++y)
        for (uint32_t x = 0; x < L; ++x) {
            uint8_t si = s[y * L + x];
            uint8_t right = s[y * L + (x + 1) % L];
            uint8_t down = s[((y + 1) % L) * L + x];
            sum += kron(si, right) + kron(si, down);
        }
    return (int32_t)(-sum);
}

uint32_t orc_mtilde(uint32_t L, uint32_t q, const uint8_t *s)
{
    uint32_t count[256];
    memset(count, 0, sizeof count);
    for (uint32_t n = 0; n < L * L; ++n) count[s[n]]++;
    uint32_t best = 0;
    for (uint32_t a = 0; a < q; ++a)
        if (count[a] > best) best = count[a];
    return best;
}

/* ------------------------------------------------------------------------ */
/* Step 1: the initial population.                                           */
/* ------------------------------------------------------------------------ */
void orc_init_replica(const orc_desc *d, uint64_t k, uint8_t *s)
{
    uint32_t N = d->L * d->L;
    if (d->init == ORC_INIT_GROUND) {
        /* eq. (6): every spin equal to alpha, alpha uniform over the q states. */
        uint32_t w[4];
        philox_seeded(d->seed, 0u, (uint32_t)k, 0u, (uint32_t)ORC_DOM_GROUND << 28, w);
        uint8_t alpha = (uint8_t)mulhi32(w[0], d->q);
        for (uint32_t n = 0; n < N; ++n) s[n] = alpha;
        return;
    }
    /* Simple sampling at infinite temperature: i.i.d. uniform spins.  Site n
     * takes word n mod 4 of the block with counter (n / 4, k, 0, INIT). */
    for (uint32_t n = 0; n < N; ++n) {
        uint32_t w[4];
        philox_seeded(d->seed, n / 4, (uint32_t)k, 0u, (uint32_t)ORC_DOM_INIT << 28, w);
        s[n] = (uint8_t)mulhi32(w[n % 4], d->q);
    }
}

/* ------------------------------------------------------------------------ */
/* Step 3: Metropolis single-spin-flip sweeps.                               */
/* ------------------------------------------------------------------------ */

/* One sweep = two half-sweeps.  Half-sweep c visits every site of colour c,
 * (x + y) mod 2 == c, so that all its updates read only sites of the other
 * colour.  The m-th colour-c site in row-major order takes the random words
 * 2(m mod 2) and 2(m mod 2)+1 of the block with counter
 * (m / 2, k, i, SWEEP << 28 | t << 1 | c): the first chooses the proposed
 * state uniformly among the q-1 states different from the current one, the
 * second decides acceptance with probability min(1, exp(-beta_i dE)). */
void orc_one_sweep(const orc_desc *d, uint32_t i, uint32_t t, uint64_t k,
                   const uint64_t T[5], uint8_t *s)
{
    uint32_t L = d->L;
    for (uint32_t c = 0; c < 2; ++c) {
        uint32_t m = 0;
        uint32_t w[4] = { 0, 0, 0, 0 };
        for (uint32_t y = 0; y < L; ++y) {
            for (uint32_t x = 0; x < L; ++x) {
                if ((x + y) % 2 != c) continue;
                if (m % 2 == 0)
                    philox_seeded(d->seed, m / 2, (uint32_t)k, i,
                                  ((uint32_t)ORC_DOM_SWEEP << 28) | (t << 1) | c, w);
                uint32_t w_prop = w[2 * (m % 2)];
                uint32_t w_acc = w[2 * (m % 2) + 1];
                ++m;

                uint8_t cur = s[y * L + x];
                uint8_t nb[4] = {
                    s[y * L + (x + L - 1) % L],   /* left  */
                    s[y * L + (x + 1) % L],       /* right */
                    s[((y + L - 1) % L) * L + x], /* up    */
                    s[((y + 1) % L) * L + x],     /* down  */
                };
                /* Proposal: uniform over the q-1 other states. */
                uint32_t r = mulhi32(w_prop, d->q - 1);
                uint8_t prop = (uint8_t)(r >= cur ? r + 1 : r);
                /* Energy change of eq. (3) with J = 1: the bonds to the four
                 * neighbours lose -#{equal to cur} and gain -#{equal to prop}. */
                int a = 0, b = 0;
                for (int n = 0; n < 4; ++n) {
                    a += (int)kron(nb[n], cur);
                    b += (int)kron(nb[n], prop);
                }
                int dE = a - b;
                int accept = (dE <= 0) || ((uint64_t)w_acc < T[dE]);
                if (accept) s[y * L + x] = prop;
            }
        }
    }
}

void orc_sweep_replica(const orc_desc *d, uint32_t i, uint64_t k, uint8_t *s)
{
    uint64_t T[5];
    orc_thresholds(d->beta[i], T);
    for (uint32_t t = 0; t < d->theta; ++t) orc_one_sweep(d, i, t, k, T, s);
}

/* ------------------------------------------------------------------------ */
/* Step 2: resampling with the relative Boltzmann weights.                   */
/* ------------------------------------------------------------------------ */
int orc_resample(const orc_desc *d, uint32_t i, uint32_t Kb, const int32_t *E,
                 uint64_t R_prev, uint64_t n_new, uint32_t *r, uint32_t *anc,
                 int32_t *E_ref)
{
    uint32_t N = d->L * d->L;
    double dbeta = d->beta[i] - d->beta[i - 1];
    double abs_dbeta = fabs(dbeta);

    /* Reference energy: the population member of largest weight. */
    int32_t ref = E[0];
    for (uint64_t j = 1; j < R_prev; ++j) {
        if (dbeta >= 0.0) { if (E[j] < ref) ref = E[j]; }
        else              { if (E[j] > ref) ref = E[j]; }
    }
    *E_ref = ref;

    uint64_t *W = (uint64_t *)malloc(sizeof(uint64_t) * (2 * N + 1));
    uint64_t *C = (uint64_t *)malloc(sizeof(uint64_t) * (R_prev ? R_prev : 1));
    if (!W || !C) { free(W); free(C); return ORC_ERR_NOMEM; }
    uint32_t D = orc_weights(abs_dbeta, Kb, N, W);

    /* Cumulative weights C_j = sum_{j' <= j} W(d_j'). */
    uint64_t run = 0;
    for (uint64_t j = 0; j < R_prev; ++j) {
        int32_t diff = E[j] - ref;
        uint32_t dd = (uint32_t)(diff < 0 ? -diff : diff);
        run += (dd < D) ? W[dd] : 0;
        C[j] = run;
    }
    uint64_t S = run;

    /* n_new independent draws of an ancestor with probability W_j / S. */
    for (uint64_t j = 0; j < R_prev; ++j) r[j] = 0;
    for (uint64_t kk = 0; kk < n_new; ++kk) {
        uint32_t w[4];
        philox_seeded(d->seed, (uint32_t)kk, 0u, i, (uint32_t)ORC_DOM_RESAMPLE << 28, w);
        uint64_t x = ((uint64_t)w[1] << 32) | (uint64_t)w[0];
        uint64_t u = mulhi64(x, S);
        /* first j with C_j > u */
        uint64_t lo = 0, hi = R_prev - 1;
        while (lo < hi) {
            uint64_t mid = lo + (hi - lo) / 2;
            if (C[mid] > u) hi = mid; else lo = mid + 1;
        }
        r[lo] += 1;
    }

    /* New population in ancestor order: copies of replica j occupy the slots
     * o_j .. o_j + r_j - 1, o_j = sum_{j' < j} r_j'. */
    uint64_t o = 0;
    for (uint64_t j = 0; j < R_prev; ++j)
        for (uint32_t c = 0; c < r[j]; ++c) anc[o++] = (uint32_t)j;

    free(W);
    free(C);
    return (o == n_new) ? ORC_OK : ORC_ERR_INVALID;
}

/* Q_i = sum_j exp(-(beta_i - beta_{i-1}) E_j) / R_{i-1} (Sec. 2 step 2), as a
 * logarithm, with the sum grouped by energy and taken around E_ref:
 * ln Q_i = -dbeta E_ref + ln sum_{d} h(d) exp(-|dbeta| d) - ln R_{i-1},
 * h(d) = #{j: |E_j - E_ref| = d}, summed in ascending d. */
double orc_lnQ(uint32_t N, double dbeta, const uint32_t *hist, uint64_t R_prev,
               int32_t *E_ref_out)
{
    int32_t two_n = (int32_t)(2 * N);
    int32_t E_ref = 0;
    int found = 0;
    if (dbeta >= 0.0) {
        for (int32_t b = 0; b <= two_n && !found; ++b)
            if (hist[b]) { E_ref = b - two_n; found = 1; }
    } else {
        for (int32_t b = two_n; b >= 0 && !found; --b)
            if (hist[b]) { E_ref = b - two_n; found = 1; }
    }
    if (E_ref_out) *E_ref_out = E_ref;
    double abs_dbeta = fabs(dbeta);
    double sum = 0.0;
    for (int32_t dd = 0; dd <= two_n; ++dd) {
        int32_t E = (dbeta >= 0.0) ? E_ref + dd : E_ref - dd;
        int32_t b = E + two_n;
        if (b < 0 || b > two_n) continue;
        double w = exp(-(abs_dbeta * (double)dd));
        sum = sum + (double)hist[b] * w;
    }
    return -dbeta * (double)E_ref + log(sum) - log((double)R_prev);
}

/* ------------------------------------------------------------------------ */
/* One step i >= 1: resample (step 2), then theta sweeps (step 3).           */
/* ------------------------------------------------------------------------ */
int orc_step(const orc_desc *d, uint32_t i, uint32_t Kb, const uint8_t *spins_old,
             const int32_t *E_old, uint64_t R_prev, uint64_t R_new, uint8_t *spins_new,
             int32_t *E_new, uint32_t *anc)
{
    uint32_t N = d->L * d->L;
    if (d->resample == ORC_RESAMPLE_NONE) {
        /* Resampling switched off: every replica is carried over once. */
        if (R_new != R_prev) return ORC_ERR_INVALID;
        for (uint64_t j = 0; j < R_prev; ++j) anc[j] = (uint32_t)j;
    } else {
        uint32_t *r = (uint32_t *)malloc(sizeof(uint32_t) * (R_prev ? R_prev : 1));
        if (!r) return ORC_ERR_NOMEM;
        int32_t E_ref;
        int rc = orc_resample(d, i, Kb, E_old, R_prev, R_new, r, anc, &E_ref);
        free(r);
        if (rc) return rc;
    }
    int64_t nk = (int64_t)R_new;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nk; ++k) {
        uint8_t *s = spins_new + (uint64_t)k * N;
        memcpy(s, spins_old + (uint64_t)anc[k] * N, N);
        orc_sweep_replica(d, i, (uint64_t)k, s);
        E_new[k] = orc_energy(d->L, s);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Histogram width (Sec. 4).                                                 */
/* ------------------------------------------------------------------------ */
double orc_fwhm(const uint32_t *h, uint32_t nb, uint32_t B)
{
    if (B == 0) B = 1;
    uint32_t nc = (nb + B - 1) / B;
    /* c[1..nc] are the bin counts; c[0] = c[nc+1] = 0 stand for the zero
     * continuation beyond both ends. */
    double *c = (double *)calloc(nc + 2, sizeof(double));
    if (!c) return -1.0;
    for (uint32_t b = 0; b < nb; ++b) c[b / B + 1] += (double)h[b];
    double H = 0.0;
    for (uint32_t j = 1; j <= nc; ++j)
        if (c[j] > H) H = c[j];
    double width = 0.0;
    if (H > 0.0) {
        double half = 0.5 * H;
        uint32_t jl = 1, jr = nc;
        while (c[jl] < half) ++jl;     /* first bin at or above H/2 from the left  */
        while (c[jr] < half) --jr;     /* ... and from the right                   */
        /* Crossing points on the straight segments into those bins; bin j of
         * c sits at abscissa j - 1. */
        double xl = (double)((int64_t)jl - 2) + (half - c[jl - 1]) / (c[jl] - c[jl - 1]);
        double xr = (double)((int64_t)jr - 1) + (c[jr] - half) / (c[jr] - c[jr + 1]);
        width = (xr - xl) * (double)B;
    }
    free(c);
    return width;
}

uint64_t orc_digest(const orc_desc *d, uint32_t i, const uint8_t *spins, uint64_t R)
{
    uint32_t N = d->L * d->L;
    uint32_t key[2] = {(uint32_t)(d->seed & 0xffffffffu), (uint32_t)(d->seed >> 32)};
    uint64_t sum = 0;
    int64_t nk = (int64_t)R;
    /* a sum modulo 2^64: the order of the terms does not matter */
#pragma omp parallel for reduction(+ : sum) schedule(static)
    for (int64_t k = 0; k < nk; ++k) {
        const uint8_t *s = spins + (uint64_t)k * N;
        for (uint32_t n = 0; n < N / 4; ++n) {
            uint32_t ctr[4] = {n, (uint32_t)k, i, (uint32_t)ORC_DOM_DIGEST << 28};
            uint32_t w[4];
            orc_philox4x32_10(ctr, key, w);
            uint64_t r = (((uint64_t)w[1] << 32) | (uint64_t)w[0]) | 1u;
            uint64_t dw = (uint64_t)s[4 * n] | ((uint64_t)s[4 * n + 1] << 8) |
                          ((uint64_t)s[4 * n + 2] << 16) | ((uint64_t)s[4 * n + 3] << 24);
            sum += r * dw;
        }
    }
    return sum;
}

int orc_width_maxima(const double *beta, const double *width, uint32_t K, uint32_t *i_max,
                     double *w_max, double *T_max)
{
    if (K == 0) return ORC_ERR_INVALID;
    uint32_t best = 0;
    for (uint32_t i = 1; i < K; ++i)
        if (width[i] > width[best]) best = i;
    *i_max = best;
    *w_max = width[best];
    *T_max = 1.0 / beta[best];
    return ORC_OK;
}

int orc_crossing(const double *beta, const double *f_cool, const double *f_heat, uint32_t K,
                 double *beta_x)
{
    int found = 0;
    double best_change = 0.0;
    for (uint32_t i = 0; i + 1 < K; ++i) {
        double d_here = f_cool[i] - f_heat[i];
        double d_next = f_cool[i + 1] - f_heat[i + 1];
        if (!(d_here > 0.0 && d_next <= 0.0)) continue;
        double change = d_here - d_next;
        if (found && change <= best_change) continue;
        found = 1;
        best_change = change;
        /* zero of the straight line through (beta_i, d_here), (beta_i+1, d_next) */
        *beta_x = beta[i] + (beta[i + 1] - beta[i]) * (d_here / (d_here - d_next));
    }
    return found ? ORC_OK : ORC_ERR_INVALID;
}

/* ------------------------------------------------------------------------ */
/* Whole run.                                                                */
/* ------------------------------------------------------------------------ */
static void observe(const orc_desc *d, uint32_t i, const uint8_t *spins, const int32_t *E,
                    uint64_t R_i, orc_result *out)
{
    uint32_t N = d->L * d->L;
    int64_t sum = 0;
    for (uint64_t k = 0; k < R_i; ++k) sum += E[k];
    out->R_i[i] = R_i;
    out->E_sum[i] = sum;
    if (out->digest) out->digest[i] = orc_digest(d, i, spins, R_i);
    /* eq. (4): population average. */
    out->E_mean[i] = (double)sum / (double)R_i;
    uint32_t *eh = out->hist ? out->hist + (uint64_t)i * (2 * N + 1)
                             : (uint32_t *)malloc(sizeof(uint32_t) * (2 * N + 1));
    if (eh) {
        memset(eh, 0, sizeof(uint32_t) * (2 * N + 1));
        for (uint64_t k = 0; k < R_i; ++k) eh[E[k] + (int32_t)(2 * N)]++;
        /* Sec. 4: width of the distribution of e = E/N over the population. */
        if (out->width_e) out->width_e[i] = orc_fwhm(eh, 2 * N + 1, d->bin_e) / (double)N;
        if (!out->hist) free(eh);
    }
    if (out->M_mean || out->Mt_sum || out->mhist || out->width_m) {
        /* eq. (5): M_k = (q M~_k - N) / (q - 1); eq. (4): the population mean
         * (1/R_i) sum_k M_k = (q sum_k M~_k - N R_i) / ((q - 1) R_i), taken from
         * the exact integer sum of M~ with one rounding. */
        int64_t mt_sum = 0;
        uint32_t *mh = out->mhist ? out->mhist + (uint64_t)i * (N + 1)
                                  : (uint32_t *)malloc(sizeof(uint32_t) * (N + 1));
        if (mh) memset(mh, 0, sizeof(uint32_t) * (N + 1));
        for (uint64_t k = 0; k < R_i; ++k) {
            uint32_t mt = orc_mtilde(d->L, d->q, spins + k * N);
            mt_sum += mt;
            if (mh) mh[mt]++;
        }
        if (out->Mt_sum) out->Mt_sum[i] = mt_sum;
        if (out->M_mean)
            out->M_mean[i] = ((double)d->q * (double)mt_sum - (double)N * (double)R_i) /
                             ((double)(d->q - 1) * (double)R_i);
        /* Sec. 4: width of the distribution of m = M/N; by eq. (5) one level of
         * M~ is q / ((q - 1) N) in m. */
        if (out->width_m && mh)
            out->width_m[i] = (orc_fwhm(mh, N + 1, d->bin_m) * (double)d->q) /
                              ((double)(d->q - 1) * (double)N);
        if (!out->mhist) free(mh);
    }
}

/* Steps i0+1 .. K-1 (steps 2-5 of the algorithm) from the population pop[0]
 * of R_prev replicas with energies E[0] at step i0, whose -beta F is
 * out->minus_beta_F[i0] and which has been observed.  pop and E hold two
 * buffers of R_cap replicas each; anc and hist are work arrays. */
static int run_steps(const orc_desc *d, uint32_t i0, uint64_t R_prev, const uint64_t *R_sched,
                     uint32_t Kb, uint8_t *pop[2], int32_t *E[2], uint32_t *anc, uint32_t *hist,
                     orc_result *out)
{
    uint32_t N = d->L * d->L;
    int cur = 0;
    for (uint32_t i = i0 + 1; i < d->K; ++i) {
        double dbeta = d->beta[i] - d->beta[i - 1];
        /* eq. (2): ln Q_i from the population at beta_{i-1}. */
        memset(hist, 0, sizeof(uint32_t) * (2 * N + 1));
        for (uint64_t k = 0; k < R_prev; ++k) hist[E[cur][k] + (int32_t)(2 * N)]++;
        double lnQ = orc_lnQ(N, dbeta, hist, R_prev, NULL);
        out->lnQ[i] = lnQ;
        out->minus_beta_F[i] = out->minus_beta_F[i - 1] + lnQ;

        uint64_t R_new = R_sched[i];
        int rc = orc_step(d, i, Kb, pop[cur], E[cur], R_prev, R_new, pop[1 - cur], E[1 - cur], anc);
        if (rc) return rc;
        cur = 1 - cur;
        R_prev = R_new;
        observe(d, i, pop[cur], E[cur], R_prev, out);
    }
    if (out->final_spins) memcpy(out->final_spins, pop[cur], R_prev * N);
    if (out->final_E) memcpy(out->final_E, E[cur], sizeof(int32_t) * R_prev);
    if (out->last_anc) {
        if (d->K > i0 + 1) memcpy(out->last_anc, anc, sizeof(uint32_t) * R_prev);
        else for (uint64_t k = 0; k < R_prev; ++k) out->last_anc[k] = (uint32_t)k;
    }
    return ORC_OK;
}

/* Whole run (steps 1-5), or its continuation from a population at step i0
 * (spins != NULL: R0 replicas, -beta F = mbF0). */
static int run_from(const orc_desc *d, uint32_t i0, uint64_t R0, const uint8_t *spins, double mbF0,
                    orc_result *out)
{
    int rc = orc_validate(d);
    if (rc) return rc;
    if (i0 >= d->K) return ORC_ERR_INVALID;
    uint32_t N = d->L * d->L;
    uint64_t *R_sched = (uint64_t *)malloc(sizeof(uint64_t) * d->K);
    if (!R_sched) return ORC_ERR_NOMEM;
    uint64_t R_cap;
    uint32_t Kb;
    rc = orc_plan(d, R_sched, &R_cap, &Kb);
    if (rc) { free(R_sched); return rc; }
    if (spins && (R0 == 0 || R0 > R_cap)) { free(R_sched); return ORC_ERR_INVALID; }

    uint8_t *pop[2];
    pop[0] = (uint8_t *)malloc(R_cap * N);
    pop[1] = (uint8_t *)malloc(R_cap * N);
    int32_t *E[2];
    E[0] = (int32_t *)malloc(sizeof(int32_t) * R_cap);
    E[1] = (int32_t *)malloc(sizeof(int32_t) * R_cap);
    uint32_t *anc = (uint32_t *)malloc(sizeof(uint32_t) * R_cap);
    uint32_t *hist = (uint32_t *)malloc(sizeof(uint32_t) * (2 * N + 1));
    if (!pop[0] || !pop[1] || !E[0] || !E[1] || !anc || !hist) {
        rc = ORC_ERR_NOMEM;
        goto done;
    }
#ifdef _OPENMP
    out->n_threads = omp_get_max_threads();
#else
    out->n_threads = 1;
#endif

    if (!spins) {
        /* Step 1: R_0 = R replicas in equilibrium at beta_0. */
        R0 = d->R;
        int64_t nk = (int64_t)R0;
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < nk; ++k) {
            orc_init_replica(d, (uint64_t)k, pop[0] + (uint64_t)k * N);
            E[0][k] = orc_energy(d->L, pop[0] + (uint64_t)k * N);
        }
        observe(d, 0, pop[0], E[0], R0, out);
        out->lnQ[0] = 0.0;
        /* ln Z at beta_0: q^N at beta = 0 (Sec. 6); for the ground-state start
         * of a heating run Z = q e^{-beta E_0}, E_0 = -2N (eq. (7)-(8)). */
        if (d->init == ORC_INIT_GROUND)
            out->minus_beta_F[0] = log((double)d->q) + 2.0 * (double)N * d->beta[0];
        else
            out->minus_beta_F[0] = (double)N * log((double)d->q);
    } else {
        /* A population at step i0 (a checkpoint): energies recomputed, observed
         * at i0; its ln Q belongs to the step before and is reported as 0. */
        memcpy(pop[0], spins, R0 * N);
        int64_t nk = (int64_t)R0;
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < nk; ++k) E[0][k] = orc_energy(d->L, pop[0] + (uint64_t)k * N);
        observe(d, i0, pop[0], E[0], R0, out);
        out->lnQ[i0] = 0.0;
        out->minus_beta_F[i0] = mbF0;
    }
    rc = run_steps(d, i0, R0, R_sched, Kb, pop, E, anc, hist, out);
done:
    free(R_sched);
    free(pop[0]);
    free(pop[1]);
    free(E[0]);
    free(E[1]);
    free(anc);
    free(hist);
    return rc;
}

int orc_run(const orc_desc *d, orc_result *out)
{
    return run_from(d, 0, 0, NULL, 0.0, out);
}

int orc_run_from(const orc_desc *d, uint32_t step, uint64_t R_cur, const uint8_t *spins,
                 double minus_beta_F, orc_result *out)
{
    if (!spins) return ORC_ERR_INVALID;
    return run_from(d, step, R_cur, spins, minus_beta_F, out);
}

/* ------------------------------------------------------------------------ */
/* Checkpoint files of the GPU library (format stated in its C header): a    */
/* 128-byte little-endian header, beta[K] as IEEE doubles, then the spins.   */
/* Read here byte by byte from that statement, independently of the writer.  */
/* ------------------------------------------------------------------------ */
static uint64_t le_bytes(const unsigned char *b, int n)
{
    uint64_t v = 0;
    for (int i = n - 1; i >= 0; --i) v = (v << 8) | b[i];
    return v;
}

int orc_read_checkpoint(const char *path, orc_checkpoint *ck)
{
    memset(ck, 0, sizeof *ck);
    FILE *f = fopen(path, "rb");
    if (!f) return ORC_ERR_INVALID;
    unsigned char h[128];
    int rc = ORC_ERR_INVALID;
    if (fread(h, 1, 128, f) != 128 || memcmp(h, "PACKPT01", 8) != 0 || le_bytes(h + 8, 4) != 128)
        goto fail;
    ck->desc.L = (uint32_t)le_bytes(h + 12, 4);
    ck->desc.q = (uint32_t)le_bytes(h + 16, 4);
    ck->desc.K = (uint32_t)le_bytes(h + 20, 4);
    ck->desc.R = le_bytes(h + 24, 8);
    ck->desc.theta = (uint32_t)le_bytes(h + 32, 4);
    ck->desc.resample = (int32_t)(uint32_t)le_bytes(h + 36, 4);
    ck->desc.seed = le_bytes(h + 40, 8);
    ck->desc.init = (int32_t)(uint32_t)le_bytes(h + 48, 4);
    ck->desc.bin_e = (uint32_t)le_bytes(h + 56, 4);
    ck->desc.bin_m = (uint32_t)le_bytes(h + 60, 4);
    ck->step = (uint32_t)le_bytes(h + 64, 4);
    ck->R_cur = le_bytes(h + 72, 8);
    uint64_t bits = le_bytes(h + 80, 8);
    memcpy(&ck->minus_beta_F, &bits, 8);
    ck->E_sum = (int64_t)le_bytes(h + 88, 8);
    if (ck->desc.K == 0 || ck->step >= ck->desc.K || ck->R_cur == 0) goto fail;
    ck->beta = (double *)malloc(sizeof(double) * ck->desc.K);
    uint64_t bytes = ck->R_cur * (uint64_t)ck->desc.L * ck->desc.L;
    ck->spins = (uint8_t *)malloc(bytes ? bytes : 1);
    if (!ck->beta || !ck->spins) { rc = ORC_ERR_NOMEM; goto fail; }
    for (uint32_t i = 0; i < ck->desc.K; ++i) {
        unsigned char b[8];
        if (fread(b, 1, 8, f) != 8) goto fail;
        uint64_t v = le_bytes(b, 8);
        memcpy(&ck->beta[i], &v, 8);
    }
    if (fread(ck->spins, 1, bytes, f) != bytes) goto fail;
    ck->desc.beta = ck->beta;
    if (orc_validate(&ck->desc)) goto fail;
    fclose(f);
    return ORC_OK;
fail:
    fclose(f);
    orc_free_checkpoint(ck);
    return rc;
}

void orc_free_checkpoint(orc_checkpoint *ck)
{
    free(ck->beta);
    free(ck->spins);
    ck->beta = NULL;
    ck->spins = NULL;
}
