// pa_host.cpp -- host side of the population-annealing library: validation,
// plan (population schedule, Metropolis thresholds, resampling weight tables),
// workspace layout, the per-step launch sequence (in-LDS or tiled sweeps),
// batched runs and their HIP-graph replay, the serving loop (scheduler thread,
// device arena, continuous batching), the host-only analysis calls, and the C
// ABI of pa.h.
//
// The plan implements, on the host, the parts of Sec. 2 of arXiv:1704.01888
// whose arithmetic must be bit-identical everywhere: the population sizes
// R_i (eq. (1), drawn as R_i ~ Pois(R)), the integer acceptance thresholds of
// the Metropolis rounds (step 3) and the integer resampling weights (step 2).
#include "pa.h"
#include "pa_device.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

namespace {

thread_local std::string g_last_error;

pa_status fail(pa_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 on the host (Salmon et al., SC'11), for the plan stream.
// ---------------------------------------------------------------------------
void philox_host(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)p1;
        c[3] = (uint32_t)p0;
        c[0] = n0;
        c[2] = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Poisson(lambda) by inversion of u in [0,1): the support is visited in the
// order m, m+1, m-1, m+2, m-2, ... from the mode m = floor(lambda), with the
// pmf carried by its ratios from p(m) = exp(-lambda + m ln lambda - lgamma(m+1)).
uint64_t poisson_inversion(double lambda, double u) {
    const double m = std::floor(lambda);
    const double pm = std::exp(-lambda + m * std::log(lambda) - std::lgamma(m + 1.0));
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
        if (phi == 0.0 && (lo == 0.0 || plo == 0.0)) return (uint64_t)hi;
    }
}

// W[d] = round(2^Kb exp(-|dbeta| d)) for d < D, where D is the first d with
// W[d] == 0 (or 2N+1); the weights decrease with d, so every W beyond D is 0.
// Writes W[0..D) and returns D.
uint32_t weight_prefix(double abs_dbeta, uint32_t Kb, uint32_t N, std::vector<uint64_t> &W) {
    const uint32_t nb = 2 * N + 1;
    for (uint32_t d = 0; d < nb; ++d) {
        const double x = abs_dbeta * (double)d;
        const uint64_t w = (uint64_t)std::nearbyint(std::ldexp(std::exp(-x), (int)Kb));
        if (w == 0) return d;
        W.push_back(w);
    }
    return nb;
}

uint32_t weight_table(double abs_dbeta, uint32_t Kb, uint32_t N, uint64_t *W) {
    std::vector<uint64_t> pre;
    const uint32_t D = weight_prefix(abs_dbeta, Kb, N, pre);
    for (uint32_t d = 0; d < 2 * N + 1; ++d) W[d] = d < D ? pre[d] : 0u;
    return D;
}

// Full width at half maximum (Sec. 4), in histogram levels, from the integer
// part the device finds (H, jl, jr and the counts of bins jl-1, jl, jr, jr+1
// in bins of B levels): the crossings of H/2 of the straight lines through
// the counts at the bin indices jl-1, jl and jr, jr+1; zero for an empty
// histogram.
double fwhm_levels(const uint64_t *f, uint32_t B) {
    const uint64_t H = f[0];
    if (H == 0) return 0.0;
    const double half = 0.5 * (double)H;
    const double l0 = (double)f[3], l1 = (double)f[4], r0 = (double)f[5], r1 = (double)f[6];
    const double xl = (double)((int64_t)f[1] - 1) + (half - l0) / (l1 - l0);
    const double xr = (double)f[2] + (r0 - half) / (r0 - r1);
    return (xr - xl) * (double)B;
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
// Elements per copy-count buffer: R_cap rounded up to 64 (256 bytes).
inline size_t counts_stride(uint64_t R_cap) { return (size_t)((R_cap + 63) & ~uint64_t(63)); }

struct Plan {
    pa_run_desc desc;
    std::vector<double> beta;
    uint32_t N = 0, nbins = 0;
    std::vector<uint64_t> R_sched;
    uint64_t R_cap = 0;
    uint32_t Kb = 0;
    std::vector<uint64_t> T;              // [K][4]
    std::vector<double> dbeta;            // [K], dbeta[0] = 0
    std::vector<uint32_t> table_of_step;  // [K]
    std::vector<uint64_t> W;              // the tables' nonzero prefixes, concatenated
    std::vector<uint64_t> W_off;          // [n_tables] start of table t in W
    std::vector<uint32_t> D;              // [n_tables] length of table t
    std::vector<double> abs_dbeta;        // [n_tables]
    uint32_t n_tables = 0;
    bool hist_all = false, mag = false, widths = false, digest = false;
    uint32_t bin_e = 1, bin_m = 1;
    // workspace layout
    size_t off_pop[2], off_E, off_C, off_r, off_anc, off_counts, off_hist, off_Esum,
        off_count, off_lnQ, off_mbF, off_Eref, off_W, off_mhist, off_Mt, off_Mtsum,
        off_fwe, off_fwm, off_bonds, off_cnt, off_pop_x, off_H, off_Hacc, off_digest, off_E2, off_Mt2, off_H2,
        off_steps, steps_bytes, off_anc2, off_counts2, total;
    bool tiled = false;   // replicas beyond one workgroup's LDS: tiled half-sweeps in HBM
    // a population small enough to resample in one workgroup inside the post
    // launch of the step before; its ancestors and copy numbers alternate
    // between two buffers by step parity
    bool small = false;
};

pa_status validate(const pa_run_desc *d) {
    if (!d) return fail(PA_ERR_INVALID, "null run description");
    if (d->L < 2 || (d->L & 1u)) return fail(PA_ERR_INVALID, "L must be even and >= 2");
    if (d->q < 2 || d->q > 255) return fail(PA_ERR_INVALID, "q must be in [2, 255]");
    if (d->R < 1 || d->R > (1ull << 31)) return fail(PA_ERR_INVALID, "R must be in [1, 2^31]");
    if (d->K < 1 || !d->beta) return fail(PA_ERR_INVALID, "K must be >= 1 with a beta array");
    if (d->theta >= (1u << 27)) return fail(PA_ERR_INVALID, "theta must be < 2^27");
    if (d->resample < 0 || d->resample > 2) return fail(PA_ERR_INVALID, "bad resample mode");
    if (d->init < 0 || d->init > 1) return fail(PA_ERR_INVALID, "bad init mode");
    for (uint32_t i = 0; i < d->K; ++i)
        if (!std::isfinite(d->beta[i]) || d->beta[i] < 0.0)
            return fail(PA_ERR_INVALID, "beta must be finite and >= 0");
    if (d->init == PA_INIT_RANDOM && d->beta[0] != 0.0)
        return fail(PA_ERR_INVALID, "a random initial population needs beta[0] == 0");
    if (d->outputs & ~(uint32_t)(PA_OUT_HIST | PA_OUT_MAG | PA_OUT_FINAL | PA_OUT_WIDTHS | PA_OUT_DIGEST))
        return fail(PA_ERR_INVALID, "unknown output bits");
    if (d->bin_e > 2 * d->L * d->L + 1 || d->bin_m > d->L * d->L + 1)
        return fail(PA_ERR_INVALID, "histogram bin wider than the histogram");
    if (d->L > 4096 || ((d->L & 3u) && d->L > 254))
        return fail(PA_ERR_UNSUPPORTED,
                    "this device path needs L <= 4096, and L <= 254 when L is not a multiple of 4");
    return PA_OK;
}

pa_status plan_layout(const pa_run_desc *d, Plan &p);

// `like`, if set, is the plan of a run with the same L, K and beta schedule
// (bit for bit): its thresholds and weight tables, which depend on nothing
// else (the weights also on K_b), are copied rather than recomputed.
pa_status build_plan(const pa_run_desc *d, Plan &p, const Plan *like = nullptr) {
    pa_status st = validate(d);
    if (st) return st;
    p.desc = *d;
    p.beta.assign(d->beta, d->beta + d->K);
    p.desc.beta = p.beta.data();
    p.N = d->L * d->L;
    p.nbins = 2 * p.N + 1;
    const uint32_t K = d->K;

    // Population sizes (eq. (1) through R_i ~ Pois(R)); one uniform per step
    // from Philox(0, 0, i, PLAN << 28).
    p.R_sched.assign(K, d->R);
    uint64_t cap = d->R;
    const uint32_t k0 = (uint32_t)(d->seed & 0xffffffffu), k1 = (uint32_t)(d->seed >> 32);
    for (uint32_t i = 1; i < K; ++i) {
        uint64_t n = d->R;
        if (d->resample == PA_RESAMPLE_POISSON) {
            uint32_t c[4] = {0u, 0u, i, (uint32_t)pa::DOM_PLAN << 28};
            philox_host(c, k0, k1);
            const uint64_t x = ((uint64_t)c[1] << 32) | (uint64_t)c[0];
            const double u = std::ldexp((double)(x >> 11), -53);
            n = poisson_inversion((double)d->R, u);
            if (n == 0 || n > (1ull << 31))
                return fail(PA_ERR_CAPACITY, "Poisson schedule drew an empty or oversized population");
        }
        p.R_sched[i] = n;
        if (n > cap) cap = n;
    }
    p.R_cap = cap;
    uint32_t lg = 0;
    while ((1ull << lg) < cap) ++lg;
    p.Kb = 63u - lg;

    if (like) {
        p.T = like->T;
        p.dbeta = like->dbeta;
        p.table_of_step = like->table_of_step;
        p.n_tables = like->n_tables;
        p.abs_dbeta = like->abs_dbeta;
        if (like->Kb == p.Kb) {
            p.W = like->W;
            p.W_off = like->W_off;
            p.D = like->D;
        } else {
            p.W.clear();
            p.W_off.assign(p.n_tables, 0);
            p.D.assign(p.n_tables, 0);
            for (uint32_t t = 0; t < p.n_tables; ++t) {
                p.W_off[t] = p.W.size();
                p.D[t] = p.abs_dbeta[t] == 0.0 ? 0u : weight_prefix(p.abs_dbeta[t], p.Kb, p.N, p.W);
            }
        }
        return plan_layout(d, p);
    }
    // Metropolis thresholds floor(2^32 exp(-beta_i dE)), dE = 1..4.
    p.T.assign((size_t)K * 4, 0);
    for (uint32_t i = 0; i < K; ++i)
        for (uint32_t dE = 1; dE <= 4; ++dE) {
            const double x = p.beta[i] * (double)dE;
            p.T[(size_t)i * 4 + dE - 1] = (uint64_t)std::floor(std::ldexp(std::exp(-x), 32));
        }

    // One weight table per distinct |beta_i - beta_{i-1}|.
    p.dbeta.assign(K, 0.0);
    p.table_of_step.assign(K, 0);
    std::unordered_map<uint64_t, uint32_t> seen;
    std::vector<double> abs_list;
    for (uint32_t i = 1; i < K; ++i) {
        p.dbeta[i] = p.beta[i] - p.beta[i - 1];
        const double a = std::fabs(p.dbeta[i]);
        uint64_t bits;
        std::memcpy(&bits, &a, sizeof bits);
        auto it = seen.find(bits);
        if (it == seen.end()) {
            const uint32_t id = (uint32_t)abs_list.size();
            seen.emplace(bits, id);
            abs_list.push_back(a);
            p.table_of_step[i] = id;
        } else {
            p.table_of_step[i] = it->second;
        }
    }
    if (abs_list.empty()) abs_list.push_back(0.0);
    p.n_tables = (uint32_t)abs_list.size();
    p.abs_dbeta = abs_list;
    // Weight tables: only the nonzero prefix of each (Sec. 2 step 2 weights of
    // one |dbeta|); its length bounds the workspace, so it is computed always.
    p.W.clear();
    p.W_off.assign(p.n_tables, 0);
    p.D.assign(p.n_tables, 0);
    for (uint32_t t = 0; t < p.n_tables; ++t) {
        p.W_off[t] = p.W.size();
        // dbeta = 0: every weight is 2^Kb, no table
        p.D[t] = abs_list[t] == 0.0 ? 0u : weight_prefix(abs_list[t], p.Kb, p.N, p.W);
    }
    return plan_layout(d, p);
}

// The workspace layout of plan p (tables built) for description d.
pa_status plan_layout(const pa_run_desc *d, Plan &p) {
    const uint32_t K = d->K;
    p.hist_all = (d->outputs & PA_OUT_HIST) != 0;
    p.mag = (d->outputs & PA_OUT_MAG) != 0;
    p.widths = (d->outputs & PA_OUT_WIDTHS) != 0;
    p.digest = (d->outputs & PA_OUT_DIGEST) != 0;
    p.bin_e = d->bin_e ? d->bin_e : 1u;
    p.bin_m = d->bin_m ? d->bin_m : 1u;
    size_t o = 0;
    const size_t popb = align256((size_t)p.R_cap * p.N);
    p.off_pop[0] = o; o += popb;
    p.off_pop[1] = o; o += popb;
    p.off_E = o; o += align256(4 * p.R_cap);
    p.off_C = o; o += align256(8 * p.R_cap);
    // copy counts, one buffer per step parity, each starting 256-byte aligned
    // (the kernels read and clear them in 16-byte pieces)
    p.off_r = o; o += 4 * 2 * counts_stride(p.R_cap);
    p.off_anc = o; o += align256(4 * p.R_cap);
    p.off_counts = o; o += align256(4 * p.R_cap);
    p.off_hist = o; o += align256((size_t)4 * p.nbins * (p.hist_all ? K : 1));
    // the per-step results, one block (read back in one copy)
    p.off_steps = o;
    p.off_Esum = o; o += align256(8 * (size_t)K);
    p.off_count = o; o += align256(8 * (size_t)K);
    p.off_lnQ = o; o += align256(8 * (size_t)K);
    p.off_mbF = o; o += align256(8 * (size_t)K);
    p.off_Mtsum = o; o += p.mag ? align256(8 * (size_t)K) : 0;
    p.off_fwe = o; o += p.widths ? align256(64 * (size_t)K) : 0;
    p.off_fwm = o; o += (p.widths && p.mag) ? align256(64 * (size_t)K) : 0;
    p.off_digest = o; o += p.digest ? align256(8 * (size_t)K) : 0;
    p.steps_bytes = o - p.off_steps;
    p.off_Eref = o; o += align256(4 * (size_t)K);
    p.off_W = o; o += align256((size_t)8 * p.W.size());
    p.off_mhist = o; o += p.mag ? align256((size_t)4 * (p.N + 1) * (p.hist_all ? K : 1)) : 0;
    p.off_Mt = o; o += p.mag ? align256(4 * p.R_cap) : 0;
    p.tiled = pa::tiled_path(d->L);
    p.off_bonds = o; o += p.tiled ? align256(4 * p.R_cap) : 0;
    p.off_cnt = o; o += (p.tiled && p.mag) ? align256((size_t)4 * p.R_cap * d->q) : 0;
    p.off_pop_x = o; o += p.tiled ? popb : 0;   // third population buffer of the tiled sweeps
    p.off_H = o; o += p.digest ? align256(8 * p.R_cap) : 0;
    p.off_Hacc = o; o += (p.digest && p.tiled) ? align256(8 * p.R_cap) : 0;
    // second energy, M~ and digest-term buffers: the team launch alternates
    // them by step (the statistics of one step and the sweeps of the next run
    // at the same time)
    p.off_E2 = o; o += p.tiled ? 0 : align256(4 * p.R_cap);
    p.off_Mt2 = o; o += (!p.tiled && p.mag) ? align256(4 * p.R_cap) : 0;
    p.off_H2 = o; o += (!p.tiled && p.digest) ? align256(8 * p.R_cap) : 0;
    p.small = !p.tiled && p.desc.resample != PA_RESAMPLE_NONE && p.R_cap <= pa::SMALL_RESAMPLE_MAX;
    p.off_anc2 = o; o += p.small ? align256(4 * p.R_cap) : 0;
    p.off_counts2 = o; o += p.small ? align256(4 * p.R_cap) : 0;
    p.total = o;
    return PA_OK;
}

}  // namespace

struct Server;

struct GraphCache {
    std::string key;
    hipGraphExec_t exec = nullptr;
};

struct pa_ctx {
    int device;
    int profiling;
    uint32_t lanes[pa::LANE_CHOICE_COUNT];   // chosen lanes per replica per lattice with choices (0 = default)
    // The serving loop, shared with the pa_serve_* calls in flight: a call
    // takes a reference under serve_mu, so that pa_serve_stop can drop the
    // context's reference while waits still use the server.
    std::shared_ptr<Server> server;
    std::mutex serve_mu;
    int graphs;          // batched runs replay a captured HIP graph
    int batch_mode;      // PA_BATCH_SEGMENTED (default) or PA_BATCH_TEAM
    uint32_t *team_abort;   // pinned host word read by the team launches' barrier waits
    std::atomic<int> abort_requested;
    uint32_t team_runs, team_launches;   // of the last pa_run_batch
    // tuned sweep shapes by (L, q above 128, population class); guarded by
    // tune_mu (the serving thread reads them too); tune_gen counts changes
    std::mutex tune_mu;
    std::map<uint64_t, pa_tune_entry> tune;
    uint64_t tune_gen;
    uint32_t tune_try_G, tune_try_wpb;   // the shape pa_tune is timing (0: none)
    // pa_run_batch calls on a context take turns; their descriptor records
    // go up from pinned host memory (asynchronous copies)
    std::mutex batch_mu;
    uint8_t *staging;
    size_t staging_bytes;
    hipStream_t graph_stream;
    hipEvent_t ev_in, ev_out;
    std::deque<GraphCache> graph_cache;
};

// Pinned host memory of at least `bytes` for the batch's copies (the caller
// holds batch_mu; a batch synchronises its stream before it returns).
static uint8_t *ctx_staging(pa_ctx *c, size_t bytes, hipStream_t s) {
    if (bytes > c->staging_bytes) {
        // copies from the old buffer may still be in flight on the stream
        if (hipStreamSynchronize(s) != hipSuccess) return nullptr;
        if (c->staging) (void)hipHostFree(c->staging);
        c->staging = nullptr;
        c->staging_bytes = 0;
        void *h = nullptr;
        const size_t want = std::max(bytes, size_t(1) << 20);
        if (hipHostMalloc(&h, want, hipHostMallocDefault) != hipSuccess || !h) return nullptr;
        c->staging = static_cast<uint8_t *>(h);
        c->staging_bytes = want;
    }
    return c->staging;
}

// Population classes of the tuned shapes: R_cap below 2^11, 2^14, 2^17, or above.
static uint32_t r_class_of(uint64_t R_cap) {
    return R_cap < (1ull << 11) ? 0u : R_cap < (1ull << 14) ? 1u : R_cap < (1ull << 17) ? 2u : 3u;
}
static uint64_t tune_key(uint32_t L, uint32_t q_large, uint32_t r_class) {
    return ((uint64_t)L << 8) | ((uint64_t)(q_large != 0) << 4) | r_class;
}

static uint32_t ctx_lanes(const pa_ctx *c, uint32_t L) {
    const int i = pa::lane_choice_index(L);
    return (c && i >= 0) ? c->lanes[i] : 0u;
}

struct pa_run_state {
    pa_ctx *ctx;
    Plan plan;
    uint8_t *ws;
    hipStream_t stream;
    uint32_t step;       // current step (population at beta_step)
    int cur;             // pop buffer holding the current population
    uint64_t R_cur, R_prev;
    uint64_t r_dirty[2];  // extent of nonzero copy counts in each parity buffer
    uint32_t G, wpb;     // sweep shape: lanes per replica, waves per workgroup
    double mbF0;
    uint32_t first_step;  // step of the initial or loaded population
    uint64_t R_first;
    bool broken;
    struct Timed { int kind; hipEvent_t a, b; };
    std::vector<Timed> timed;
    template <typename T> T *at(size_t off) { return reinterpret_cast<T *>(ws + off); }
};

namespace {

pa_status hip_check(pa_run_state *r, hipError_t e, const char *what) {
    if (e == hipSuccess) return PA_OK;
    if (r) r->broken = true;
    return fail(PA_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Launch through `fn`, bracketed by HIP events on the run's stream when the
// context profiles.
template <typename F>
pa_status timed_launch(pa_run_state *r, int kind, const char *what, F fn) {
    hipEvent_t a = nullptr, b = nullptr;
    const bool prof = r->ctx && r->ctx->profiling;
    if (prof) {
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
            return fail(PA_ERR_DEVICE, "hipEventCreate");
        (void)hipEventRecord(a, r->stream);
    }
    pa_status st = hip_check(r, fn(), what);
    if (prof) {
        (void)hipEventRecord(b, r->stream);
        r->timed.push_back({kind, a, b});
    }
    return st;
}

void release_events(pa_run_state *r, double *ms, uint64_t *count) {
    if (ms) for (int k = 0; k < PA_KERNEL_KINDS; ++k) ms[k] = 0.0;
    if (count) for (int k = 0; k < PA_KERNEL_KINDS; ++k) count[k] = 0;
    for (auto &t : r->timed) {
        float e = 0.f;
        if (ms && hipEventElapsedTime(&e, t.a, t.b) == hipSuccess) ms[t.kind] += e;
        if (count) count[t.kind] += 1;
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    r->timed.clear();
}

// Histogram buffers: one per step when they are outputs, else one reused.
uint32_t *hist_of(pa_run_state *r, uint32_t i) {
    const Plan &p = r->plan;
    const size_t slot = p.hist_all ? i : 0u;
    return r->at<uint32_t>(p.off_hist) + slot * p.nbins;
}

uint32_t *mhist_of(pa_run_state *r, uint32_t i) {
    const Plan &p = r->plan;
    if (!p.mag) return nullptr;
    const size_t slot = p.hist_all ? i : 0u;
    return r->at<uint32_t>(p.off_mhist) + slot * (p.N + 1);
}

uint32_t *anc_of(pa_run_state *r, uint32_t i);
uint32_t *counts_of(pa_run_state *r, uint32_t i);
pa::SmallResample small_resample_args(pa_run_state *r, uint32_t i);

// Post-kernel arguments of step i (population size R_cur): statistics of step
// i, ln Q_{i+1}, and the weights of the resampling to i+1 (for a small
// population: the whole resampling to i+1).
pa::PostArgs post_args(pa_run_state *r, uint32_t i) {
    const Plan &p = r->plan;
    pa::PostArgs s{};
    s.hist = hist_of(r, i);
    s.store_hist = p.hist_all ? 1u : 0u;
    s.nbins = p.nbins;
    s.two_n = (int32_t)(2 * p.N);
    s.R_i = r->R_cur;
    s.step = i;
    s.has_next = (i + 1 < p.desc.K) ? 1u : 0u;
    s.dbeta_next = s.has_next ? p.dbeta[i + 1] : 0.0;
    const uint32_t tab = s.has_next ? p.table_of_step[i + 1] : 0;
    s.abs_dbeta_next = s.has_next ? p.abs_dbeta[tab] : 0.0;
    s.E_sum = r->at<int64_t>(p.off_Esum);
    s.count = r->at<uint64_t>(p.off_count);
    s.lnQ = r->at<double>(p.off_lnQ);
    s.mbF = r->at<double>(p.off_mbF);
    s.E_ref = r->at<int32_t>(p.off_Eref);
    s.do_weights = (s.has_next && p.desc.resample != PA_RESAMPLE_NONE) ? 1u : 0u;
    s.wblock = pa::scan_block(s.R_i);
    s.E = r->at<int32_t>(p.off_E);
    s.W = r->at<uint64_t>(p.off_W) + p.W_off[tab];
    s.D = p.D[tab];
    s.w_const = p.abs_dbeta[tab] == 0.0 ? (1ull << p.Kb) : 0ull;
    s.C = r->at<uint64_t>(p.off_C);
    s.Mt = p.mag ? r->at<uint32_t>(p.off_Mt) : nullptr;
    s.H = p.digest ? r->at<uint64_t>(p.off_H) : nullptr;
    s.digest = p.digest ? r->at<uint64_t>(p.off_digest) : nullptr;
    s.mhist = mhist_of(r, i);
    s.q = p.desc.q;
    s.N = p.N;
    s.Mt_sum = p.mag ? r->at<int64_t>(p.off_Mtsum) : nullptr;
    s.widths = p.widths ? 1u : 0u;
    s.bin_e = p.bin_e;
    s.bin_m = p.bin_m;
    s.fw_e = p.widths ? r->at<uint64_t>(p.off_fwe) : nullptr;
    s.fw_m = (p.widths && p.mag) ? r->at<uint64_t>(p.off_fwm) : nullptr;
    if (p.small && s.has_next) {      // the whole resampling into i+1 in one workgroup
        s.do_weights = 0;
        s.small = 1;
        s.rs = small_resample_args(r, i + 1);
    }
    return s;
}

pa_status launch_post_for(pa_run_state *r, uint32_t i) {
    const pa::PostArgs s = post_args(r, i);
    return timed_launch(r, PA_KERNEL_POST, "post kernel", [&] { return pa::launch_post(s, r->stream); });
}

pa::SweepArgs sweep_args(pa_run_state *r, uint32_t i, uint32_t mode, const uint8_t *old_pop,
                         const uint32_t *anc, uint8_t *new_pop, uint32_t theta) {
    const Plan &p = r->plan;
    pa::SweepArgs a{};
    a.old_pop = old_pop;
    a.anc = anc;
    a.new_pop = new_pop;
    a.E_out = r->at<int32_t>(p.off_E);
    a.Mt_out = p.mag ? r->at<uint32_t>(p.off_Mt) : nullptr;
    a.H_out = p.digest ? r->at<uint64_t>(p.off_H) : nullptr;
    for (int d = 0; d < 4; ++d) a.T[d] = p.T[(size_t)i * 4 + d];
    a.L = p.desc.L;
    a.q = p.desc.q;
    a.N = p.N;
    a.R_new = (uint32_t)r->R_cur;
    a.step = i;
    a.theta = theta;
    a.mode = mode;
    a.key0 = (uint32_t)(p.desc.seed & 0xffffffffu);
    a.key1 = (uint32_t)(p.desc.seed >> 32);
    a.G = r->G;
    a.waves_per_block = r->wpb;
    return a;
}

// Tiled (large-lattice) launches of step i on R_cur replicas.
pa::TiledArgs tiled_args(pa_run_state *r, uint32_t i, const uint8_t *src, const uint32_t *anc,
                         uint8_t *dst) {
    const Plan &p = r->plan;
    pa::TiledArgs a{};
    a.src = src;
    a.anc = anc;
    a.dst = dst;
    for (int d = 0; d < 4; ++d) a.T[d] = p.T[(size_t)i * 4 + d];
    a.L = p.desc.L;
    a.q = p.desc.q;
    a.N = p.N;
    a.R = (uint32_t)r->R_cur;
    a.rows = pa::tiled_rows(p.desc.L);
    a.tiles = (p.desc.L + a.rows - 1) / a.rows;
    a.step = i;
    a.key0 = (uint32_t)(p.desc.seed & 0xffffffffu);
    a.key1 = (uint32_t)(p.desc.seed >> 32);
    a.init = p.desc.init == PA_INIT_GROUND ? pa::SWEEP_INIT_GROUND : pa::SWEEP_INIT_RANDOM;
    a.bonds = r->at<uint32_t>(p.off_bonds);
    a.cnt = p.mag ? r->at<uint32_t>(p.off_cnt) : nullptr;
    a.Hacc = p.digest ? r->at<uint64_t>(p.off_Hacc) : nullptr;
    a.H_out = p.digest ? r->at<uint64_t>(p.off_H) : nullptr;
    a.E_out = r->at<int32_t>(p.off_E);
    a.Mt_out = p.mag ? r->at<uint32_t>(p.off_Mt) : nullptr;
    return a;
}

// theta tiled sweeps from src (through anc) into dst, then the energies
// (theta = 0 copies).  A launch that fuses several half-sweeps recomputes the
// rows next to its tile, so it must not read rows that neighbouring tiles of
// the same launch write: no launch works in place.  The launches alternate
// between dst and the spare buffer `x`, the last one writing dst.
hipError_t launch_tiled_sweeps(pa::TiledArgs a, uint32_t theta, uint8_t *x, hipStream_t s) {
    hipError_t e;
    const uint32_t total = 2 * theta, S = pa::tiled_max_halves(a.L);
    const uint32_t launches = total == 0 ? 1u : (total + S - 1) / S;
    uint8_t *const dst = a.dst;
    a.h0 = 0;
    for (uint32_t i = 0; i < launches; ++i) {
        a.halves = std::min(total - a.h0, S);
        a.dst = ((launches - 1 - i) & 1u) ? x : dst;
        if ((e = pa::launch_tiled_half(a, s)) != hipSuccess) return e;
        a.src = a.dst;
        a.anc = nullptr;
        a.h0 += a.halves;
    }
    return pa::launch_tiled_measure(a, s);
}

// Copy-count buffer of step parity `par`.
uint32_t *counts_buf(pa_run_state *r, uint32_t par) {
    return r->at<uint32_t>(r->plan.off_r) + (size_t)(par & 1u) * counts_stride(r->plan.R_cap);
}

// Records of the resampling into step i (draws from the R_prev replicas of
// step i-1, R_new of them).  The draws count into the buffer of parity i,
// which is zero; the count scan clears the other buffer for step i+1.
// The ancestors and copy numbers of the resampling into step i.
uint32_t *anc_of(pa_run_state *r, uint32_t i) {
    const Plan &p = r->plan;
    return r->at<uint32_t>(p.small && (i & 1u) ? p.off_anc2 : p.off_anc);
}
uint32_t *counts_of(pa_run_state *r, uint32_t i) {
    const Plan &p = r->plan;
    return r->at<uint32_t>(p.small && (i & 1u) ? p.off_counts2 : p.off_counts);
}

// The resampling into step i of a small population, done by the post launch
// of step i-1 from its energies (r->R_cur = R_{i-1}).
pa::SmallResample small_resample_args(pa_run_state *r, uint32_t i) {
    const Plan &p = r->plan;
    pa::SmallResample t{};
    t.E_prev = r->at<int32_t>(p.off_E);
    t.anc_out = anc_of(r, i);
    t.counts_out = counts_of(r, i);
    t.R_prev = r->R_cur;
    t.n_new = p.R_sched[i];
    const uint32_t tab = p.table_of_step[i];
    t.W = r->at<uint64_t>(p.off_W) + p.W_off[tab];
    t.D = p.D[tab];
    t.w_const = p.abs_dbeta[tab] == 0.0 ? (1ull << p.Kb) : 0ull;
    t.ref_max = p.dbeta[i] < 0.0 ? 1u : 0u;
    t.resample = p.desc.resample != PA_RESAMPLE_NONE ? 1u : 0u;
    t.step = i;
    t.key0 = (uint32_t)(p.desc.seed & 0xffffffffu);
    t.key1 = (uint32_t)(p.desc.seed >> 32);
    return t;
}

void resample_args(pa_run_state *r, uint32_t i, uint64_t R_prev, uint64_t R_new, pa::SampleArgs &s,
                   pa::SlotmapArgs &m) {
    const Plan &p = r->plan;
    s = pa::SampleArgs{};
    s.C = r->at<uint64_t>(p.off_C);
    s.R_prev = R_prev;
    s.n_new = R_new;
    s.step = i;
    s.key0 = (uint32_t)(p.desc.seed & 0xffffffffu);
    s.key1 = (uint32_t)(p.desc.seed >> 32);
    s.r = counts_buf(r, i);
    m = pa::SlotmapArgs{};
    m.r = s.r;
    m.R_prev = R_prev;
    m.anc = r->at<uint32_t>(p.off_anc);
    m.anc_cap = p.R_cap;
    m.counts_last = r->at<uint32_t>(p.off_counts);
    m.block = pa::scan_block(R_prev);
    m.r_clear = counts_buf(r, i + 1);
    m.clear_n = r->r_dirty[(i + 1) & 1u];
    r->r_dirty[(i + 1) & 1u] = 0;
    r->r_dirty[i & 1u] = R_prev;
}

pa_status do_step(pa_run_state *r) {
    const Plan &p = r->plan;
    const uint32_t i = r->step + 1;
    const uint64_t R_prev = r->R_cur, R_new = p.R_sched[i];
    pa_status st;
    const uint32_t *anc = nullptr;
    if (p.small) {
        anc = anc_of(r, i);              // written by the post launch of step i-1
    } else if (p.desc.resample != PA_RESAMPLE_NONE) {
        // C (inclusive weight scan over the step i-1 population) was written
        // by the post kernel of step i-1.
        pa::SampleArgs s;
        pa::SlotmapArgs m;
        resample_args(r, i, R_prev, R_new, s, m);
        if ((st = timed_launch(r, PA_KERNEL_RESAMPLE, "resample kernel",
                               [&] { return pa::launch_resample(s, m, r->stream); })))
            return st;
        anc = m.anc;
    } else if (R_new != R_prev) {
        return fail(PA_ERR_INVALID, "resampling off needs a constant population");
    }
    r->R_prev = R_prev;
    r->R_cur = R_new;
    const uint8_t *old_pop = r->at<uint8_t>(p.off_pop[r->cur]);
    uint8_t *new_pop = r->at<uint8_t>(p.off_pop[1 - r->cur]);
    if (p.tiled) {
        const pa::TiledArgs ta = tiled_args(r, i, old_pop, anc, new_pop);
        uint8_t *x = r->at<uint8_t>(p.off_pop_x);
        if ((st = timed_launch(r, PA_KERNEL_SWEEP, "tiled sweep kernels",
                               [&] { return launch_tiled_sweeps(ta, p.desc.theta, x, r->stream); })))
            return st;
    } else {
        pa::SweepArgs a = sweep_args(r, i, pa::SWEEP_UPDATE, old_pop, anc, new_pop, p.desc.theta);
        if ((st = timed_launch(r, PA_KERNEL_SWEEP, "sweep kernel", [&] { return pa::launch_sweep(a, r->stream); })))
            return st;
    }
    r->cur = 1 - r->cur;
    r->step = i;
    return launch_post_for(r, i);
}

}  // namespace

extern "C" {

const char *pa_status_str(pa_status s) {
    switch (s) {
        case PA_OK: return "ok";
        case PA_ERR_INVALID: return "invalid argument";
        case PA_ERR_NOMEM: return "workspace too small";
        case PA_ERR_DEVICE: return "device error";
        case PA_ERR_CAPACITY: return "population capacity";
        case PA_ERR_UNSUPPORTED: return "unsupported on this device path";
        case PA_ERR_BUSY: return "busy";
        case PA_ERR_CANCELLED: return "cancelled";
        case PA_ERR_TIMEOUT: return "timed out";
    }
    return "unknown status";
}

const char *pa_last_error(void) { return g_last_error.c_str(); }

pa_status pa_plan(const pa_run_desc *desc, pa_plan_info *info) {
    if (!info) return fail(PA_ERR_INVALID, "null plan info");
    Plan p;
    pa_status st = build_plan(desc, p);
    if (st) return st;
    info->R_cap = p.R_cap;
    info->R_final = p.R_sched.back();
    info->workspace_bytes = p.total;
    info->Kb = p.Kb;
    info->n_tables = p.n_tables;
    return PA_OK;
}

pa_status pa_plan_tables(const pa_run_desc *desc, uint64_t *T, uint64_t *R_sched) {
    Plan p;
    pa_status st = build_plan(desc, p);
    if (st) return st;
    if (T) std::memcpy(T, p.T.data(), sizeof(uint64_t) * p.T.size());
    if (R_sched) std::memcpy(R_sched, p.R_sched.data(), sizeof(uint64_t) * p.R_sched.size());
    return PA_OK;
}

pa_status pa_weight_table(double abs_dbeta, uint32_t Kb, uint32_t N, uint64_t *W, uint32_t *D) {
    if (!W || !D || Kb > 63 || !(abs_dbeta >= 0.0)) return fail(PA_ERR_INVALID, "bad weight table request");
    *D = weight_table(abs_dbeta, Kb, N, W);
    return PA_OK;
}

pa_status pa_width_maxima(const double *beta, const double *width, uint32_t K, uint32_t *i_max,
                          double *w_max, double *T_max) {
    if (!beta || !width || K == 0) return fail(PA_ERR_INVALID, "empty width curve");
    uint32_t best = 0;
    for (uint32_t i = 0; i < K; ++i) {
        if (std::isnan(width[i])) return fail(PA_ERR_INVALID, "NaN width");
        if (width[i] > width[best]) best = i;
    }
    if (i_max) *i_max = best;
    if (w_max) *w_max = width[best];
    if (T_max) *T_max = 1.0 / beta[best];
    return PA_OK;
}

pa_status pa_free_energy_crossing(const double *beta, const double *mbf_cool, const double *mbf_heat,
                                  uint32_t K, double *beta_x) {
    if (!beta || !mbf_cool || !mbf_heat || !beta_x || K < 2) return fail(PA_ERR_INVALID, "need two or more points");
    for (uint32_t i = 0; i + 1 < K; ++i)
        if (!(beta[i + 1] > beta[i])) return fail(PA_ERR_INVALID, "beta must increase strictly");
    double jump = -1.0;
    for (uint32_t i = 0; i + 1 < K; ++i) {
        const double d0 = mbf_cool[i] - mbf_heat[i], d1 = mbf_cool[i + 1] - mbf_heat[i + 1];
        if (d0 > 0.0 && d1 <= 0.0 && d0 - d1 > jump) {
            jump = d0 - d1;
            *beta_x = beta[i] + (beta[i + 1] - beta[i]) * (d0 / (d0 - d1));
        }
    }
    if (jump < 0.0) return fail(PA_ERR_INVALID, "the cooling and heating estimates do not cross");
    return PA_OK;
}

pa_status pa_ctx_create(int device, pa_ctx **out) {
    if (!out) return fail(PA_ERR_INVALID, "null output");
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || device < 0 || device >= n)
        return fail(PA_ERR_DEVICE, "no such HIP device");
    // the fixed workspace of pa_run_static: its device address on this device,
    // looked up with the device current
    int prev = 0;
    (void)hipGetDevice(&prev);
    hipError_t se = hipSetDevice(device);
    if (se == hipSuccess) (void)pa::static_scratch(device, &se);
    (void)hipSetDevice(prev);
    if (se != hipSuccess) return fail(PA_ERR_DEVICE, std::string("static workspace: ") + hipGetErrorString(se));
    // the abort word of the team launches: pinned, coherent host memory the
    // kernels poll while they wait at a barrier
    void *abort_word = nullptr;
    if (hipHostMalloc(&abort_word, 256, hipHostMallocCoherent) != hipSuccess || !abort_word)
        return fail(PA_ERR_DEVICE, "cannot allocate the abort word");
    *static_cast<volatile uint32_t *>(abort_word) = 0u;
    pa_ctx *c = new (std::nothrow) pa_ctx;
    if (!c) {
        (void)hipHostFree(abort_word);
        return fail(PA_ERR_NOMEM, "out of host memory");
    }
    c->device = device;
    c->profiling = 0;
    for (auto &x : c->lanes) x = 0;
    c->graphs = 0;
    c->batch_mode = PA_BATCH_SEGMENTED;
    c->team_abort = static_cast<uint32_t *>(abort_word);
    c->abort_requested = 0;
    c->team_runs = c->team_launches = 0;
    c->staging = nullptr;
    c->staging_bytes = 0;
    c->tune_gen = 0;
    c->tune_try_G = c->tune_try_wpb = 0;
    c->graph_stream = nullptr;
    c->ev_in = c->ev_out = nullptr;
    *out = c;
    return PA_OK;
}

void pa_ctx_destroy(pa_ctx *ctx) {
    if (!ctx) return;
    bool serving;
    {
        std::lock_guard<std::mutex> lk(ctx->serve_mu);
        serving = ctx->server != nullptr;
    }
    if (serving) pa_serve_stop(ctx);
    for (auto &g : ctx->graph_cache) (void)hipGraphExecDestroy(g.exec);
    if (ctx->graph_stream) (void)hipStreamDestroy(ctx->graph_stream);
    if (ctx->ev_in) (void)hipEventDestroy(ctx->ev_in);
    if (ctx->ev_out) (void)hipEventDestroy(ctx->ev_out);
    if (ctx->team_abort) (void)hipHostFree(ctx->team_abort);
    if (ctx->staging) (void)hipHostFree(ctx->staging);
    delete ctx;
}

pa_status pa_ctx_set_graphs(pa_ctx *ctx, int enable) {
    if (!ctx) return fail(PA_ERR_INVALID, "null context");
    if (enable && !ctx->graph_stream) {
        if (hipSetDevice(ctx->device) != hipSuccess ||
            hipStreamCreateWithFlags(&ctx->graph_stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&ctx->ev_out, hipEventDisableTiming) != hipSuccess)
            return fail(PA_ERR_DEVICE, "cannot create the graph stream");
    }
    ctx->graphs = enable ? 1 : 0;
    return PA_OK;
}

pa_status pa_ctx_set_batch_mode(pa_ctx *ctx, int mode) {
    if (!ctx || (mode != PA_BATCH_TEAM && mode != PA_BATCH_SEGMENTED)) return fail(PA_ERR_INVALID, "bad batch mode");
    ctx->batch_mode = mode;
    return PA_OK;
}

pa_status pa_ctx_batch_info(pa_ctx *ctx, uint32_t *team_runs, uint32_t *team_launches) {
    if (!ctx) return fail(PA_ERR_INVALID, "null context");
    if (team_runs) *team_runs = ctx->team_runs;
    if (team_launches) *team_launches = ctx->team_launches;
    return PA_OK;
}

pa_status pa_ctx_abort_batch(pa_ctx *ctx) {
    if (!ctx) return fail(PA_ERR_INVALID, "null context");
    ctx->abort_requested = 1;
    __atomic_store_n(ctx->team_abort, 1u, __ATOMIC_SEQ_CST);
    return PA_OK;
}

pa_status pa_ctx_set_profiling(pa_ctx *ctx, int enable) {
    if (!ctx) return fail(PA_ERR_INVALID, "null context");
    ctx->profiling = enable ? 1 : 0;
    return PA_OK;
}

pa_status pa_ctx_set_lanes(pa_ctx *ctx, uint32_t L, uint32_t lanes) {
    if (!ctx) return fail(PA_ERR_INVALID, "null context");
    uint32_t cand[2];
    const uint32_t n = pa::lane_candidates(L, cand);
    if (n == 0) return fail(PA_ERR_INVALID, "no lane choices for this lattice side");
    if (lanes != 0 && lanes != cand[0] && !(n > 1 && lanes == cand[1]))
        return fail(PA_ERR_INVALID, "lanes is not a candidate for this lattice side");
    ctx->lanes[pa::lane_choice_index(L)] = lanes;
    return PA_OK;
}

pa_status pa_ctx_get_lanes(pa_ctx *ctx, uint32_t L, uint32_t *lanes, uint32_t *candidates,
                           uint32_t *n_candidates) {
    if (!ctx) return fail(PA_ERR_INVALID, "null context");
    uint32_t cand[2] = {0, 0};
    const uint32_t n = pa::lane_candidates(L, cand);
    uint32_t G = 0, wpb;
    if (!pa::tiled_path(L)) pa::sweep_shape(L, ctx_lanes(ctx, L), &G, &wpb);
    if (lanes) *lanes = G;
    if (candidates) { candidates[0] = cand[0]; candidates[1] = cand[1]; }
    if (n_candidates) *n_candidates = n;
    return PA_OK;
}

pa_status pa_autotune(pa_ctx *ctx, uint32_t L, uint32_t q, void *d_ws, uint64_t ws_bytes, void *stream,
                      uint32_t *best_lanes, double *best_attempts_per_ns) {
    if (!ctx) return fail(PA_ERR_INVALID, "null context");
    uint32_t cand[2];
    const uint32_t n = pa::lane_candidates(L, cand);
    if (n == 0) return fail(PA_ERR_INVALID, "no lane choices for this lattice side");
    // A population of about 64 MB of spins (4096 .. 65536 replicas) fills the GPU.
    const uint64_t N = (uint64_t)L * L;
    uint64_t R = std::max<uint64_t>(1024, std::min<uint64_t>(65536, (1ull << 26) / N));
    const double beta[3] = {0.0, 0.5, 1.0};
    pa_run_desc d{};
    d.L = L; d.q = q; d.K = 3; d.beta = beta; d.theta = 4; d.seed = 12345;
    d.resample = PA_RESAMPLE_MULTINOMIAL; d.init = PA_INIT_RANDOM; d.outputs = 0;
    pa_plan_info info;
    for (;;) {
        d.R = R;
        pa_status st = pa_plan(&d, &info);
        if (st) return st;
        if (info.workspace_bytes <= ws_bytes || R <= 64) break;
        R /= 2;
    }
    if (info.workspace_bytes > ws_bytes) return fail(PA_ERR_NOMEM, "workspace too small for tuning");
    const int saved_prof = ctx->profiling;
    const uint32_t saved = ctx_lanes(ctx, L);
    double best = -1.0;
    uint32_t best_g = cand[0];
    for (uint32_t c = 0; c < n; ++c) {
        pa_ctx_set_lanes(ctx, L, cand[c]);
        pa_result res{};
        double kms[PA_KERNEL_KINDS];
        uint64_t kn[PA_KERNEL_KINDS];
        res.kernel_ms = kms;
        res.kernel_launches = kn;
        ctx->profiling = 0;
        pa_status st = pa_run(ctx, &d, d_ws, ws_bytes, stream, nullptr);   // warm-up
        ctx->profiling = 1;
        if (!st) st = pa_run(ctx, &d, d_ws, ws_bytes, stream, &res);
        ctx->profiling = saved_prof;
        if (st) { pa_ctx_set_lanes(ctx, L, saved); return st; }
        const double rate = 4.0 * (double)N * (double)(2 * R) / (kms[PA_KERNEL_SWEEP] * 1e6);
        if (rate > best) { best = rate; best_g = cand[c]; }
    }
    pa_ctx_set_lanes(ctx, L, best_g);
    if (best_lanes) *best_lanes = best_g;
    if (best_attempts_per_ns) *best_attempts_per_ns = best;
    return PA_OK;
}

// The sweep shapes a tuned entry may take for lattice side L: every lane
// count with a kernel for L, and for each the waves per workgroup that keep a
// workgroup within 1024 threads (256 for the byte kernel) and the LDS.
static std::vector<std::pair<uint32_t, uint32_t>> tune_candidates(uint32_t L, int device) {
    std::vector<std::pair<uint32_t, uint32_t>> out;
    if (pa::tiled_path(L)) return out;
    const uint32_t N = L * L;
    const size_t lds_max = pa::max_lds_per_block(device);
    auto add = [&](uint32_t G, uint32_t w) {
        if (pa::sweep_lds_bytes(N, G, w, 0u) <= lds_max) out.push_back({G, w});
    };
    if (L & 3u) {                                        // byte kernel: one replica per wave
        for (uint32_t w = 1; w <= 4; w *= 2) add(64, w);
        return out;
    }
    uint32_t cand[2];
    uint32_t nc = pa::lane_candidates(L, cand);
    if (nc == 0) {                                       // the generic kernel's one lane count
        uint32_t G, w;
        pa::sweep_shape(L, 0, &G, &w);
        cand[0] = G;
        nc = 1;
    }
    for (uint32_t c = 0; c < nc; ++c) {
        const uint32_t G = cand[c];
        if (G > 64 && G % 64 == 0) {
            add(G, G / 64);                              // one replica per workgroup
        } else if (64 % G != 0) {
            uint32_t w0 = 1;                             // replicas spanning waves
            while ((64 * w0) % G != 0) ++w0;
            for (uint32_t w = w0; 64 * w <= 1024; w += w0) add(G, w);
        } else {
            for (uint32_t w = 1; w <= 16; w *= 2) add(G, w);
        }
    }
    return out;
}

static pa_status tune_check(pa_ctx *ctx, const pa_tune_entry *e) {
    for (const auto &c : tune_candidates(e->L, ctx->device))
        if (c.first == e->lanes && c.second == e->waves_per_block) return PA_OK;
    return fail(PA_ERR_INVALID, "not a sweep shape of this lattice side");
}

pa_status pa_tune_set(pa_ctx *ctx, const pa_tune_entry *e) {
    if (!ctx || !e || e->r_class > 3) return fail(PA_ERR_INVALID, "bad tuned entry");
    pa_status st = tune_check(ctx, e);
    if (st) return st;
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    ctx->tune[tune_key(e->L, e->q_large, e->r_class)] = *e;
    ++ctx->tune_gen;
    return PA_OK;
}

pa_status pa_tune_get(pa_ctx *ctx, uint32_t L, uint32_t q, uint64_t R, pa_tune_entry *e) {
    if (!ctx || !e) return fail(PA_ERR_INVALID, "null argument");
    pa_tune_entry t{};
    t.L = L;
    t.q_large = q > 128 ? 1u : 0u;
    t.r_class = r_class_of(R);
    if (pa::tiled_path(L)) return fail(PA_ERR_INVALID, "the tiled path has no sweep shape");
    pa::sweep_shape(L, ctx_lanes(ctx, L), &t.lanes, &t.waves_per_block);
    if (ctx_lanes(ctx, L) == 0) {
        std::lock_guard<std::mutex> lk(ctx->tune_mu);
        auto it = ctx->tune.find(tune_key(t.L, t.q_large, t.r_class));
        if (it != ctx->tune.end()) t = it->second;
    }
    *e = t;
    return PA_OK;
}

pa_status pa_tune(pa_ctx *ctx, uint32_t L, uint32_t q, uint64_t R, void *d_ws, uint64_t ws_bytes, void *stream,
                  pa_tune_entry *best, pa_tune_entry *timed, uint32_t timed_cap, uint32_t *n_timed) {
    if (!ctx || !best) return fail(PA_ERR_INVALID, "null argument");
    const auto cands = tune_candidates(L, ctx->device);
    if (cands.empty()) return fail(PA_ERR_INVALID, "no sweep shapes for this lattice side");
    const double beta[3] = {0.0, 0.5, 1.0};
    pa_run_desc d{};
    d.L = L; d.q = q; d.R = R; d.K = 3; d.beta = beta; d.theta = 10; d.seed = 12345;
    d.resample = PA_RESAMPLE_MULTINOMIAL; d.init = PA_INIT_RANDOM; d.outputs = 0;
    pa_plan_info info;
    pa_status st = pa_plan(&d, &info);
    if (st) return st;
    if (info.workspace_bytes > ws_bytes) return fail(PA_ERR_NOMEM, "workspace too small for tuning");
    const int saved_prof = ctx->profiling;
    pa_tune_entry b{};
    b.L = L;
    b.q_large = q > 128 ? 1u : 0u;
    b.r_class = r_class_of(R);
    b.attempts_per_ns = -1.0;
    uint32_t nt = 0;
    for (const auto &c : cands) {
        ctx->tune_try_G = c.first;
        ctx->tune_try_wpb = c.second;
        pa_result res{};
        double kms[PA_KERNEL_KINDS];
        uint64_t kn[PA_KERNEL_KINDS];
        res.kernel_ms = kms;
        res.kernel_launches = kn;
        ctx->profiling = 0;
        st = pa_run(ctx, &d, d_ws, ws_bytes, stream, nullptr);   // warm-up
        ctx->profiling = 1;
        if (!st) st = pa_run(ctx, &d, d_ws, ws_bytes, stream, &res);
        ctx->profiling = saved_prof;
        if (st) break;
        const double rate = (double)d.theta * (double)L * L * (double)(2 * R) / (kms[PA_KERNEL_SWEEP] * 1e6);
        if (timed && nt < timed_cap) {
            timed[nt] = b;
            timed[nt].lanes = c.first;
            timed[nt].waves_per_block = c.second;
            timed[nt].attempts_per_ns = rate;
        }
        ++nt;
        if (rate > b.attempts_per_ns) {
            b.lanes = c.first;
            b.waves_per_block = c.second;
            b.attempts_per_ns = rate;
        }
    }
    ctx->tune_try_G = ctx->tune_try_wpb = 0;
    if (st) return st;
    if (n_timed) *n_timed = nt;
    {
        std::lock_guard<std::mutex> lk(ctx->tune_mu);
        ctx->tune[tune_key(b.L, b.q_large, b.r_class)] = b;
        ++ctx->tune_gen;
    }
    *best = b;
    return PA_OK;
}

// The device's architecture name (gfx950, without target features).
static std::string ctx_arch(pa_ctx *ctx) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, ctx->device) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

pa_status pa_tune_save(pa_ctx *ctx, const char *path) {
    if (!ctx || !path) return fail(PA_ERR_INVALID, "null argument");
    const std::string arch = ctx_arch(ctx);
    std::vector<pa_tune_entry> all;
    {
        std::lock_guard<std::mutex> lk(ctx->tune_mu);
        for (const auto &kv : ctx->tune) all.push_back(kv.second);
    }
    FILE *f = std::fopen(path, "w");
    if (!f) return fail(PA_ERR_INVALID, std::string("cannot write ") + path);
    for (const auto &e : all)
        std::fprintf(f,
                     "{\"arch\": \"%s\", \"L\": %u, \"q_large\": %u, \"r_class\": %u, \"lanes\": %u, "
                     "\"waves_per_block\": %u, \"attempts_per_ns\": %.3f}\n",
                     arch.c_str(), e.L, e.q_large, e.r_class, e.lanes, e.waves_per_block, e.attempts_per_ns);
    const bool ok = std::fclose(f) == 0;
    return ok ? PA_OK : fail(PA_ERR_INVALID, std::string("cannot write ") + path);
}

// The value after "key": on a line of the cache file.
static bool json_field(const std::string &line, const char *key, std::string *out) {
    const std::string k = std::string("\"") + key + "\"";
    size_t i = line.find(k);
    if (i == std::string::npos) return false;
    i = line.find(':', i + k.size());
    if (i == std::string::npos) return false;
    ++i;
    while (i < line.size() && line[i] == ' ') ++i;
    size_t j = i;
    if (j < line.size() && line[j] == '"') {
        const size_t e = line.find('"', j + 1);
        if (e == std::string::npos) return false;
        *out = line.substr(j + 1, e - j - 1);
        return true;
    }
    while (j < line.size() && line[j] != ',' && line[j] != '}') ++j;
    *out = line.substr(i, j - i);
    return !out->empty();
}

pa_status pa_tune_load(pa_ctx *ctx, const char *path, uint32_t *n_loaded) {
    if (!ctx || !path) return fail(PA_ERR_INVALID, "null argument");
    FILE *f = std::fopen(path, "r");
    if (!f) return fail(PA_ERR_INVALID, std::string("cannot read ") + path);
    const std::string arch = ctx_arch(ctx);
    std::vector<pa_tune_entry> got;
    char buf[512];
    pa_status st = PA_OK;
    unsigned line_no = 0;
    while (!st && std::fgets(buf, sizeof buf, f)) {
        ++line_no;
        const std::string line(buf);
        if (line.find_first_not_of(" \t\r\n") == std::string::npos) continue;
        std::string a, v[6];
        const char *keys[6] = {"L", "q_large", "r_class", "lanes", "waves_per_block", "attempts_per_ns"};
        bool ok = json_field(line, "arch", &a);
        for (int k = 0; k < 6 && ok; ++k) ok = json_field(line, keys[k], &v[k]);
        if (!ok) {
            st = fail(PA_ERR_INVALID, std::string(path) + ": malformed line " + std::to_string(line_no));
            break;
        }
        if (a != arch) continue;                      // tuned on another architecture
        pa_tune_entry e{};
        e.L = (uint32_t)std::strtoul(v[0].c_str(), nullptr, 10);
        e.q_large = (uint32_t)std::strtoul(v[1].c_str(), nullptr, 10);
        e.r_class = (uint32_t)std::strtoul(v[2].c_str(), nullptr, 10);
        e.lanes = (uint32_t)std::strtoul(v[3].c_str(), nullptr, 10);
        e.waves_per_block = (uint32_t)std::strtoul(v[4].c_str(), nullptr, 10);
        e.attempts_per_ns = std::strtod(v[5].c_str(), nullptr);
        if (e.r_class > 3 || (st = tune_check(ctx, &e)))
            st = fail(PA_ERR_INVALID, std::string(path) + ": line " + std::to_string(line_no) +
                                          " is not a sweep shape of its lattice side");
        else
            got.push_back(e);
    }
    std::fclose(f);
    if (st) return st;
    {
        std::lock_guard<std::mutex> lk(ctx->tune_mu);
        for (const auto &e : got) ctx->tune[tune_key(e.L, e.q_large, e.r_class)] = e;
        ++ctx->tune_gen;
    }
    if (n_loaded) *n_loaded = (uint32_t)got.size();
    return PA_OK;
}

pa_status pa_issue_probe(pa_ctx *ctx, uint32_t kind, void *d_out, uint64_t out_bytes, void *stream,
                         double *lane_instr_per_s) {
    if (!ctx || !d_out || !lane_instr_per_s || kind >= PA_PROBE_KINDS)
        return fail(PA_ERR_INVALID, "bad probe arguments");
    int cus = 0;
    if (hipSetDevice(ctx->device) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus <= 0)
        return fail(PA_ERR_DEVICE, "cannot query the compute units");
    const uint32_t blocks = 8u * (uint32_t)cus;   // 32 waves per compute unit
    if (out_bytes < (uint64_t)blocks * pa::probe_threads() * 4u)
        return fail(PA_ERR_NOMEM, "probe output buffer too small");
    const uint32_t iters = kind == PA_PROBE_MIX ? 8192u : 32768u;
    double ms = 0;
    return hip_check(nullptr, pa::issue_probe(kind, blocks, iters, static_cast<uint32_t *>(d_out),
                                              static_cast<hipStream_t>(stream), lane_instr_per_s, &ms),
                     "issue probe");
}

}  // extern "C"

namespace {

// The buffers a run starts from, as fills: zeroed histograms, copy counts and
// ln Q sums, the tiled sweeps' accumulators, and -beta_0 F_0 (r->mbF0) as two
// 32-bit words.
struct Fill { uint32_t *dst; uint64_t words; uint32_t value; };

std::vector<Fill> start_fills(pa_run_state *r) {
    const Plan &p = r->plan;
    std::vector<Fill> f;
    const size_t hist_words = (size_t)p.nbins * (p.hist_all ? p.desc.K : 1);
    const size_t mhist_words = p.mag ? (size_t)(p.N + 1) * (p.hist_all ? p.desc.K : 1) : 0;
    f.push_back({r->at<uint32_t>(p.off_hist), hist_words, 0u});
    if (mhist_words) f.push_back({r->at<uint32_t>(p.off_mhist), mhist_words, 0u});
    f.push_back({r->at<uint32_t>(p.off_r), 2 * counts_stride(p.R_cap), 0u});
    f.push_back({r->at<uint32_t>(p.off_lnQ), 2 * (size_t)p.desc.K, 0u});
    if (p.tiled) f.push_back({r->at<uint32_t>(p.off_bonds), p.R_cap, 0u});
    if (p.tiled && p.mag) f.push_back({r->at<uint32_t>(p.off_cnt), p.R_cap * p.desc.q, 0u});
    if (p.tiled && p.digest) f.push_back({r->at<uint32_t>(p.off_Hacc), 2 * p.R_cap, 0u});
    uint64_t bits;
    std::memcpy(&bits, &r->mbF0, 8);
    f.push_back({r->at<uint32_t>(p.off_mbF), 1, (uint32_t)bits});
    f.push_back({r->at<uint32_t>(p.off_mbF) + 1, 1, (uint32_t)(bits >> 32)});
    return f;
}

// pa_run_begin: a run's host state in workspace d_ws and, unless `deferred`,
// its start on the stream: the weight tables, the fills of start_fills and (if
// `initial`; not for a run that loads a population right after, from a
// checkpoint) the initial population with its statistics.  With `wait`,
// returns once the uploads and launches are done; otherwise the caller
// synchronises the stream before freeing the run (its plan holds the uploaded
// host tables).  A deferred run leaves the start to the caller (a batch does
// it for all its runs in a few launches).
pa_status begin_run(pa_ctx *ctx, const pa_run_desc *desc, void *d_ws, uint64_t ws_bytes, void *stream,
                    bool initial, pa_run_state **out, bool wait = true, bool deferred = false,
                    Plan *plan = nullptr) {
    if (!ctx || !out) return fail(PA_ERR_INVALID, "null context or output");
    pa_run_state *r = new (std::nothrow) pa_run_state;
    if (!r) return fail(PA_ERR_NOMEM, "out of host memory");
    pa_status st = PA_OK;
    if (plan) {
        r->plan = std::move(*plan);          // built already (a batch's layout, which gives it up)
        r->plan.desc.beta = r->plan.beta.data();
    } else
        st = build_plan(desc, r->plan);
    if (st) { delete r; return st; }
    const Plan &p = r->plan;
    if (!d_ws || ws_bytes < p.total || ((uintptr_t)d_ws & 255u)) {
        delete r;
        return fail(PA_ERR_NOMEM, "workspace missing, unaligned or smaller than pa_plan's workspace_bytes");
    }
    r->ctx = ctx;
    r->ws = static_cast<uint8_t *>(d_ws);
    r->stream = static_cast<hipStream_t>(stream);
    r->step = 0;
    r->cur = 0;
    r->R_cur = p.desc.R;
    r->R_prev = p.desc.R;
    r->first_step = 0;
    r->R_first = p.desc.R;
    r->r_dirty[0] = r->r_dirty[1] = 0;
    r->broken = false;
    r->G = 0;
    r->wpb = 0;
    if (!p.tiled) {
        // a lane count set on the context, else the tuned shape of this
        // class, else the default
        pa::sweep_shape(p.desc.L, ctx_lanes(ctx, p.desc.L), &r->G, &r->wpb);
        uint32_t tG = 0, tw = 0;
        if (ctx->tune_try_G) {
            tG = ctx->tune_try_G;
            tw = ctx->tune_try_wpb;
        } else if (ctx_lanes(ctx, p.desc.L) == 0) {
            std::lock_guard<std::mutex> lk(ctx->tune_mu);
            auto it = ctx->tune.find(tune_key(p.desc.L, p.desc.q > 128, r_class_of(p.R_cap)));
            if (it != ctx->tune.end()) {
                tG = it->second.lanes;
                tw = it->second.waves_per_block;
            }
        }
        if (tG && pa::sweep_lds_bytes(p.N, tG, tw, p.mag ? p.desc.q : 0u) <= pa::max_lds_per_block(ctx->device)) {
            r->G = tG;
            r->wpb = tw;
        }
    }
    if (!p.tiled && pa::sweep_lds_bytes(p.N, r->G, r->wpb, p.mag ? p.desc.q : 0u) >
                        pa::max_lds_per_block(ctx->device)) {
        delete r;
        return fail(PA_ERR_UNSUPPORTED, "lattice does not fit the LDS of one workgroup on this device");
    }
    if ((st = hip_check(r, hipSetDevice(ctx->device), "hipSetDevice"))) { delete r; return st; }
    // ln Z at beta_0: N ln q (Z = q^N at beta = 0, Sec. 6) or, for ground
    // states, ln q + 2N beta_0 (eq. (7)-(8), E_0 = -2N).
    r->mbF0 = (p.desc.init == PA_INIT_GROUND)
                  ? std::log((double)p.desc.q) + 2.0 * (double)p.N * p.beta[0]
                  : (double)p.N * std::log((double)p.desc.q);
    if (deferred) {
        *out = r;
        return PA_OK;
    }

    // Tables and initial state.
    hipStream_t s = r->stream;
    // on an error after the first upload: let the stream drain before the
    // run (and the host tables the copies read) goes
    auto drop = [&](pa_status e) {
        (void)hipStreamSynchronize(s);
        delete r;
        return e;
    };
    if (!p.W.empty() &&
        (st = hip_check(r, hipMemcpyAsync(r->ws + p.off_W, p.W.data(), 8 * p.W.size(), hipMemcpyHostToDevice, s),
                        "upload W")))
        return drop(st);
    for (const Fill &f : start_fills(r))
        if ((st = hip_check(r, pa::launch_fill_u32(f.dst, f.words, f.value, s), "fill"))) return drop(st);
    const uint32_t mode = p.desc.init == PA_INIT_GROUND ? pa::SWEEP_INIT_GROUND : pa::SWEEP_INIT_RANDOM;
    pa::SweepArgs a = sweep_args(r, 0, mode, nullptr, nullptr, r->at<uint8_t>(p.off_pop[0]), 0);
    const pa::TiledArgs ta = tiled_args(r, 0, nullptr, nullptr, r->at<uint8_t>(p.off_pop[0]));
    auto init = [&]() -> hipError_t {
        if (!p.tiled) return pa::launch_sweep(a, s);
        const hipError_t e = pa::launch_tiled_init(ta, s);
        return e != hipSuccess ? e : pa::launch_tiled_measure(ta, s);
    };
    if (initial && ((st = timed_launch(r, PA_KERNEL_INIT, "init kernel", init)) ||
                    (st = launch_post_for(r, 0)))) {
        release_events(r, nullptr, nullptr);
        return drop(st);
    }
    // The uploads read host memory owned by the run.
    if (wait && (st = hip_check(r, hipStreamSynchronize(s), "sync"))) { delete r; return st; }
    *out = r;
    return PA_OK;
}

}  // namespace

static pa_status finish_run(pa_run_state *r, pa_result *out, const uint8_t *blk_in);

extern "C" {

pa_status pa_run_begin(pa_ctx *ctx, const pa_run_desc *desc, void *d_ws, uint64_t ws_bytes,
                       void *stream, pa_run_state **out) {
    return begin_run(ctx, desc, d_ws, ws_bytes, stream, true, out);
}

pa_status pa_run_advance(pa_run_state *r, uint32_t n_steps) {
    if (!r) return fail(PA_ERR_INVALID, "null run");
    if (r->broken) return fail(PA_ERR_DEVICE, "run is unusable after a device error");
    if ((uint64_t)r->step + n_steps > (uint64_t)r->plan.desc.K - 1)
        return fail(PA_ERR_INVALID, "advancing past the last temperature");
    for (uint32_t n = 0; n < n_steps; ++n) {
        pa_status st = do_step(r);
        if (st) return st;
    }
    return PA_OK;
}

pa_status pa_run_sync(pa_run_state *r) {
    if (!r) return fail(PA_ERR_INVALID, "null run");
    return hip_check(r, hipStreamSynchronize(r->stream), "sync");
}

pa_status pa_run_read(pa_run_state *r, uint32_t *step, uint64_t *R_cur, uint64_t *R_prev,
                      uint8_t *spins, int32_t *E, uint32_t *anc, uint32_t *counts) {
    if (!r) return fail(PA_ERR_INVALID, "null run");
    pa_status st = hip_check(r, hipStreamSynchronize(r->stream), "sync");
    if (st) return st;
    const Plan &p = r->plan;
    if (step) *step = r->step;
    if (R_cur) *R_cur = r->R_cur;
    if (R_prev) *R_prev = r->R_prev;
    struct { void *dst; size_t off, bytes; } cp[4] = {
        {spins, p.off_pop[r->cur], (size_t)r->R_cur * p.N},
        {E, p.off_E, 4 * (size_t)r->R_cur},
        {anc, (size_t)((uint8_t *)anc_of(r, r->step) - r->ws), 4 * (size_t)r->R_cur},
        {counts, (size_t)((uint8_t *)counts_of(r, r->step) - r->ws), 4 * (size_t)r->R_prev},
    };
    for (auto &c : cp) {
        if (!c.dst) continue;
        if ((st = hip_check(r, hipMemcpy(c.dst, r->ws + c.off, c.bytes, hipMemcpyDeviceToHost), "read")))
            return st;
    }
    return PA_OK;
}

pa_status pa_run_read_free_energy(pa_run_state *r, uint32_t *step, double *minus_beta_F) {
    if (!r || !minus_beta_F) return fail(PA_ERR_INVALID, "null run or output");
    pa_status st = hip_check(r, hipStreamSynchronize(r->stream), "sync");
    if (st) return st;
    if (step) *step = r->step;
    return hip_check(r, hipMemcpy(minus_beta_F, r->at<double>(r->plan.off_mbF) + r->step, 8,
                                  hipMemcpyDeviceToHost), "read");
}

pa_status pa_run_load(pa_run_state *r, uint32_t step, uint64_t R_cur, const uint8_t *spins,
                      double minus_beta_F) {
    if (!r || !spins) return fail(PA_ERR_INVALID, "null run or spins");
    const Plan &p = r->plan;
    if (step >= p.desc.K || R_cur < 1 || R_cur > p.R_cap)
        return fail(PA_ERR_INVALID, "step or population size out of range");
    pa_status st;
    hipStream_t s = r->stream;
    r->step = step;
    r->R_cur = R_cur;
    r->R_prev = R_cur;
    r->first_step = step;
    r->R_first = R_cur;
    // the draws of step + 1 count into a zero buffer
    const uint32_t next = (step + 1) & 1u;
    if (r->r_dirty[next]) {
        if ((st = hip_check(r, pa::launch_fill_u32(counts_buf(r, next), r->r_dirty[next], 0u, s), "fill")))
            return st;
        r->r_dirty[next] = 0;
    }
    // Upload into the idle buffer, then recompute E with a sweep of zero
    // rounds into the other buffer and the statistics with the post kernel.
    const int idle = 1 - r->cur;
    if ((st = hip_check(r, hipMemcpyAsync(r->ws + p.off_pop[idle], spins, (size_t)R_cur * p.N,
                                          hipMemcpyHostToDevice, s), "upload spins")))
        return st;
    r->mbF0 = minus_beta_F;
    if ((st = hip_check(r, hipMemcpyAsync(r->at<double>(p.off_mbF) + step, &r->mbF0, 8,
                                          hipMemcpyHostToDevice, s), "upload")))
        return st;
    if (p.tiled) {
        const pa::TiledArgs ta = tiled_args(r, step, r->at<uint8_t>(p.off_pop[idle]), nullptr,
                                            r->at<uint8_t>(p.off_pop[r->cur]));
        if ((st = hip_check(r, launch_tiled_sweeps(ta, 0, r->at<uint8_t>(p.off_pop_x), s), "load kernels")))
            return st;
    } else {
        pa::SweepArgs a = sweep_args(r, step, pa::SWEEP_UPDATE, r->at<uint8_t>(p.off_pop[idle]), nullptr,
                                     r->at<uint8_t>(p.off_pop[r->cur]), 0);
        if ((st = hip_check(r, pa::launch_sweep(a, s), "load kernel"))) return st;
    }
    if ((st = launch_post_for(r, step))) return st;
    return hip_check(r, hipStreamSynchronize(s), "sync");
}

pa_status pa_run_read_slots(pa_run_state *r, int previous, const uint32_t *slots, uint32_t n,
                            uint8_t *spins_out) {
    if (!r || (n && (!slots || !spins_out))) return fail(PA_ERR_INVALID, "null argument");
    pa_status st = hip_check(r, hipStreamSynchronize(r->stream), "sync");
    if (st) return st;
    const Plan &p = r->plan;
    const uint64_t R = previous ? r->R_prev : r->R_cur;
    const size_t off = p.off_pop[previous ? 1 - r->cur : r->cur];
    for (uint32_t j = 0; j < n; ++j) {
        if (slots[j] >= R) return fail(PA_ERR_INVALID, "slot out of range");
        if ((st = hip_check(r, hipMemcpy(spins_out + (size_t)j * p.N, r->ws + off + (size_t)slots[j] * p.N,
                                         p.N, hipMemcpyDeviceToHost), "read")))
            return st;
    }
    return PA_OK;
}

pa_status pa_run_finish(pa_run_state *r, pa_result *out) {
    return finish_run(r, out, nullptr);
}

}  // extern "C"

// pa_run_finish, with the run's per-step block already read (blk_in, by a
// batch that reads every run's block in one round) or not (null).
static pa_status finish_run(pa_run_state *r, pa_result *out, const uint8_t *blk_in) {
    if (!r) return fail(PA_ERR_INVALID, "null run");
    pa_status st = blk_in ? PA_OK : hip_check(r, hipStreamSynchronize(r->stream), "sync");
    const Plan &p = r->plan;
    const uint32_t K = p.desc.K;
    if (!st && out) {
        // the per-step block in one copy
        std::vector<uint8_t> own;
        const uint8_t *blk = blk_in;
        if (!blk) {
            own.resize(p.steps_bytes);
            st = hip_check(r, hipMemcpy(own.data(), r->ws + p.off_steps, p.steps_bytes, hipMemcpyDeviceToHost),
                           "read");
            blk = own.data();
        }
        auto field = [&](size_t off) { return blk + (off - p.off_steps); };
        std::vector<uint64_t> count(K);
        if (!st) std::memcpy(count.data(), field(p.off_count), 8 * (size_t)K);
        for (uint32_t i = r->first_step; !st && i <= r->step; ++i)
            if (count[i] != (i == r->first_step ? r->R_first : p.R_sched[i]))
                st = fail(PA_ERR_DEVICE, "population histogram does not add up to R_i");
        if (!st && out->R_i) {
            for (uint32_t i = 0; i < K; ++i) out->R_i[i] = p.R_sched[i];
            out->R_i[r->first_step] = r->R_first;
        }
        if (!st) {
            if (out->lnQ) std::memcpy(out->lnQ, field(p.off_lnQ), 8 * (size_t)K);
            if (out->minus_beta_F) std::memcpy(out->minus_beta_F, field(p.off_mbF), 8 * (size_t)K);
            if (p.digest && out->digest) std::memcpy(out->digest, field(p.off_digest), 8 * (size_t)K);
        }
        struct { void *dst; size_t off, bytes; } cp[] = {
            {p.hist_all ? out->hist : nullptr, p.off_hist, 4 * (size_t)K * p.nbins},
            {(p.mag && p.hist_all) ? out->mhist : nullptr, p.off_mhist, 4 * (size_t)K * (p.N + 1)},
        };
        for (auto &c : cp) {
            if (st || !c.dst) continue;
            st = hip_check(r, hipMemcpy(c.dst, r->ws + c.off, c.bytes, hipMemcpyDeviceToHost), "read");
        }
        // Population averages (eq. (4)-(5)) and widths (Sec. 4) on the host,
        // from the exact integer sums and the integer parts of the widths.
        std::vector<int64_t> esum(K), mtsum(p.mag ? K : 0);
        std::vector<uint64_t> fwe(p.widths ? 8 * (size_t)K : 0), fwm(p.widths && p.mag ? 8 * (size_t)K : 0);
        if (!st) {
            std::memcpy(esum.data(), field(p.off_Esum), 8 * (size_t)K);
            if (p.mag) std::memcpy(mtsum.data(), field(p.off_Mtsum), 8 * (size_t)K);
            if (p.widths) std::memcpy(fwe.data(), field(p.off_fwe), 8 * fwe.size());
            if (p.widths && p.mag) std::memcpy(fwm.data(), field(p.off_fwm), 8 * fwm.size());
        }
        if (!st) {
            const double N = (double)p.N, q = (double)p.desc.q;
            for (uint32_t i = 0; i < K; ++i) {
                const uint64_t Ri = i == r->first_step ? r->R_first : p.R_sched[i];
                const bool measured = i >= r->first_step && i <= r->step;
                const double R = (double)Ri;
                if (out->E_sum) out->E_sum[i] = measured ? esum[i] : 0;
                if (out->E_mean) out->E_mean[i] = measured ? (double)esum[i] / R : 0.0;
                if (p.mag && out->Mt_sum) out->Mt_sum[i] = measured ? mtsum[i] : 0;
                if (p.mag && out->M_mean)
                    out->M_mean[i] = measured ? (q * (double)mtsum[i] - N * R) / ((q - 1.0) * R) : 0.0;
                if (p.widths && out->width_e)
                    out->width_e[i] = measured ? fwhm_levels(&fwe[8 * (size_t)i], p.bin_e) / N : 0.0;
                if (p.widths && p.mag && out->width_m)
                    out->width_m[i] = measured ? (fwhm_levels(&fwm[8 * (size_t)i], p.bin_m) * q) / ((q - 1.0) * N)
                                               : 0.0;
            }
        }
        if (!st && out->lnQ) out->lnQ[0] = 0.0;
        if (!st && (out->kernel_ms || out->kernel_launches))
            release_events(r, out->kernel_ms, out->kernel_launches);
        // the final population, only for a run that reached its last temperature
        // (the buffers are sized for R_{K-1})
        if (!st && (p.desc.outputs & PA_OUT_FINAL) && r->step + 1 == K) {
            if (out->final_spins)
                st = hip_check(r, hipMemcpy(out->final_spins, r->ws + p.off_pop[r->cur], (size_t)r->R_cur * p.N, hipMemcpyDeviceToHost), "read");
            if (!st && out->final_E)
                st = hip_check(r, hipMemcpy(out->final_E, r->ws + p.off_E, 4 * (size_t)r->R_cur, hipMemcpyDeviceToHost), "read");
            if (!st && out->last_anc) {
                if (r->step == 0 || p.desc.resample == PA_RESAMPLE_NONE) {
                    for (uint64_t k = 0; k < r->R_cur; ++k) out->last_anc[k] = (uint32_t)k;
                } else {
                    st = hip_check(r, hipMemcpy(out->last_anc, anc_of(r, r->step), 4 * (size_t)r->R_cur, hipMemcpyDeviceToHost), "read");
                }
            }
        }
    }
    release_events(r, nullptr, nullptr);
    delete r;
    return st;
}

// ---------------------------------------------------------------------------
// Checkpoints: a run's population at a step, with -beta F of that step and the
// run description, in the binary format documented in pa.h.
// ---------------------------------------------------------------------------

namespace {

constexpr char kCkptMagic[8] = {'P', 'A', 'C', 'K', 'P', 'T', '0', '1'};
constexpr uint32_t kCkptHeader = 128;

struct Checkpoint {
    pa_run_desc desc{};
    std::vector<double> beta;
    uint32_t step = 0;
    uint64_t R_cur = 0;
    double mbF = 0;
    int64_t E_sum = 0;
};

template <typename T> void put(uint8_t *h, size_t off, T v) { std::memcpy(h + off, &v, sizeof v); }
template <typename T> T get(const uint8_t *h, size_t off) { T v; std::memcpy(&v, h + off, sizeof v); return v; }

pa_status write_checkpoint(pa_run_state *r, const char *path) {
    if (!r || !path) return fail(PA_ERR_INVALID, "null run or path");
    if (r->broken) return fail(PA_ERR_DEVICE, "run is unusable after a device error");
    pa_status st = hip_check(r, hipStreamSynchronize(r->stream), "sync");
    if (st) return st;
    const Plan &p = r->plan;
    std::vector<uint8_t> spins((size_t)r->R_cur * p.N);
    double mbF = 0;
    int64_t esum = 0;
    if ((st = hip_check(r, hipMemcpy(spins.data(), r->ws + p.off_pop[r->cur], spins.size(), hipMemcpyDeviceToHost),
                        "read")) ||
        (st = hip_check(r, hipMemcpy(&mbF, r->at<double>(p.off_mbF) + r->step, 8, hipMemcpyDeviceToHost), "read")) ||
        (st = hip_check(r, hipMemcpy(&esum, r->at<int64_t>(p.off_Esum) + r->step, 8, hipMemcpyDeviceToHost), "read")))
        return st;
    uint8_t h[kCkptHeader] = {};
    std::memcpy(h, kCkptMagic, 8);
    const pa_run_desc &d = p.desc;
    put<uint32_t>(h, 8, kCkptHeader);
    put<uint32_t>(h, 12, d.L);
    put<uint32_t>(h, 16, d.q);
    put<uint32_t>(h, 20, d.K);
    put<uint64_t>(h, 24, d.R);
    put<uint32_t>(h, 32, d.theta);
    put<int32_t>(h, 36, d.resample);
    put<uint64_t>(h, 40, d.seed);
    put<int32_t>(h, 48, d.init);
    put<uint32_t>(h, 52, d.outputs);
    put<uint32_t>(h, 56, d.bin_e);
    put<uint32_t>(h, 60, d.bin_m);
    put<uint32_t>(h, 64, r->step);
    put<uint64_t>(h, 72, r->R_cur);
    put<double>(h, 80, mbF);
    put<int64_t>(h, 88, esum);
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(PA_ERR_INVALID, std::string("cannot open ") + path + " for writing");
    bool ok = std::fwrite(h, 1, kCkptHeader, f) == kCkptHeader &&
              std::fwrite(p.beta.data(), 8, p.beta.size(), f) == p.beta.size() &&
              std::fwrite(spins.data(), 1, spins.size(), f) == spins.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? PA_OK : fail(PA_ERR_INVALID, std::string("cannot write ") + path);
}

// Reads and checks the header and beta of a checkpoint; with `spins`, also
// the population.
pa_status read_checkpoint(const char *path, Checkpoint &c, std::vector<uint8_t> *spins) {
    if (!path) return fail(PA_ERR_INVALID, "null path");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(PA_ERR_INVALID, std::string("cannot open ") + path);
    std::unique_ptr<FILE, int (*)(FILE *)> guard(f, std::fclose);
    uint8_t h[kCkptHeader];
    if (std::fread(h, 1, kCkptHeader, f) != kCkptHeader || std::memcmp(h, kCkptMagic, 8) != 0 ||
        get<uint32_t>(h, 8) != kCkptHeader)
        return fail(PA_ERR_INVALID, "not a checkpoint file (magic or header size)");
    pa_run_desc &d = c.desc;
    d = pa_run_desc{};
    d.L = get<uint32_t>(h, 12);
    d.q = get<uint32_t>(h, 16);
    d.K = get<uint32_t>(h, 20);
    d.R = get<uint64_t>(h, 24);
    d.theta = get<uint32_t>(h, 32);
    d.resample = get<int32_t>(h, 36);
    d.seed = get<uint64_t>(h, 40);
    d.init = get<int32_t>(h, 48);
    d.outputs = get<uint32_t>(h, 52);
    d.bin_e = get<uint32_t>(h, 56);
    d.bin_m = get<uint32_t>(h, 60);
    c.step = get<uint32_t>(h, 64);
    c.R_cur = get<uint64_t>(h, 72);
    c.mbF = get<double>(h, 80);
    c.E_sum = get<int64_t>(h, 88);
    if (d.K == 0 || d.K > (1u << 27) || c.step >= d.K || d.L < 2 || d.L > 65536 || c.R_cur == 0 ||
        c.R_cur > (1ull << 31))
        return fail(PA_ERR_INVALID, "checkpoint header out of range");
    c.beta.resize(d.K);
    if (std::fread(c.beta.data(), 8, d.K, f) != d.K) return fail(PA_ERR_INVALID, "checkpoint truncated (beta)");
    d.beta = c.beta.data();
    const uint64_t bytes = c.R_cur * (uint64_t)d.L * d.L;
    const long at = std::ftell(f);
    if (at < 0 || std::fseek(f, 0, SEEK_END) != 0) return fail(PA_ERR_INVALID, "cannot size the checkpoint file");
    const long end = std::ftell(f);
    if (end < 0 || (uint64_t)end != (uint64_t)at + bytes)
        return fail(PA_ERR_INVALID, "checkpoint file size does not match its header (truncated or extended)");
    if (spins) {
        spins->resize(bytes);
        if (std::fseek(f, at, SEEK_SET) != 0 || std::fread(spins->data(), 1, bytes, f) != bytes)
            return fail(PA_ERR_INVALID, "checkpoint truncated (spins)");
    }
    return PA_OK;
}

// A new run in the workspace continued from checkpoint c (population spins):
// begun without an initial population, the population loaded at c.step, and
// the energy sum the device recomputes checked against the stored one.
pa_status resume_run(pa_ctx *ctx, const Checkpoint &c, const std::vector<uint8_t> &spins, void *d_ws,
                     uint64_t ws_bytes, void *stream, pa_run_state **out) {
    pa_run_state *r = nullptr;
    pa_status st = begin_run(ctx, &c.desc, d_ws, ws_bytes, stream, false, &r);
    if (st) return st;
    if ((st = pa_run_load(r, c.step, c.R_cur, spins.data(), c.mbF))) {
        const std::string msg = g_last_error;
        pa_run_finish(r, nullptr);
        return fail(st, msg);
    }
    int64_t esum = 0;
    st = hip_check(r, hipMemcpy(&esum, r->at<int64_t>(r->plan.off_Esum) + c.step, 8, hipMemcpyDeviceToHost), "read");
    if (!st && esum != c.E_sum) st = fail(PA_ERR_INVALID, "checkpoint energies do not match its population");
    if (st) {
        const std::string msg = g_last_error;
        pa_run_finish(r, nullptr);
        return fail(st, msg);
    }
    *out = r;
    return PA_OK;
}

}  // namespace

extern "C" {

pa_status pa_checkpoint(pa_run_state *run, const char *path) { return write_checkpoint(run, path); }

pa_status pa_checkpoint_info(const char *path, pa_run_desc *desc, double *beta, uint32_t beta_cap, uint32_t *step,
                             uint64_t *R_cur) {
    Checkpoint c;
    pa_status st = read_checkpoint(path, c, nullptr);
    if (st) return st;
    if (desc) {
        *desc = c.desc;
        desc->beta = nullptr;
    }
    if (step) *step = c.step;
    if (R_cur) *R_cur = c.R_cur;
    if (beta) {
        if (beta_cap < c.desc.K) return fail(PA_ERR_NOMEM, "beta buffer shorter than K");
        std::memcpy(beta, c.beta.data(), 8 * (size_t)c.desc.K);
        if (desc) desc->beta = beta;
    }
    return PA_OK;
}

pa_status pa_resume(pa_ctx *ctx, const char *path, void *d_ws, uint64_t ws_bytes, void *stream,
                    pa_run_state **out) {
    if (!ctx || !out) return fail(PA_ERR_INVALID, "null context or output");
    Checkpoint c;
    std::vector<uint8_t> spins;
    pa_status st = read_checkpoint(path, c, &spins);
    if (st) return st;
    return resume_run(ctx, c, spins, d_ws, ws_bytes, stream, out);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Several runs per launch (batched runs and the serving loop): every run keeps
// its own workspace region and plan; one "global step" advances each listed
// run by one temperature step with segmented launches (one sampling launch
// over all runs' draws, one count-scan launch over all runs' blocks, one sweep
// launch per kernel class, one post launch over all runs' statistics and
// weight workgroups).  The descriptor records are built
// on the host and uploaded before the launches.
// ---------------------------------------------------------------------------
namespace {

size_t step_desc_bytes(size_t n) {
    return align256(n * sizeof(pa::SampleArgs)) + align256((n + 1) * 4) +
           align256(n * sizeof(pa::SlotmapArgs)) + align256((n + 1) * 4) + align256(n * sizeof(pa::SweepArgs)) +
           align256(2 * (n + 1) * 4 + 4 * n) + align256(n * sizeof(pa::PostArgs)) + align256((n + 1) * 4);
}

struct StepLaunch {
    size_t sample_off, sample_start_off, slot_off, slot_start_off, sweep_off, sweep_start_off, post_off,
        post_start_off;
    uint32_t n_res, sample_blocks, slot_blocks, n_post, post_blocks;
    struct Group { uint32_t cls, first, count, blocks, threads; size_t lds; };
    std::vector<Group> groups;
    struct Tiled { pa::TiledArgs a; uint32_t theta; uint8_t *x; bool init; };
    std::vector<Tiled> tiled;   // large lattices, launched one by one
};

// Advance the host state of every run in `active` (each with step < K-1) by one
// step and write the step's descriptor records at blob + cursor.  With `init`,
// the records of step 0 instead (runs begun deferred): the initial population
// of each run and its statistics.
StepLaunch build_step(const std::vector<pa_run_state *> &active, std::vector<uint8_t> &blob,
                      size_t &cursor, bool init = false) {
    const size_t n = active.size();
    StepLaunch L{};
    std::vector<pa::SampleArgs> sa;
    std::vector<uint32_t> sstart, mstart;
    std::vector<pa::SlotmapArgs> sm;
    std::vector<pa::PostArgs> po;
    struct SW { uint32_t cls, blocks, threads; size_t lds; pa::SweepArgs a; };
    std::vector<SW> sw;
    uint32_t sblocks = 0, mblocks = 0;
    auto add_sweep = [&](pa_run_state *r, const pa::SweepArgs &a) {
        const Plan &p = r->plan;
        const uint64_t per_block = pa::replicas_per_block(r->G, r->wpb);
        SW e;
        e.cls = pa::sweep_class(p.desc.L, p.desc.q, a.T[3] == 0, r->G);
        e.blocks = (uint32_t)((r->R_cur + per_block - 1) / per_block);
        e.threads = 64u * r->wpb;
        e.lds = pa::sweep_lds_bytes(p.N, r->G, r->wpb, p.mag ? p.desc.q : 0u);
        e.a = a;
        sw.push_back(e);
    };
    for (pa_run_state *r : active) {
        const Plan &p = r->plan;
        if (init) {
            uint8_t *pop0 = r->at<uint8_t>(p.off_pop[0]);
            if (p.tiled)
                L.tiled.push_back({tiled_args(r, 0, nullptr, nullptr, pop0), 0u, nullptr, true});
            else
                add_sweep(r, sweep_args(r, 0, p.desc.init == PA_INIT_GROUND ? pa::SWEEP_INIT_GROUND
                                                                            : pa::SWEEP_INIT_RANDOM,
                                        nullptr, nullptr, pop0, 0));
            po.push_back(post_args(r, 0));
            continue;
        }
        const uint32_t g = r->step + 1;
        const uint64_t R_prev = r->R_cur, R_new = p.R_sched[g];
        const int prev_buf = r->cur, new_buf = 1 - r->cur;
        const uint32_t *anc = nullptr;
        if (p.small) {
            anc = anc_of(r, g);                  // written by the post launch of step g-1
        } else if (p.desc.resample != PA_RESAMPLE_NONE) {
            pa::SampleArgs a;
            pa::SlotmapArgs m;
            resample_args(r, g, R_prev, R_new, a, m);
            sstart.push_back(sblocks);
            sblocks += (uint32_t)((R_new + 255) / 256);
            sa.push_back(a);
            mstart.push_back(mblocks);
            mblocks += pa::countfill_blocks(m);
            sm.push_back(m);
            anc = m.anc;
        }
        r->R_prev = R_prev;
        r->R_cur = R_new;
        if (p.tiled) {
            L.tiled.push_back({tiled_args(r, g, r->at<uint8_t>(p.off_pop[prev_buf]), anc,
                                          r->at<uint8_t>(p.off_pop[new_buf])),
                               p.desc.theta, r->at<uint8_t>(p.off_pop_x), false});
            r->cur = new_buf;
            r->step = g;
            po.push_back(post_args(r, g));
            continue;
        }
        add_sweep(r, sweep_args(r, g, pa::SWEEP_UPDATE, r->at<uint8_t>(p.off_pop[prev_buf]), anc,
                                r->at<uint8_t>(p.off_pop[new_buf]), p.desc.theta));
        r->cur = new_buf;
        r->step = g;
        po.push_back(post_args(r, g));
    }
    auto take = [&](size_t bytes) { size_t at = cursor; cursor += align256(bytes); return at; };
    if (blob.size() < cursor + step_desc_bytes(n)) blob.resize(cursor + step_desc_bytes(n), 0);
    L.n_res = (uint32_t)sa.size();
    L.sample_blocks = sblocks;
    L.slot_blocks = mblocks;
    sstart.push_back(sblocks);
    mstart.push_back(mblocks);
    L.sample_off = take(n * sizeof(pa::SampleArgs));
    L.sample_start_off = take((n + 1) * 4);
    L.slot_off = take(n * sizeof(pa::SlotmapArgs));
    L.slot_start_off = take((n + 1) * 4);
    std::memcpy(blob.data() + L.sample_off, sa.data(), sa.size() * sizeof(pa::SampleArgs));
    std::memcpy(blob.data() + L.sample_start_off, sstart.data(), sstart.size() * 4);
    std::memcpy(blob.data() + L.slot_off, sm.data(), sm.size() * sizeof(pa::SlotmapArgs));
    std::memcpy(blob.data() + L.slot_start_off, mstart.data(), mstart.size() * 4);
    // sweep groups: runs of one kernel class contiguous in the table
    // (a class's runs may differ in waves per workgroup when tuned shapes
    // apply: a launch takes one block size)
    std::stable_sort(sw.begin(), sw.end(), [](const SW &x, const SW &y) {
        return x.cls != y.cls ? x.cls < y.cls : x.threads < y.threads;
    });
    L.sweep_off = take(n * sizeof(pa::SweepArgs));
    L.sweep_start_off = take(2 * (n + 1) * 4 + 4 * n);
    std::vector<uint32_t> starts;
    for (size_t k = 0; k < sw.size();) {
        StepLaunch::Group G{sw[k].cls, (uint32_t)starts.size(), 0, 0, sw[k].threads, sw[k].lds};
        while (k < sw.size() && sw[k].cls == G.cls && sw[k].threads == G.threads) {
            G.lds = std::max(G.lds, sw[k].lds);   // runs of one class may differ in q and outputs
            starts.push_back(G.blocks);
            G.blocks += sw[k].blocks;
            ++G.count;
            ++k;
        }
        starts.push_back(G.blocks);
        L.groups.push_back(G);
    }
    for (size_t k = 0; k < sw.size(); ++k)
        std::memcpy(blob.data() + L.sweep_off + k * sizeof(pa::SweepArgs), &sw[k].a, sizeof(pa::SweepArgs));
    std::memcpy(blob.data() + L.sweep_start_off, starts.data(), starts.size() * 4);
    L.n_post = (uint32_t)po.size();
    std::vector<uint32_t> pstart;
    uint32_t pblocks = 0;
    for (const auto &a : po) {
        pstart.push_back(pblocks);
        pblocks += pa::post_blocks(a);
    }
    pstart.push_back(pblocks);
    L.post_blocks = pblocks;
    L.post_off = take(n * sizeof(pa::PostArgs));
    L.post_start_off = take((n + 1) * 4);
    std::memcpy(blob.data() + L.post_off, po.data(), po.size() * sizeof(pa::PostArgs));
    std::memcpy(blob.data() + L.post_start_off, pstart.data(), pstart.size() * 4);
    return L;
}

pa_status launch_step(const StepLaunch &L, const uint8_t *dtab, hipStream_t s) {
    pa_status st;
    if (L.n_res &&
        (st = hip_check(nullptr, pa::launch_resample_batch(
                                     reinterpret_cast<const pa::SampleArgs *>(dtab + L.sample_off),
                                     reinterpret_cast<const uint32_t *>(dtab + L.sample_start_off), L.n_res,
                                     L.sample_blocks, reinterpret_cast<const pa::SlotmapArgs *>(dtab + L.slot_off),
                                     reinterpret_cast<const uint32_t *>(dtab + L.slot_start_off), L.slot_blocks, s),
                        "batched resample")))
        return st;
    uint32_t run_index = 0;
    for (const auto &G : L.groups) {
        if ((st = hip_check(nullptr, pa::launch_sweep_batch(
                                         G.cls, reinterpret_cast<const pa::SweepArgs *>(dtab + L.sweep_off) + run_index,
                                         reinterpret_cast<const uint32_t *>(dtab + L.sweep_start_off) + G.first,
                                         G.count, G.blocks, G.threads, G.lds, s),
                            "batched sweep")))
            return st;
        run_index += G.count;
    }
    for (const auto &t : L.tiled) {
        if (t.init) {
            if ((st = hip_check(nullptr, pa::launch_tiled_init(t.a, s), "tiled init")) ||
                (st = hip_check(nullptr, pa::launch_tiled_measure(t.a, s), "tiled init")))
                return st;
        } else if ((st = hip_check(nullptr, launch_tiled_sweeps(t.a, t.theta, t.x, s), "tiled sweeps"))) {
            return st;
        }
    }
    return hip_check(nullptr, pa::launch_post_batch(reinterpret_cast<const pa::PostArgs *>(dtab + L.post_off),
                                                    reinterpret_cast<const uint32_t *>(dtab + L.post_start_off),
                                                    L.n_post, L.post_blocks, s),
                     "batched post");
}

struct BatchLayout {
    std::vector<Plan> plans;
    std::vector<size_t> run_off;
    size_t desc_off = 0, desc_bytes = 0, out_off = 0, team_off = 0, team_bytes = 0, total = 0;
    uint32_t max_K = 0;
};

// A k_prep_batch launch whose records sit in the descriptor table.
struct PrepLaunch {
    size_t rec_off = 0, start_off = 0;
    uint32_t n = 0, blocks = 0;
};

// Write the records (none of zero words) and their workgroup starts at blob + cursor.
PrepLaunch pack_prep(const std::vector<pa::PrepRec> &recs, std::vector<uint8_t> &blob, size_t &cursor) {
    PrepLaunch P;
    std::vector<uint32_t> start;
    for (const auto &e : recs) {
        start.push_back(P.blocks);
        P.blocks += (uint32_t)((e.words + pa::PREP_CHUNK - 1) / pa::PREP_CHUNK);
    }
    start.push_back(P.blocks);
    P.n = (uint32_t)recs.size();
    P.rec_off = cursor;
    P.start_off = P.rec_off + align256(recs.size() * sizeof(pa::PrepRec));
    cursor = P.start_off + align256(start.size() * 4);
    if (blob.size() < cursor) blob.resize(cursor, 0);
    std::memcpy(blob.data() + P.rec_off, recs.data(), recs.size() * sizeof(pa::PrepRec));
    std::memcpy(blob.data() + P.start_off, start.data(), start.size() * 4);
    return P;
}

pa_status launch_prep(const PrepLaunch &P, const uint8_t *dtab, hipStream_t s) {
    return hip_check(nullptr,
                     pa::launch_prep_batch(reinterpret_cast<const pa::PrepRec *>(dtab + P.rec_off),
                                           reinterpret_cast<const uint32_t *>(dtab + P.start_off), P.n, P.blocks, s),
                     "batched fills");
}

// Descriptor bytes of a batch's start and end: the weight tables, up to ten
// fill and copy records per run (start_fills and the table), the records of
// step 0, and one gather record per run.
size_t prep_bytes(const std::vector<Plan> &plans) {
    const size_t n = plans.size();
    size_t w = 0;
    for (const Plan &p : plans) w += align256(8 * p.W.size());
    return w + align256(10 * n * sizeof(pa::PrepRec)) + align256((10 * n + 1) * 4) + step_desc_bytes(n) +
           align256(n * sizeof(pa::PrepRec)) + align256((n + 1) * 4);
}

// Device bytes of the team launches' records for runs with these plans: one
// TeamStep per step after the first, one TeamRun, a 256-byte barrier counter
// and the per-step claim counters per run.
size_t team_record_bytes(const std::vector<Plan> &plans) {
    size_t steps = 0, counters = 0;
    for (const Plan &p : plans) {
        steps += p.desc.K;
        counters += 256 + align256(4 * (size_t)p.desc.K);
    }
    return align256(steps * sizeof(pa::TeamStep)) + align256(plans.size() * sizeof(pa::TeamRun)) + counters;
}

pa_status batch_layout(const pa_run_desc *descs, uint32_t n, BatchLayout &b) {
    if (!descs || n == 0) return fail(PA_ERR_INVALID, "empty batch");
    b.plans.resize(n);
    b.run_off.resize(n);
    size_t o = 0;
    // runs with one (L, K, beta schedule) share their tables
    std::unordered_map<std::string, uint32_t> first_of;
    for (uint32_t r = 0; r < n; ++r) {
        const Plan *like = nullptr;
        if (descs[r].beta && descs[r].K) {
            std::string key((const char *)descs[r].beta, 8 * (size_t)descs[r].K);
            key.append((const char *)&descs[r].L, sizeof descs[r].L);
            auto it = first_of.find(key);
            if (it != first_of.end()) like = &b.plans[it->second];
            else first_of.emplace(std::move(key), r);
        }
        pa_status st = build_plan(&descs[r], b.plans[r], like);
        if (st) return fail(st, "run " + std::to_string(r) + ": " + g_last_error);
        b.run_off[r] = o;
        o += align256(b.plans[r].total);
        b.max_K = std::max(b.max_K, descs[r].K);
    }
    b.desc_off = o;
    b.desc_bytes = prep_bytes(b.plans) + step_desc_bytes(n) * (b.max_K > 1 ? b.max_K - 1 : 1);
    // every run's per-step block, gathered for one read-back
    b.out_off = align256(o + b.desc_bytes);
    size_t out_bytes = 0;
    for (const Plan &p : b.plans) out_bytes += align256(p.steps_bytes);
    b.team_off = align256(b.out_off + out_bytes);
    b.team_bytes = team_record_bytes(b.plans);
    b.total = b.team_off + b.team_bytes;
    return PA_OK;
}

// ---------------------------------------------------------------------------
// Team launches (k_team): runs of one sweep class with small populations go
// through all their remaining steps in one cooperative launch; each run owns a
// team of workgroups (one for the statistics, the rest for resampling and
// sweeps) that meet at one barrier per step.
// ---------------------------------------------------------------------------
constexpr uint64_t kTeamRMax = 8192;              // largest population in a team launch
constexpr uint64_t kTeamTimeoutTicks = 1000000000ull;   // 10 s of the 100 MHz counter

// The class of a run's sweeps if every step of it can go to a team launch,
// else 0 (tiled, byte-kernel or 64-bit-threshold steps, a population above
// kTeamRMax, or no team kernel for the class).
uint32_t team_class(const pa_run_state *r) {
    const Plan &p = r->plan;
    if (p.tiled || p.R_cap > kTeamRMax || r->step + 1 >= p.desc.K) return 0;
    for (uint32_t i = r->step + 1; i < p.desc.K; ++i)
        if (p.T[(size_t)i * 4 + 3] == 0) return 0;
    const uint32_t cls = pa::sweep_class(p.desc.L, p.desc.q, false, r->G);
    return pa::team_kernel(cls) ? cls : 0u;
}

// The buffers of step i in a team launch ending at step K-1: the last step
// writes the run's main energy, M~ and digest-term buffers.
struct TeamBufs { int32_t *E; uint32_t *Mt; uint64_t *H; };
TeamBufs team_bufs(pa_run_state *r, uint32_t i) {
    const Plan &p = r->plan;
    const bool alt = ((p.desc.K - 1 - i) & 1u) != 0;
    return {r->at<int32_t>(alt ? p.off_E2 : p.off_E),
            p.mag ? r->at<uint32_t>(alt ? p.off_Mt2 : p.off_Mt) : nullptr,
            p.digest ? r->at<uint64_t>(alt ? p.off_H2 : p.off_H) : nullptr};
}

// Statistics of step i (R_cur replicas) reading the team buffers of step i.
pa::PostArgs team_post(pa_run_state *r, uint32_t i) {
    pa::PostArgs a = post_args(r, i);
    const TeamBufs b = team_bufs(r, i);
    a.E = b.E;
    a.Mt = b.Mt;
    a.H = b.H;
    a.do_weights = 0;
    a.small = 0;
    return a;
}

// The records of run r's remaining steps; advances its host state to the
// last step.
void team_records(pa_run_state *r, std::vector<pa::TeamStep> &recs, pa::TeamRun &tr) {
    const Plan &p = r->plan;
    const uint32_t K = p.desc.K, i0 = r->step;
    tr.rec0 = (uint32_t)recs.size();
    tr.n_steps = K - 1 - i0;
    for (uint32_t i = i0 + 1; i < K; ++i) {
        pa::TeamStep t{};
        const uint64_t R_prev = r->R_cur, R_new = p.R_sched[i];
        t.stats = i - 1 > i0 ? 1u : 0u;
        if (t.stats) t.p = team_post(r, i - 1);         // r->R_cur is R_{i-1} here
        const TeamBufs prev = team_bufs(r, i - 1), cur = team_bufs(r, i);
        t.r = small_resample_args(r, i);            // from the energies of step i-1
        t.r.E_prev = prev.E;
        r->R_prev = R_prev;
        r->R_cur = R_new;
        t.w = sweep_args(r, i, pa::SWEEP_UPDATE, r->at<uint8_t>(p.off_pop[r->cur]), nullptr,
                         r->at<uint8_t>(p.off_pop[1 - r->cur]), p.desc.theta);
        t.w.E_out = cur.E;
        t.w.Mt_out = cur.Mt;
        t.w.H_out = cur.H;
        recs.push_back(t);
        r->cur = 1 - r->cur;
        r->step = i;
    }
    tr.last = team_post(r, K - 1);
    tr.last_stats = 1;
}

pa_status run_team_launch(pa_ctx *ctx, uint32_t cls, std::vector<pa_run_state *> &group, uint8_t *dtab,
                          size_t dtab_bytes, hipStream_t s) {
    const uint32_t n = (uint32_t)group.size();
    pa_status st;
    // shape of the class: sweep groups of 64 * waves_per_block threads
    const pa_run_state *r0 = group[0];
    const uint32_t BS = 64u * r0->wpb, SUB = pa::team_threads() / BS;
    const uint32_t rpb = (uint32_t)pa::replicas_per_block(r0->G, r0->wpb);
    size_t sub_lds = 0;
    uint64_t r_max = 1;
    uint32_t n_max = 1;
    std::vector<uint32_t> useful(n), sweepers(n);
    std::vector<double> cost(n);
    for (uint32_t k = 0; k < n; ++k) {
        const pa_run_state *r = group[k];
        const Plan &p = r->plan;
        sub_lds = std::max(sub_lds, (pa::sweep_lds_bytes(p.N, r->G, r->wpb, p.mag ? p.desc.q : 0u) + 15) & ~size_t(15));
        r_max = std::max(r_max, p.R_cap);
        n_max = std::max(n_max, p.N);
        // sweep workgroups beyond one block each would only repeat the
        // resampling
        const uint64_t blocks = (p.R_cap + rpb - 1) / rpb;
        useful[k] = (uint32_t)blocks;
        // site updates (and the gather) of the run's remaining steps
        cost[k] = (double)p.N * (p.desc.theta + 1.0) * (double)p.R_cap * (double)(p.desc.K - 1 - r->step);
    }
    // LDS: the ancestors of every new slot, then a work area for the
    // resampling's counts and weights, the sweep groups, or the statistics'
    // energy and M~ histograms, in turn
    const size_t anc_bytes = (4 * r_max + 15) & ~uint64_t(15);
    const size_t work = (std::max({anc_bytes + 8 * r_max, SUB * sub_lds, 4 * (2 * (size_t)n_max + 1)}) + 15) & ~size_t(15);
    const size_t lds = anc_bytes + work;
    if (lds > pa::max_lds_per_block(ctx->device)) return fail(PA_ERR_UNSUPPORTED, "team launch exceeds the LDS");
    const uint32_t cap = pa::team_capacity(cls, lds, ctx->device);
    if (cap < 2 * n) return fail(PA_ERR_UNSUPPORTED, "team launch does not fit the device");
    // teams: one statistics workgroup each, and the resident workgroups left
    // shared out as sweep workgroups in proportion to the runs' work, none
    // beyond its useful number and at least one
    uint32_t avail = cap - n;
    std::vector<bool> fixed(n, false);
    for (bool again = true; again;) {
        again = false;
        double total = 0;
        for (uint32_t k = 0; k < n; ++k)
            if (!fixed[k]) total += cost[k];
        for (uint32_t k = 0; k < n && !again; ++k)
            if (!fixed[k] && (total <= 0 || (double)avail * cost[k] / total >= useful[k])) {
                sweepers[k] = useful[k];
                avail -= std::min(avail, useful[k]);
                fixed[k] = again = true;
            }
        if (!again)
            for (uint32_t k = 0; k < n; ++k)
                if (!fixed[k]) sweepers[k] = std::max<uint32_t>(1, (uint32_t)((double)avail * cost[k] / total));
    }
    uint32_t team_total = n;
    for (uint32_t k = 0; k < n; ++k) team_total += sweepers[k];
    while (team_total > cap) {   // the floor of one each may overshoot: trim the largest
        uint32_t big = 0;
        for (uint32_t k = 1; k < n; ++k)
            if (sweepers[k] > sweepers[big]) big = k;
        if (sweepers[big] <= 1) return fail(PA_ERR_UNSUPPORTED, "team launch does not fit the device");
        --sweepers[big];
        --team_total;
    }
    // records
    std::vector<pa::TeamStep> recs;
    std::vector<pa::TeamRun> truns(n);
    uint32_t team0 = 0;
    for (uint32_t k = 0; k < n; ++k) {
        pa_run_state *r = group[k];
        const Plan &p = r->plan;
        // the population of the first step must sit in the buffers that step
        // reads (step i0 alternates with the last step's parity)
        const TeamBufs b0 = team_bufs(r, r->step);
        if (b0.E != r->at<int32_t>(p.off_E)) {
            if ((st = hip_check(r, hipMemcpyAsync(b0.E, r->at<int32_t>(p.off_E), 4 * r->R_cur, hipMemcpyDeviceToDevice, s),
                                "copy energies")) ||
                (b0.Mt && (st = hip_check(r, hipMemcpyAsync(b0.Mt, r->at<uint32_t>(p.off_Mt), 4 * r->R_cur,
                                                             hipMemcpyDeviceToDevice, s), "copy M~"))) ||
                (b0.H && (st = hip_check(r, hipMemcpyAsync(b0.H, r->at<uint64_t>(p.off_H), 8 * r->R_cur,
                                                            hipMemcpyDeviceToDevice, s), "copy digest terms"))))
                return st;
        }
        truns[k].team0 = team0;
        truns[k].team = 1 + sweepers[k];
        team0 += truns[k].team;
        team_records(r, recs, truns[k]);
    }
    const size_t steps_bytes = align256(recs.size() * sizeof(pa::TeamStep));
    const size_t runs_bytes = align256(n * sizeof(pa::TeamRun));
    // per run: a 256-byte barrier counter, then its claim counters
    size_t counter_bytes = 0;
    for (uint32_t k = 0; k < n; ++k) {
        truns[k].barrier = reinterpret_cast<uint32_t *>(dtab + steps_bytes + runs_bytes + counter_bytes);
        truns[k].claims = truns[k].barrier + 64;
        counter_bytes += 256 + align256(4 * (size_t)truns[k].n_steps);
    }
    if (steps_bytes + runs_bytes + counter_bytes > dtab_bytes)
        return fail(PA_ERR_DEVICE, "team record table overflow");
    uint32_t *barriers = reinterpret_cast<uint32_t *>(dtab + steps_bytes + runs_bytes);
    uint8_t *stage = ctx_staging(ctx, steps_bytes + runs_bytes, s);
    if (!stage) return fail(PA_ERR_DEVICE, "cannot allocate pinned staging memory");
    std::memcpy(stage, recs.data(), recs.size() * sizeof(pa::TeamStep));
    std::memcpy(stage + steps_bytes, truns.data(), n * sizeof(pa::TeamRun));
    if ((st = hip_check(nullptr, hipMemcpyAsync(dtab, stage, steps_bytes + runs_bytes, hipMemcpyHostToDevice, s),
                        "upload team records")) ||
        (st = hip_check(nullptr, pa::launch_fill_u32(barriers, counter_bytes / 4, 0u, s), "clear counters")))
        return st;
    pa::TeamCtl ctl{};
    ctl.abort = ctx->team_abort;
    ctl.timeout_ticks = kTeamTimeoutTicks;
    ctl.r_max = (uint32_t)r_max;
    ctl.anc_bytes = (uint32_t)anc_bytes;
    ctl.work_bytes = (uint32_t)work;
    ctl.sub_lds = (uint32_t)sub_lds;
    // the uploads above read host memory; the abort word is reset once the
    // stream has drained
    if ((st = hip_check(nullptr, hipStreamSynchronize(s), "sync"))) return st;
    if (ctx->abort_requested) return fail(PA_ERR_CANCELLED, "batch aborted");
    __atomic_store_n(ctx->team_abort, 0u, __ATOMIC_SEQ_CST);
    if (ctx->abort_requested) __atomic_store_n(ctx->team_abort, 1u, __ATOMIC_SEQ_CST);
    if ((st = hip_check(nullptr, pa::launch_team(cls, reinterpret_cast<const pa::TeamRun *>(dtab + steps_bytes), n,
                                                 reinterpret_cast<const pa::TeamStep *>(dtab), ctl, team0, lds, s),
                        "team launch")) ||
        (st = hip_check(nullptr, hipStreamSynchronize(s), "sync")))
        return st;
    const uint32_t ab = __atomic_load_n(ctx->team_abort, __ATOMIC_SEQ_CST);
    if (ab == 1u) return fail(PA_ERR_CANCELLED, "batch aborted");
    if (ab) return fail(PA_ERR_DEVICE, "a team barrier wait timed out");
    return PA_OK;
}

}  // namespace

extern "C" pa_status pa_plan_batch(const pa_run_desc *descs, uint32_t n, uint64_t *workspace_bytes) {
    if (!workspace_bytes) return fail(PA_ERR_INVALID, "null output");
    BatchLayout b;
    pa_status st = batch_layout(descs, n, b);
    if (st) return st;
    *workspace_bytes = b.total;
    return PA_OK;
}

extern "C" pa_status pa_run_batch(pa_ctx *ctx, const pa_run_desc *descs, uint32_t n, void *d_ws,
                                  uint64_t ws_bytes, void *stream, pa_result *outs) {
    if (!ctx) return fail(PA_ERR_INVALID, "null context");
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    BatchLayout b;
    pa_status st = batch_layout(descs, n, b);
    if (st) return st;
    if (!d_ws || ws_bytes < b.total || ((uintptr_t)d_ws & 255u))
        return fail(PA_ERR_NOMEM, "workspace missing, unaligned or smaller than pa_plan_batch's size");
    uint8_t *ws = static_cast<uint8_t *>(d_ws);
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<pa_run_state *> runs(n, nullptr);
    auto cleanup = [&](pa_status code) {
        const std::string msg = g_last_error;
        for (auto *r : runs)
            if (r) pa_run_finish(r, nullptr);
        return fail(code, msg);
    };
    ctx->abort_requested = 0;
    ctx->team_runs = ctx->team_launches = 0;
    for (uint32_t r = 0; r < n; ++r) {
        st = begin_run(ctx, &descs[r], ws + b.run_off[r], align256(b.plans[r].total), stream, true, &runs[r],
                       /*wait=*/false, /*deferred=*/true, &b.plans[r]);
        if (st) return cleanup(fail(st, "run " + std::to_string(r) + ": " + g_last_error));
    }
    uint8_t *dtab = ws + b.desc_off;
    std::vector<uint8_t> blob;
    size_t cursor = 0;
    auto take = [&](size_t bytes) {
        const size_t at = cursor;
        cursor += align256(bytes);
        if (blob.size() < cursor) blob.resize(cursor, 0);
        return at;
    };
    // The runs' start in three launches: the weight tables (copied from the
    // descriptor table) and the fills of every run, then the initial
    // populations and their statistics (step 0) of all runs.
    std::vector<pa::PrepRec> recs;
    for (pa_run_state *r : runs) {
        const Plan &p = r->plan;
        if (!p.W.empty()) {
            const size_t at = take(8 * p.W.size());
            std::memcpy(blob.data() + at, p.W.data(), 8 * p.W.size());
            recs.push_back({r->at<uint32_t>(p.off_W), reinterpret_cast<const uint32_t *>(dtab + at),
                            2 * (uint64_t)p.W.size(), 0u, 0u});
        }
        for (const Fill &f : start_fills(r))
            if (f.words) recs.push_back({f.dst, nullptr, f.words, f.value, 0u});
    }
    const PrepLaunch prep = pack_prep(recs, blob, cursor);
    const StepLaunch init = build_step(runs, blob, cursor, /*init=*/true);
    // and its end: every run's per-step block gathered in one launch, read
    // back in one copy
    std::vector<size_t> blk_off(n);
    size_t blk_total = 0;
    recs.clear();
    for (uint32_t r = 0; r < n; ++r) {
        blk_off[r] = blk_total;
        const Plan &p = runs[r]->plan;
        recs.push_back({reinterpret_cast<uint32_t *>(ws + b.out_off + blk_total),
                        reinterpret_cast<const uint32_t *>(runs[r]->ws + p.off_steps), p.steps_bytes / 4, 0u, 0u});
        blk_total += align256(p.steps_bytes);
    }
    const PrepLaunch gather = pack_prep(recs, blob, cursor);

    // The descriptor table goes up from pinned memory that mirrors it (each
    // part at its own offset, so that the host can write the next part while
    // the last one is still being copied); the results come back behind it.
    const size_t stage_bytes = align256(b.desc_bytes) + blk_total;
    auto upload = [&](size_t from) -> pa_status {
        if (cursor > b.desc_bytes) return fail(PA_ERR_DEVICE, "descriptor table overflow");
        if (cursor == from) return PA_OK;
        uint8_t *stage = ctx_staging(ctx, stage_bytes, s);
        if (!stage) return fail(PA_ERR_DEVICE, "cannot allocate pinned staging memory");
        std::memcpy(stage + from, blob.data() + from, cursor - from);
        return hip_check(nullptr, hipMemcpyAsync(dtab + from, stage + from, cursor - from, hipMemcpyHostToDevice, s),
                         "upload descriptors");
    };
    if ((st = upload(0)) || (st = launch_prep(prep, dtab, s)) || (st = launch_step(init, dtab, s)))
        return cleanup(st);
    const bool team = ctx->batch_mode == PA_BATCH_TEAM && !ctx->graphs;
    std::vector<bool> finished(n, false);
    if (team) {
        // Team launches, one per sweep class, for the runs that qualify; they
        // finish those runs.  (The wait: the staging memory is reused.)
        if ((st = hip_check(nullptr, hipStreamSynchronize(s), "sync"))) return cleanup(st);
        std::map<std::pair<uint32_t, uint32_t>, std::vector<uint32_t>> by_class;   // (class, waves per group)
        for (uint32_t r = 0; r < n; ++r)
            if (const uint32_t cls = team_class(runs[r])) by_class[{cls, runs[r]->wpb}].push_back(r);
        for (auto &kv : by_class) {
            // a group too large for one launch is split in halves (launched one
            // after the other); a single run that does not fit goes segmented
            std::vector<std::vector<uint32_t>> pending{kv.second};
            while (!pending.empty()) {
                const std::vector<uint32_t> idx = pending.back();
                pending.pop_back();
                std::vector<pa_run_state *> group;
                for (uint32_t r : idx) group.push_back(runs[r]);
                st = run_team_launch(ctx, kv.first.first, group, ws + b.team_off, b.team_bytes, s);
                if (st == PA_ERR_UNSUPPORTED) {
                    if (idx.size() > 1) {
                        const size_t h = idx.size() / 2;
                        pending.emplace_back(idx.begin() + h, idx.end());
                        pending.emplace_back(idx.begin(), idx.begin() + h);
                    }
                    continue;
                }
                if (st) return cleanup(st);
                for (uint32_t r : idx) finished[r] = true;
                ctx->team_runs += (uint32_t)idx.size();
                ++ctx->team_launches;
            }
        }
    }
    // The global steps of the runs left: records built on the host from the
    // plans, global step g advancing every run with g < K.
    std::vector<StepLaunch> steps;
    uint32_t next_g = 1;
    auto build_steps = [&](uint32_t count) {
        for (const uint32_t end = std::min(b.max_K, next_g + count); next_g < end; ++next_g) {
            std::vector<pa_run_state *> active;
            for (uint32_t r = 0; r < n; ++r)
                if (!finished[r] && next_g < runs[r]->plan.desc.K) active.push_back(runs[r]);
            if (active.empty()) {
                next_g = b.max_K;
                break;
            }
            steps.push_back(build_step(active, blob, cursor));
        }
    };
    if (ctx->graphs) {
        const size_t from = cursor;
        build_steps(b.max_K);
        if ((st = upload(from))) return cleanup(st);
        // Replay (capturing first if needed) the step sequence as one graph on
        // the context's stream, ordered after everything on the caller's stream.
        std::string key((const char *)descs, sizeof(pa_run_desc) * n);
        for (uint32_t r = 0; r < n; ++r)
            key.append((const char *)descs[r].beta, sizeof(double) * descs[r].K);
        key.append((const char *)&d_ws, sizeof d_ws);
        key.append((const char *)&ws_bytes, sizeof ws_bytes);
        for (int i = 0; i < pa::LANE_CHOICE_COUNT; ++i) key.append((const char *)&ctx->lanes[i], 4);
        {
            std::lock_guard<std::mutex> lk(ctx->tune_mu);
            key.append((const char *)&ctx->tune_gen, sizeof ctx->tune_gen);
        }
        hipGraphExec_t exec = nullptr;
        for (auto &g : ctx->graph_cache)
            if (g.key == key) exec = g.exec;
        hipStream_t gs = ctx->graph_stream;
        if (!exec) {
            hipGraph_t graph = nullptr;
            if ((st = hip_check(nullptr, hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal), "capture")))
                return cleanup(st);
            for (const StepLaunch &L : steps)
                if (!st) st = launch_step(L, dtab, gs);
            pa_status st2 = hip_check(nullptr, hipStreamEndCapture(gs, &graph), "end capture");
            if (st || st2) { if (graph) (void)hipGraphDestroy(graph); return cleanup(st ? st : st2); }
            st = hip_check(nullptr, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "instantiate");
            (void)hipGraphDestroy(graph);
            if (st) return cleanup(st);
            if (ctx->graph_cache.size() >= 8) {
                (void)hipGraphExecDestroy(ctx->graph_cache.front().exec);
                ctx->graph_cache.pop_front();
            }
            ctx->graph_cache.push_back({key, exec});
        }
        if ((st = hip_check(nullptr, hipEventRecord(ctx->ev_in, s), "record")) ||
            (st = hip_check(nullptr, hipStreamWaitEvent(gs, ctx->ev_in, 0), "wait")) ||
            (st = hip_check(nullptr, hipGraphLaunch(exec, gs), "graph launch")) ||
            (st = hip_check(nullptr, hipEventRecord(ctx->ev_out, gs), "record")) ||
            (st = hip_check(nullptr, hipStreamWaitEvent(s, ctx->ev_out, 0), "wait")))
            return cleanup(st);
    } else {
        // in growing chunks of steps: the device starts on the first steps
        // while the host builds the next
        for (uint32_t chunk = 4; next_g < b.max_K; chunk = std::min(2 * chunk, 64u)) {
            const size_t from = cursor, first = steps.size();
            build_steps(chunk);
            if ((st = upload(from))) return cleanup(st);
            for (size_t k = first; k < steps.size(); ++k) {
                if (ctx->abort_requested) return cleanup(fail(PA_ERR_CANCELLED, "batch aborted"));
                if ((st = launch_step(steps[k], dtab, s))) return cleanup(st);
            }
        }
    }
    uint8_t *blk = nullptr;
    if (outs) {
        blk = ctx_staging(ctx, stage_bytes, s);
        if (!blk) return cleanup(fail(PA_ERR_DEVICE, "cannot allocate pinned staging memory"));
        blk += align256(b.desc_bytes);
        if ((st = launch_prep(gather, dtab, s)) ||
            (st = hip_check(nullptr, hipMemcpyAsync(blk, ws + b.out_off, blk_total, hipMemcpyDeviceToHost, s),
                            "read results")))
            return cleanup(st);
    }
    if ((st = hip_check(nullptr, hipStreamSynchronize(s), "sync"))) return cleanup(st);
    pa_status first = PA_OK;
    for (uint32_t r = 0; r < n; ++r) {
        pa_status sr = finish_run(runs[r], outs ? &outs[r] : nullptr, outs ? blk + blk_off[r] : nullptr);
        runs[r] = nullptr;
        if (sr && !first) first = sr;
    }
    return first;
}

extern "C" pa_status pa_run_static(pa_ctx *ctx, const pa_run_desc *desc, void *stream, pa_result *out) {
    if (!ctx || !desc) return fail(PA_ERR_INVALID, "null context or description");
    pa_plan_info info;
    pa_status st = pa_plan(desc, &info);
    if (st) return st;
    if (info.workspace_bytes > PA_STATIC_SCRATCH_BYTES)
        return fail(PA_ERR_NOMEM, "the run's workspace exceeds the fixed workspace of pa_run_static (" +
                                      std::to_string(info.workspace_bytes) + " > " +
                                      std::to_string(PA_STATIC_SCRATCH_BYTES) + " bytes)");
    hipError_t e = hipSuccess;
    void *ws = pa::static_scratch(ctx->device, &e);
    if (!ws) return fail(PA_ERR_DEVICE, std::string("static workspace: ") + hipGetErrorString(e));
    const int prof = ctx->profiling;   // no timing events: they would be created per launch
    ctx->profiling = 0;
    st = pa_run(ctx, desc, ws, PA_STATIC_SCRATCH_BYTES, stream, out);
    ctx->profiling = prof;
    return st;
}

extern "C" pa_status pa_run(pa_ctx *ctx, const pa_run_desc *desc, void *d_ws, uint64_t ws_bytes, void *stream,
                 pa_result *out) {
    pa_run_state *r = nullptr;
    pa_status st = pa_run_begin(ctx, desc, d_ws, ws_bytes, stream, &r);
    if (st) return st;
    st = pa_run_advance(r, desc->K - 1);
    pa_status st2 = pa_run_finish(r, out);
    return st ? st : st2;
}


// ---------------------------------------------------------------------------
// Serving loop: continuous batching of PA runs inside a caller-provided arena.
// A scheduler thread admits queued requests whenever a run slot is free and
// the request's workspace fits the arena (first fit), then advances every
// admitted run by up to kStepsPerIteration global steps with the batched
// launches, retires finished runs (results copied into the caller's buffers,
// memory and slot released) and wakes their waiters.  Populations stay in the
// arena for the whole run.
// ---------------------------------------------------------------------------
namespace {

constexpr uint32_t kStepsPerIteration = 8;

double now_us() {
    using namespace std::chrono;
    return (double)duration_cast<nanoseconds>(steady_clock::now().time_since_epoch()).count() * 1e-3;
}

// First-fit allocator over [0, size) in 256-byte units, with coalescing.
class Arena {
  public:
    void reset(size_t size) { free_.clear(); if (size) free_[0] = size; }
    bool alloc(size_t bytes, size_t *off) {
        bytes = align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align256(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t largest() const {
        size_t m = 0;
        for (auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }

  private:
    std::map<size_t, size_t> free_;
};

enum class ReqState { Queued, Running, Done };

struct Request {
    uint64_t ticket = 0;
    pa_run_desc desc{};
    std::vector<double> beta;
    pa_result out{};
    size_t bytes = 0, off = 0;
    double arrival_us = 0, admit_us = 0, done_us = 0;
    uint64_t attempts = 0;
    ReqState state = ReqState::Queued;
    bool cancel = false;
    pa_status status = PA_OK;
    std::string message;
    pa_run_state *run = nullptr;
    // a checkpoint asked for by pa_serve_checkpoint: 0 none, 1 pending, 2 written
    int ckpt_state = 0;
    std::string ckpt_path;
    pa_status ckpt_status = PA_OK;
    std::string ckpt_msg;
    // a request resumed from a checkpoint (pa_serve_resume)
    bool resume = false;
    Checkpoint from;
    std::vector<uint8_t> from_spins;
};

}  // namespace

struct Server {
    pa_ctx *ctx = nullptr;
    uint8_t *arena = nullptr;
    size_t desc_bytes = 0;        // descriptor region at the start of the arena
    size_t run_bytes = 0;         // the rest, for run workspaces
    uint32_t max_slots = 0;
    hipStream_t stream = nullptr;
    double t0 = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queue;
    std::map<uint64_t, std::shared_ptr<Request>> tickets;
    std::vector<std::shared_ptr<Request>> active;
    Arena alloc;
    uint64_t next_ticket = 1;
    bool stopping = false;
    std::thread thread;

    void finish(const std::shared_ptr<Request> &q, pa_status st, const std::string &msg) {
        q->status = st;
        q->message = msg;
        q->done_us = now_us() - t0;
        q->state = ReqState::Done;
    }

    void loop() {
        (void)hipSetDevice(ctx->device);
        std::vector<uint8_t> blob;
        for (;;) {
            std::vector<std::shared_ptr<Request>> admitted;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] { return stopping || !queue.empty() || !active.empty(); });
                if (stopping && active.empty()) {
                    for (auto &q : queue) finish(q, PA_ERR_CANCELLED, "server stopped");
                    queue.clear();
                    cv_done.notify_all();
                    return;
                }
                // Admission in arrival order; a request that does not fit yet
                // lets later, smaller ones pass.
                for (auto it = queue.begin(); it != queue.end();) {
                    auto q = *it;
                    if (q->cancel) {
                        finish(q, PA_ERR_CANCELLED, "cancelled while queued");
                        it = queue.erase(it);
                        continue;
                    }
                    if (stopping) break;
                    if (active.size() + admitted.size() >= max_slots) break;
                    size_t off;
                    if (!alloc.alloc(q->bytes, &off)) { ++it; continue; }
                    q->off = off;
                    q->admit_us = now_us() - t0;
                    q->state = ReqState::Running;
                    admitted.push_back(q);
                    it = queue.erase(it);
                }
                cv_done.notify_all();
            }
            for (auto &q : admitted) {
                pa_run_state *run = nullptr;
                pa_status st = q->resume ? resume_run(ctx, q->from, q->from_spins, arena + desc_bytes + q->off,
                                                      align256(q->bytes), stream, &run)
                                         : pa_run_begin(ctx, &q->desc, arena + desc_bytes + q->off,
                                                        align256(q->bytes), stream, &run);
                q->from_spins = std::vector<uint8_t>();   // loaded; release the host copy
                std::lock_guard<std::mutex> lk(mu);
                if (st) {
                    alloc.release(q->off, q->bytes);
                    finish(q, st, g_last_error);
                    continue;
                }
                q->run = run;
                active.push_back(q);
            }
            // Checkpoints asked for since the last round (the runs are
            // synchronised at a step boundary here), written outside the lock.
            std::vector<std::shared_ptr<Request>> ckpts;
            {
                std::lock_guard<std::mutex> lk(mu);
                for (auto &q : active)
                    if (q->ckpt_state == 1) ckpts.push_back(q);
            }
            for (auto &q : ckpts) {
                const pa_status cs = write_checkpoint(q->run, q->ckpt_path.c_str());
                std::lock_guard<std::mutex> lk(mu);
                q->ckpt_status = cs;
                q->ckpt_msg = cs ? g_last_error : std::string();
                q->ckpt_state = 2;
            }
            if (!ckpts.empty()) {
                std::lock_guard<std::mutex> lk(mu);
                cv_done.notify_all();
            }
            // Up to kStepsPerIteration global steps of every active run.
            std::vector<pa_run_state *> runs;
            {
                std::lock_guard<std::mutex> lk(mu);
                for (auto &q : active)
                    if (!q->cancel) runs.push_back(q->run);
            }
            size_t cursor = 0;
            std::vector<StepLaunch> steps;
            for (uint32_t k = 0; k < kStepsPerIteration; ++k) {
                std::vector<pa_run_state *> act;
                for (auto *r : runs)
                    if (r->step + 1 < r->plan.desc.K) act.push_back(r);
                if (act.empty()) break;
                steps.push_back(build_step(act, blob, cursor));
            }
            pa_status st = PA_OK;
            if (!steps.empty()) {
                st = hip_check(nullptr, hipMemcpyAsync(arena, blob.data(), cursor, hipMemcpyHostToDevice, stream),
                               "upload descriptors");
                for (const auto &L : steps)
                    if (!st) st = launch_step(L, arena, stream);
            }
            if (!st) st = hip_check(nullptr, hipStreamSynchronize(stream), "sync");
            const std::string msg = st ? g_last_error : std::string();
            // Retire finished, cancelled or failed runs.
            std::lock_guard<std::mutex> lk(mu);
            for (auto it = active.begin(); it != active.end();) {
                auto q = *it;
                const bool done = q->run->step + 1 >= q->run->plan.desc.K;
                if (!(done || q->cancel || st)) { ++it; continue; }
                pa_status fs;
                if (st) {
                    pa_run_finish(q->run, nullptr);
                    fs = st;
                } else if (q->cancel) {
                    pa_run_finish(q->run, nullptr);
                    fs = PA_ERR_CANCELLED;
                } else {
                    fs = pa_run_finish(q->run, &q->out);
                }
                q->run = nullptr;
                alloc.release(q->off, q->bytes);
                if (q->ckpt_state == 1) {
                    q->ckpt_status = PA_ERR_INVALID;
                    q->ckpt_msg = "the request finished before its checkpoint";
                    q->ckpt_state = 2;
                }
                finish(q, fs, fs ? (st ? msg : (q->cancel ? "cancelled while running" : g_last_error)) : "");
                it = active.erase(it);
            }
            cv_done.notify_all();
        }
    }
};

extern "C" {

// The context's server, or null; the reference keeps it alive for the call.
static std::shared_ptr<Server> server_of(pa_ctx *ctx) {
    std::lock_guard<std::mutex> lk(ctx->serve_mu);
    return ctx->server;
}

pa_status pa_serve_start(pa_ctx *ctx, void *d_arena, uint64_t arena_bytes, uint32_t max_slots, void *stream) {
    if (!ctx || !d_arena || max_slots == 0 || ((uintptr_t)d_arena & 255u))
        return fail(PA_ERR_INVALID, "bad serving arguments");
    std::lock_guard<std::mutex> lk(ctx->serve_mu);
    if (ctx->server) return fail(PA_ERR_BUSY, "a server is already running on this context");
    std::shared_ptr<Server> sv;
    try {
        sv = std::make_shared<Server>();
    } catch (const std::bad_alloc &) {
        return fail(PA_ERR_NOMEM, "out of host memory");
    }
    sv->ctx = ctx;
    sv->arena = static_cast<uint8_t *>(d_arena);
    sv->max_slots = max_slots;
    sv->desc_bytes = align256(step_desc_bytes(max_slots) * kStepsPerIteration);
    if (arena_bytes <= sv->desc_bytes) return fail(PA_ERR_NOMEM, "arena too small");
    sv->run_bytes = (arena_bytes - sv->desc_bytes) & ~size_t(255);
    sv->alloc.reset(sv->run_bytes);
    sv->stream = static_cast<hipStream_t>(stream);
    sv->t0 = now_us();
    Server *raw = sv.get();
    sv->thread = std::thread([raw] { raw->loop(); });
    ctx->server = std::move(sv);
    return PA_OK;
}

// Queue request q for run description desc (first step to run: step0 + 1).
static pa_status enqueue(const std::shared_ptr<Server> &sv, const std::shared_ptr<Request> &q,
                         const pa_run_desc *desc, uint32_t step0, pa_result *out, uint64_t *ticket) {
    Plan p;
    pa_status st = build_plan(desc, p);
    if (st) return st;
    if (align256(p.total) > sv->run_bytes)
        return fail(PA_ERR_NOMEM, "the run's workspace exceeds the serving arena");
    q->desc = *desc;
    q->beta.assign(desc->beta, desc->beta + desc->K);
    q->desc.beta = q->beta.data();
    if (q->resume) q->from.desc.beta = q->from.beta.data();
    if (out) q->out = *out;
    q->bytes = p.total;
    double att = 0;
    for (uint32_t i = step0 + 1; i < desc->K; ++i) att += (double)desc->theta * p.N * (double)p.R_sched[i];
    q->attempts = (uint64_t)att;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stopping) return fail(PA_ERR_CANCELLED, "server stopping");
    q->ticket = sv->next_ticket++;
    q->arrival_us = now_us() - sv->t0;
    sv->tickets[q->ticket] = q;
    sv->queue.push_back(q);
    *ticket = q->ticket;
    sv->cv_work.notify_one();
    return PA_OK;
}

pa_status pa_serve_submit(pa_ctx *ctx, const pa_run_desc *desc, pa_result *out, uint64_t *ticket) {
    if (!ctx || !desc || !ticket) return fail(PA_ERR_INVALID, "null argument");
    const std::shared_ptr<Server> sv = server_of(ctx);
    if (!sv) return fail(PA_ERR_INVALID, "no server");
    return enqueue(sv, std::make_shared<Request>(), desc, 0, out, ticket);
}

pa_status pa_serve_resume(pa_ctx *ctx, const char *path, pa_result *out, uint64_t *ticket) {
    if (!ctx || !ticket) return fail(PA_ERR_INVALID, "null argument");
    const std::shared_ptr<Server> sv = server_of(ctx);
    if (!sv) return fail(PA_ERR_INVALID, "no server");
    auto q = std::make_shared<Request>();
    pa_status st = read_checkpoint(path, q->from, &q->from_spins);
    if (st) return st;
    q->resume = true;
    return enqueue(sv, q, &q->from.desc, q->from.step, out, ticket);
}

pa_status pa_serve_checkpoint(pa_ctx *ctx, uint64_t ticket, const char *path) {
    if (!ctx || !path) return fail(PA_ERR_INVALID, "null argument");
    const std::shared_ptr<Server> sv = server_of(ctx);
    if (!sv) return fail(PA_ERR_INVALID, "no server");
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return fail(PA_ERR_INVALID, "unknown ticket");
    const std::shared_ptr<Request> q = it->second;
    if (q->state == ReqState::Queued) return fail(PA_ERR_BUSY, "request not admitted yet");
    if (q->state == ReqState::Done) return fail(PA_ERR_INVALID, "request already finished");
    if (q->ckpt_state != 0) return fail(PA_ERR_BUSY, "a checkpoint of this ticket is in progress");
    q->ckpt_path = path;
    q->ckpt_state = 1;
    sv->cv_work.notify_one();
    sv->cv_done.wait(lk, [&] { return q->ckpt_state == 2; });
    q->ckpt_state = 0;
    if (q->ckpt_status) return fail(q->ckpt_status, q->ckpt_msg);
    return PA_OK;
}

pa_status pa_serve_wait(pa_ctx *ctx, uint64_t ticket, int64_t timeout_us, pa_timing *timing) {
    if (!ctx) return fail(PA_ERR_INVALID, "null context");
    const std::shared_ptr<Server> sv = server_of(ctx);
    if (!sv) return fail(PA_ERR_INVALID, "no server");
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return fail(PA_ERR_INVALID, "unknown ticket");
    const std::shared_ptr<Request> q = it->second;
    auto ready = [&] { return q->state == ReqState::Done; };
    if (timeout_us < 0) sv->cv_done.wait(lk, ready);
    else if (!sv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready))
        return fail(PA_ERR_TIMEOUT, "request not finished");
    // Another wait on the same ticket may have consumed it meanwhile.
    auto again = sv->tickets.find(ticket);
    if (again == sv->tickets.end() || again->second != q)
        return fail(PA_ERR_INVALID, "ticket consumed by another wait");
    sv->tickets.erase(again);
    if (timing) {
        timing->arrival_us = q->arrival_us;
        timing->admit_us = q->admit_us;
        timing->done_us = q->done_us;
        timing->attempts = q->attempts;
    }
    if (q->status) return fail(q->status, q->message);
    return PA_OK;
}

pa_status pa_serve_cancel(pa_ctx *ctx, uint64_t ticket) {
    if (!ctx) return fail(PA_ERR_INVALID, "null context");
    const std::shared_ptr<Server> sv = server_of(ctx);
    if (!sv) return fail(PA_ERR_INVALID, "no server");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return fail(PA_ERR_INVALID, "unknown ticket");
    it->second->cancel = true;
    sv->cv_work.notify_one();
    return PA_OK;
}

pa_status pa_serve_stop(pa_ctx *ctx) {
    if (!ctx) return fail(PA_ERR_INVALID, "null context");
    std::shared_ptr<Server> sv;
    {
        std::lock_guard<std::mutex> lk(ctx->serve_mu);
        sv = std::move(ctx->server);
        ctx->server.reset();
    }
    if (!sv) return fail(PA_ERR_INVALID, "no server");
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stopping = true;
        sv->cv_work.notify_one();
    }
    sv->thread.join();
    // Waits still in flight hold their own references; the server is freed
    // when the last of them returns.
    return PA_OK;
}

}  // extern "C"
