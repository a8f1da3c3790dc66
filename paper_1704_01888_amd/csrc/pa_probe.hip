// pa_probe.hip -- instruction issue-rate probes for gfx950.
//
// The Metropolis sweep is bound by the issue of plain 32-bit integer vector
// instructions, whose rates on gfx950 differ by kind: simple bitwise
// operations issue faster than one wave64 instruction per clock and compute
// unit, the 32x32->64 multiply-add and the byte permutations and SADs slower.
// Each probe runs a stream of one kind of instruction (or the sweep's mix of
// kinds) in eight independent chains per lane, with enough resident waves that
// latency is hidden, and reports lane-instructions per second.  These rates
// bound the sweep from above: its inner loop is a fixed multiset of these
// instructions per attempt, so it cannot issue faster than the sum of their
// times.
//
// Every instruction is written as inline assembly so that the compiler
// neither merges nor removes any; the chains are folded into one word per
// thread at the end and stored, so the work is live.
#include "pa_device.h"
#include "pa.h"

namespace pa {
namespace {

constexpr uint32_t PROBE_THREADS = 256;
constexpr uint32_t PROBE_CHAINS = 8;

// One instruction of kind K on chain value x (32-bit) or acc (64-bit).
#define P_XOR(x) asm volatile("v_xor_b32 %0, %1, %0" : "+v"(x) : "v"(b))
#define P_AND(x) asm volatile("v_and_b32 %0, %1, %0" : "+v"(x) : "v"(b))
#define P_BITOP3(x) asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(x) : "v"(b), "v"(c))
#define P_PERM(x) asm volatile("v_perm_b32 %0, %0, %1, %2" : "+v"(x) : "v"(b), "v"(c))
#define P_SAD(x) asm volatile("v_sad_u8 %0, %1, %2, %0" : "+v"(x) : "v"(b), "v"(c))
#define P_XAD(x) asm volatile("v_xad_u32 %0, %0, %1, %2" : "+v"(x) : "v"(b), "v"(c))
#define P_MULHI(x) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(x) : "v"(b))
// The 32x32->64 multiply-add is written in C, as the sweep's Philox products
// are: the compiler emits one v_mad_u64_u32 (low word of y times b, plus the
// 64-bit d) and, knowing the instruction, no hazard padding around it.
#define P_MAD64(y) (y = (uint64_t)(uint32_t)(y) * b + d)
#define P_CMPSEL(x) \
    asm volatile("v_cmp_le_u32 vcc, %0, %1\n\tv_cndmask_b32 %0, %0, %2, vcc" : "+v"(x) : "v"(b), "v"(c) : "vcc")

template <uint32_t KIND>
__global__ void __launch_bounds__(PROBE_THREADS) k_issue_probe(uint32_t iters, uint32_t *out) {
    const uint32_t t = blockIdx.x * PROBE_THREADS + threadIdx.x;
    const uint32_t b = t * 0x9E3779B9u + 1u, c = t ^ 0x5bd1e995u;
    const uint64_t d = ((uint64_t)c << 32) | b;
    uint32_t x[PROBE_CHAINS];
    uint64_t y[PROBE_CHAINS];
#pragma unroll
    for (uint32_t j = 0; j < PROBE_CHAINS; ++j) {
        x[j] = t + j * 0x01000193u;
        y[j] = ((uint64_t)x[j] << 32) | (t ^ j);
    }
    for (uint32_t it = 0; it < iters; ++it) {
        // two instructions per chain, the chains interleaved, so that
        // neighbouring instructions never depend on each other
#pragma unroll
        for (uint32_t rep = 0; rep < 2; ++rep) {
#pragma unroll
            for (uint32_t j = 0; j < PROBE_CHAINS; ++j) {
                if constexpr (KIND == PA_PROBE_XOR) P_XOR(x[j]);
                if constexpr (KIND == PA_PROBE_BITOP3) P_BITOP3(x[j]);
                if constexpr (KIND == PA_PROBE_MAD64) P_MAD64(y[j]);
                if constexpr (KIND == PA_PROBE_PERM) P_PERM(x[j]);
                if constexpr (KIND == PA_PROBE_SAD) P_SAD(x[j]);
                if constexpr (KIND == PA_PROBE_XAD) P_XAD(x[j]);
                if constexpr (KIND == PA_PROBE_MULHI) P_MULHI(x[j]);
            }
        }
        if constexpr (KIND == PA_PROBE_CMPSEL) {
#pragma unroll
            for (uint32_t j = 0; j < PROBE_CHAINS; ++j) P_CMPSEL(x[j]);
        }
        if constexpr (KIND == PA_PROBE_MIX) {
            // The kinds of one pair update of the sweep's inner loop (two
            // attempts): 18 multiply-adds and 19 three-input bitops (Philox and
            // the proposal), 4 each of perm, xad and sad (neighbour packing,
            // flags, threshold address), 2 xor, 2 and, and 2 compare-select
            // pairs: 57 instructions over the eight 32-bit and eight 64-bit
            // chains, no two neighbours on one chain.
#pragma unroll
            for (uint32_t rep = 0; rep < 2; ++rep) {
#pragma unroll
                for (uint32_t j = 0; j < PROBE_CHAINS; ++j) { P_MAD64(y[j]); P_BITOP3(x[j]); }
            }
            P_MAD64(y[0]); P_BITOP3(x[2]); P_MAD64(y[1]); P_BITOP3(x[3]); P_PERM(x[0]);
            P_BITOP3(x[4]); P_PERM(x[1]); P_XAD(x[5]); P_PERM(x[2]); P_XAD(x[6]);
            P_PERM(x[3]); P_XAD(x[7]); P_SAD(x[0]); P_XAD(x[4]); P_SAD(x[1]); P_XOR(x[5]);
            P_SAD(x[2]); P_XOR(x[6]); P_SAD(x[3]); P_AND(x[7]); P_CMPSEL(x[1]); P_AND(x[0]);
            P_CMPSEL(x[2]);
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (uint32_t j = 0; j < PROBE_CHAINS; ++j) r ^= x[j] ^ (uint32_t)y[j] ^ (uint32_t)(y[j] >> 32);
    out[t] = r;
}

// Lane-instructions one thread issues per iteration of kind K.
uint32_t probe_instr_per_iter(uint32_t kind) {
    switch (kind) {
        case PA_PROBE_CMPSEL: return 2u * PROBE_CHAINS;
        case PA_PROBE_MIX: return 57u;
        default: return 2u * PROBE_CHAINS;
    }
}

void *probe_kernel(uint32_t kind) {
    switch (kind) {
        case PA_PROBE_XOR: return (void *)k_issue_probe<PA_PROBE_XOR>;
        case PA_PROBE_BITOP3: return (void *)k_issue_probe<PA_PROBE_BITOP3>;
        case PA_PROBE_MAD64: return (void *)k_issue_probe<PA_PROBE_MAD64>;
        case PA_PROBE_PERM: return (void *)k_issue_probe<PA_PROBE_PERM>;
        case PA_PROBE_SAD: return (void *)k_issue_probe<PA_PROBE_SAD>;
        case PA_PROBE_XAD: return (void *)k_issue_probe<PA_PROBE_XAD>;
        case PA_PROBE_MULHI: return (void *)k_issue_probe<PA_PROBE_MULHI>;
        case PA_PROBE_CMPSEL: return (void *)k_issue_probe<PA_PROBE_CMPSEL>;
        case PA_PROBE_MIX: return (void *)k_issue_probe<PA_PROBE_MIX>;
        default: return nullptr;
    }
}

}  // namespace

hipError_t issue_probe(uint32_t kind, uint32_t blocks, uint32_t iters, uint32_t *out, hipStream_t s,
                       double *lane_instr_per_s, double *ms_out) {
    void *k = probe_kernel(kind);
    if (!k) return hipErrorInvalidValue;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e;
    if ((e = hipEventCreate(&a)) != hipSuccess) return e;
    if ((e = hipEventCreate(&b)) != hipSuccess) { (void)hipEventDestroy(a); return e; }
    double best = 1e300;
    // one warm-up launch, then the fastest of three timed ones
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
        (void)hipEventRecord(a, s);
        hipLaunchKernelGGL((void (*)(uint32_t, uint32_t *))k, dim3(blocks), dim3(PROBE_THREADS), 0, s, iters, out);
        e = hipGetLastError();
        if (e != hipSuccess) break;
        (void)hipEventRecord(b, s);
        if ((e = hipEventSynchronize(b)) != hipSuccess) break;
        float ms = 0.f;
        if ((e = hipEventElapsedTime(&ms, a, b)) != hipSuccess) break;
        if (rep > 0 && ms < best) best = ms;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return e;
    const double lanes = (double)blocks * PROBE_THREADS;
    *lane_instr_per_s = lanes * (double)iters * probe_instr_per_iter(kind) / (best * 1e-3);
    if (ms_out) *ms_out = best;
    return hipSuccess;
}

uint32_t probe_threads() { return PROBE_THREADS; }

}  // namespace pa
