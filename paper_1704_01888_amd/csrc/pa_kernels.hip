// pa_kernels.hip -- gfx950 kernels for population annealing of the 2D q-state
// Potts model (arXiv:1704.01888, Sec. 2-3).
//
//   k_sweep        : initial population (step 1 of Sec. 2) or, per step, the
//                    gather of each new replica from its ancestor (eq. (1)) plus
//                    theta checkerboard Metropolis sweeps (step 3) held in LDS,
//                    then the energy of eq. (3) (and M~ of eq. (5)) per replica.
//   k_tiled_*      : the same for lattices beyond one workgroup's LDS, in HBM.
//   k_post         : workgroup 0: the energy (and M~) histograms from the
//                    per-replica values, population sums for eq. (4), the
//                    reference energy and ln Q of step 2 / eq. (2) in FP64,
//                    histogram widths (Sec. 4); workgroups 1, 2, ...: the
//                    integer weights W(|E_j - E_ref|) of the next resampling
//                    and their scan, one block of replicas each.
//   k_sample       : the multinomial draws of the resampling step.
//   k_countfill    : exclusive scan of the copy numbers -> ancestor of each new
//                    slot, one block of ancestors per workgroup.
//   *_batch        : the same for several runs in one launch.
//
// A replica held in LDS is updated by G lanes: part of a wave (small L), one
// or several waves, or lanes spanning wave boundaries.  Within one wave the two
// half-sweeps of a sweep need no workgroup barrier (LDS operations of a wave
// execute in order; a compiler fence keeps the half-sweeps apart); a replica
// spread over several waves uses barriers.
#include "pa_device.h"

namespace pa {

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

constexpr uint32_t PHILOX_M0 = 0xD2511F53u;
constexpr uint32_t PHILOX_M1 = 0xCD9E8D57u;
constexpr uint32_t PHILOX_W0 = 0x9E3779B9u;
constexpr uint32_t PHILOX_W1 = 0xBB67AE85u;

// Philox4x32-10 (Salmon et al., SC'11), all in registers.  The two xors of
// each output word are one three-input bitop (truth table 0x96 = a ^ b ^ c).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// The truth table of a three-input bitop weighs its operands 0xF0, 0xCC, 0xAA.
// Bitwise select m ? a : b.
__device__ __forceinline__ uint32_t bit_select(uint32_t m, uint32_t a, uint32_t b) {
    return __builtin_amdgcn_bitop3_b32(a, b, m, 0xE4);
}

// ~a & b.
__device__ __forceinline__ uint32_t and_not(uint32_t a, uint32_t b) {
    return __builtin_amdgcn_bitop3_b32(a, b, 0u, 0x0C);
}

// Rounds 2..10 of Philox after a first round whose product M0 * c0 is given.
__device__ __forceinline__ uint4 philox_from(uint64_t p0, uint32_t c1, uint32_t c2, uint32_t c3,
                                             uint32_t k0, uint32_t k1) {
    {
        const uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        uint32_t c0 = n0;
        c2 = n2;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
#pragma unroll
        for (int r = 1; r < 10; ++r) {
            const uint64_t q0 = (uint64_t)PHILOX_M0 * c0;
            const uint64_t q1 = (uint64_t)PHILOX_M1 * c2;
            const uint32_t m0 = xor3((uint32_t)(q1 >> 32), c1, k0);
            const uint32_t m2 = xor3((uint32_t)(q0 >> 32), c3, k1);
            c1 = (uint32_t)q1;
            c3 = (uint32_t)q0;
            c0 = m0;
            c2 = m2;
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        return make_uint4(c0, c1, c2, c3);
    }
}

__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
    return philox_from((uint64_t)PHILOX_M0 * c0, c1, c2, c3, k0, k1);
}

__device__ __forceinline__ uint64_t digest_term(uint32_t n, uint32_t k, uint32_t step, uint32_t d,
                                                uint32_t key0, uint32_t key1) {
    const uint4 w = philox(n, k, step, DOM_DIGEST << 28, key0, key1);
    return ((((uint64_t)w.y << 32) | (uint64_t)w.x) | 1ull) * (uint64_t)d;
}

__device__ __forceinline__ uint32_t mulhi32(uint32_t w, uint32_t n) { return __umulhi(w, n); }

// floor(w * n / 2^32) through the full 32x32->64 multiply: v_mad_u64_u32
// issues at about twice the rate of v_mul_hi_u32 on gfx950, but the compiler
// picks the latter when only the high half is used.
__device__ __forceinline__ uint32_t mulhi32_wide(uint32_t w, uint32_t n) {
    uint64_t prod, carry;
    asm("v_mad_u64_u32 %0, %1, %2, %3, 0" : "=v"(prod), "=s"(carry) : "v"(w), "s"(n));
    return (uint32_t)(prod >> 32);
}

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
    return __builtin_amdgcn_perm(hi, lo, sel);   // byte sel 0-3 from lo, 4-7 from hi
}

// Digest term of one dword of a replica: r * d mod 2^64, r the 64-bit word of
// Philox(n, k, step, DIGEST) made odd (so any change of d changes the term).
__device__ __forceinline__ uint64_t digest_term(uint32_t n, uint32_t k, uint32_t step, uint32_t d,
                                                uint32_t key0, uint32_t key1);

// Number of equal bytes between two words.
__device__ __forceinline__ uint32_t eq_bytes(uint32_t a, uint32_t b) {
    const uint32_t x = a ^ b;
    const uint32_t nz = (((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u;
    return 4u - __popc(nz);
}

// LDS of the sweep and tiled workgroups: a 128-byte header (the 64-bit
// thresholds, and the energy and digest sums of a multi-wave replica at bytes
// 96 and 104), the replica or tile rows, sums, and last the pair threshold
// table.  Thresholds are indexed by i = dE + 4; entries for dE <= 0 accept
// always.  T64: the exact 64-bit form "w < T" (T <= 2^32) in the header;
// otherwise the 32-bit form "w <= T - 1", valid when every T >= 1 (the host
// checks), in the pair table: entry (i0, i1), at byte 8 i0 + 72 i1 of it, holds
// the thresholds of i0 and i1 (81 entries, 648 bytes).  The table starts at
// least PAIR_SAD_BIAS bytes into the LDS, the constant the pair update's four
// flag SADs add, so that their sum can start from table - PAIR_SAD_BIAS.
constexpr uint32_t LDS_HDR = 128;
constexpr uint32_t PAIR_SAD_BIAS = 704, PAIR_TAB_BYTES = 648;

__host__ __device__ inline uint32_t pair_tab_off(uint32_t end) {
    const uint32_t e = (end + 7u) & ~7u;
    return e > PAIR_SAD_BIAS ? e : PAIR_SAD_BIAS;
}

// End of a sweep workgroup's LDS before the pair table: header, rpb replicas of
// N + 2L bytes, then the per-state counters of a multi-wave replica (eq. (5))
// or the digest, bond and per-state sums of spanning replicas.
__host__ __device__ inline uint32_t sweep_lds_end(uint32_t N, uint32_t L, uint32_t G, uint32_t rpb,
                                                  uint32_t q_counters) {
    uint32_t b = LDS_HDR + rpb * (N + 2u * L);
    if (G > 64u && G % 64u == 0) b += 1024u;
    else if (64u % G != 0) b += rpb * (12u + 4u * q_counters);
    return b;
}

// End of a tiled workgroup's LDS before the pair table: tile and side rows,
// plus the padding rows the fixed-layout kernel reads past the update range
// (one row per row step of a lane: RS = nt / (L/4) rows, at least one).
__host__ __device__ inline uint32_t tiled_lds_end(uint32_t rows, uint32_t halves, uint32_t L,
                                                  uint32_t nt, bool fixed) {
    const uint32_t rs = L / 4u >= nt ? 1u : nt / (L / 4u);
    return LDS_HDR + (rows + 2u * halves + (fixed ? rs : 0u)) * L;
}

template <bool T64>
__device__ __forceinline__ void load_thresholds(uint8_t *smem, uint32_t tab, const uint64_t *T, uint32_t tid,
                                                uint32_t nthreads) {
    if (T64) {
        if (tid < 9) {
            const int dE = (int)tid - 4;
            reinterpret_cast<uint64_t *>(smem)[tid] = dE <= 0 ? (1ull << 32) : T[dE - 1];
        }
        return;
    }
    for (uint32_t t = tid; t < 81u; t += nthreads) {
        const uint32_t i0 = t % 9u, i1 = t / 9u;
        const uint32_t a = i0 <= 4u ? 0xFFFFFFFFu : (uint32_t)(T[i0 - 5u] - 1u);
        const uint32_t b = i1 <= 4u ? 0xFFFFFFFFu : (uint32_t)(T[i1 - 5u] - 1u);
        *reinterpret_cast<uint2 *>(smem + tab + 8u * i0 + 72u * i1) = make_uint2(a, b);
    }
}

template <bool T64>
struct Thresholds {
    const uint8_t *smem;
    uint32_t tab;   // byte offset of the pair table
    // 64-bit form, by index dE + 4
    __device__ __forceinline__ bool accept_idx(uint32_t idx, uint32_t w) const {
        return reinterpret_cast<const uint64_t *>(smem)[idx] > (uint64_t)w;
    }
    // LDS byte address of the pair table, less PAIR_SAD_BIAS
    __device__ __forceinline__ uint32_t sad_start() const {
        return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) uint8_t *)smem + tab -
               PAIR_SAD_BIAS;
    }
    // the two thresholds at LDS byte address `at`
    __device__ __forceinline__ u32x2 pair_at(uint32_t at) const {
        return *(const __attribute__((address_space(3))) u32x2 *)(uintptr_t)at;
    }
};

// Flags (0x80 per byte) of the equal / unequal bytes of x = a ^ b.  With
// q <= 128 every byte of x has bit 7 clear, so adding 0x7F to each byte never
// carries into the next one and bit 7 of the sum marks a nonzero byte; for
// larger q the low seven bits are masked first.
template <bool QSMALL>
__device__ __forceinline__ uint32_t flags_eq(uint32_t x) {
    // one xor-add and one bitop (written as ~(x + c) & m, the compiler forms
    // the sum as m - x and spends a third instruction)
    if (QSMALL) return and_not(x + 0x7F7F7F7Fu, 0x80808080u);
    return ~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u;
}
template <bool QSMALL>
__device__ __forceinline__ uint32_t flags_ne(uint32_t x) {
    if (QSMALL) return (x + 0x7F7F7F7Fu) & 0x80808080u;
    return (((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u;
}

// Metropolis update of one site (Sec. 2 step 3; proposal and acceptance as in
// the header comment of pa.h) with the 64-bit thresholds.  sb = current spin in
// all four bytes, n = the four neighbours, one per byte.  Returns the new spin
// in all four bytes.
template <bool QSMALL, bool T64>
__device__ __forceinline__ uint32_t site_update(uint32_t sb, uint32_t n, uint32_t w_prop,
                                                uint32_t w_acc, uint32_t qm1,
                                                const Thresholds<T64> &thr) {
    const uint32_t s = sb & 0xFFu;
    const uint32_t rr = mulhi32_wide(w_prop, qm1);
    const uint32_t sp = rr + (rr >= s ? 1u : 0u);
    const uint32_t spb = perm(0u, sp, 0u);                 // broadcast byte 0
    const uint32_t eq_a = flags_eq<QSMALL>(n ^ sb), ne_b = flags_ne<QSMALL>(n ^ spb);
    // #equal(current) + #unequal(proposed) = 4 + dE
    uint32_t idx = __popc(ne_b) + __popc(eq_a);
    asm volatile("" : "+v"(idx));   // keep the index one add (no re-association)
    return thr.accept_idx(idx, w_acc) ? spb : sb;
}

// Per-parity constants of a pair update (see update_pair).
struct PairSel {
    uint32_t selH, selV, sel0, sel1, selS, mask;
    PairSel() = default;
    __device__ __forceinline__ explicit PairSel(uint32_t par) {
        const uint32_t pb = par * 0x01010101u;
        selH = par ? 0x04020200u : 0x03010107u;
        selV = 0x06020400u + pb;
        sel0 = pb;
        sel1 = pb + 0x02020202u;
        selS = pb + 0x02020000u;
        mask = 0x00FF00FFu << (par << 3);
    }
};

// Update of the two colour-c sites x0 = xb + par and x0 + 2 held in the row
// dword D0 (bytes xb..xb+3).  Dx is the dword left of D0 (par = 0) or right of
// it (par = 1); U and Dn are the dwords above and below.
template <bool QSMALL, bool T64>
__device__ __forceinline__ uint32_t update_pair(uint32_t D0, uint32_t Dx, uint32_t U, uint32_t Dn,
                                                const PairSel &ps, uint4 w, uint32_t qm1,
                                                const Thresholds<T64> &thr) {
    const uint32_t H = perm(Dx, D0, ps.selH);            // x0-1, x0+1, x0+1, x0+3
    const uint32_t V = perm(Dn, U, ps.selV);             // up0, down0, up1, down1
    if constexpr (!T64) {
        // Bytes 0-1 of H, V, S and P belong to site 0, bytes 2-3 to site 1.
        const uint32_t S = perm(0u, D0, ps.selS);        // s0, s0, s1, s1
        const uint32_t r0 = mulhi32_wide(w.x, qm1), r1 = mulhi32_wide(w.z, qm1);
        const uint32_t p0 = r0 + (r0 >= (S & 0xFFu) ? 1u : 0u);
        const uint32_t p1 = r1 + (r1 >= ((S >> 16) & 0xFFu) ? 1u : 0u);
        const uint32_t P = perm(p1, p0, 0x04040000u);    // s0', s0', s1', s1'
        // Flag bytes are 0x80 or 0.  A byte-SAD against 0x1C1C3C3C adds 60 + 8
        // or 60 per byte of site 0 and 28 + 72 or 28 per byte of site 1, so the
        // four SADs of the equal flags of s and the unequal flags of s' add
        // PAIR_SAD_BIAS + 8 i0 + 72 i1 (i = #equal(s) + #unequal(s') = dE + 4
        // per site): from sad_start(), the LDS address of the pair's two
        // thresholds, with no counts.
        uint32_t at = thr.sad_start();
        at = __builtin_amdgcn_sad_u8(flags_eq<QSMALL>(H ^ S), 0x1C1C3C3Cu, at);
        at = __builtin_amdgcn_sad_u8(flags_eq<QSMALL>(V ^ S), 0x1C1C3C3Cu, at);
        at = __builtin_amdgcn_sad_u8(flags_ne<QSMALL>(H ^ P), 0x1C1C3C3Cu, at);
        at = __builtin_amdgcn_sad_u8(flags_ne<QSMALL>(V ^ P), 0x1C1C3C3Cu, at);
        const u32x2 T = thr.pair_at(at);
        // X = bytes 0-1 of (w.y <= T.x ? P : S), bytes 2-3 of (w.w <= T.y ? P : S):
        // the second select takes the upper halves of S and P and writes only
        // the upper half of X (SDWA, lower half preserved), so no byte permute
        // merges the two sites.  A compare's VCC
        // is read two wait states later, as the compiler's own code does.
        uint32_t X;
        asm("v_cmp_le_u32 vcc, %[wy], %[tx]\n\t"
            "s_nop 1\n\t"
            "v_cndmask_b32 %[X], %[S], %[P], vcc\n\t"
            "v_cmp_le_u32 vcc, %[ww], %[ty]\n\t"
            "s_nop 1\n\t"
            "v_cndmask_b32_sdwa %[X], %[S], %[P], vcc dst_sel:WORD_1 dst_unused:UNUSED_PRESERVE "
            "src0_sel:WORD_1 src1_sel:WORD_1"
            : [X] "=&v"(X)
            : [wy] "v"(w.y), [tx] "v"(T.x), [ww] "v"(w.w), [ty] "v"(T.y), [S] "v"(S), [P] "v"(P)
            : "vcc");
        return bit_select(ps.mask, X, D0);
    }
    const uint32_t n0 = perm(V, H, 0x05040100u);
    const uint32_t n1 = perm(V, H, 0x07060302u);
    const uint32_t sb0 = perm(0u, D0, ps.sel0);
    const uint32_t sb1 = perm(0u, D0, ps.sel1);
    const uint32_t t0 = site_update<QSMALL, T64>(sb0, n0, w.x, w.y, qm1, thr);
    const uint32_t t1 = site_update<QSMALL, T64>(sb1, n1, w.z, w.w, qm1, thr);
    const uint32_t X = perm(t1, t0, 0x05040100u);         // s0', s0', s1', s1'
    return bit_select(ps.mask, X, D0);
}

// Philox for the sweep counter (p, k, step, c3) with k, step, c3 and the key
// wave-uniform: the first two rounds are half scalar.  P0 = M0 * p.
struct SweepKey {
    uint32_t n0, n1, c3k1, k0[10], k1[10];
};

__device__ __forceinline__ SweepKey sweep_key(uint32_t k, uint32_t step, uint32_t c3, uint32_t key0,
                                              uint32_t key1) {
    SweepKey s;
    uint32_t a0 = key0, a1 = key1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        s.k0[r] = a0;
        s.k1[r] = a1;
        a0 += PHILOX_W0;
        a1 += PHILOX_W1;
    }
    const uint64_t p1 = (uint64_t)PHILOX_M1 * step;
    s.n0 = (uint32_t)(p1 >> 32) ^ k ^ key0;
    s.n1 = (uint32_t)p1;
    s.c3k1 = c3 ^ key1;
    return s;
}

__device__ __forceinline__ uint4 philox_sweep(uint64_t P0, const SweepKey &s) {
    // round 1
    const uint32_t a2 = (uint32_t)(P0 >> 32) ^ s.c3k1;
    const uint32_t a3 = (uint32_t)P0;
    // round 2: M0 * n0 is uniform
    const uint64_t q0 = (uint64_t)PHILOX_M0 * s.n0;
    const uint64_t q1 = (uint64_t)PHILOX_M1 * a2;
    uint32_t c0 = (uint32_t)(q1 >> 32) ^ (s.n1 ^ s.k0[1]);
    uint32_t c1 = (uint32_t)q1;
    uint32_t c2 = a3 ^ ((uint32_t)(q0 >> 32) ^ s.k1[1]);
    uint32_t c3 = (uint32_t)q0;
#pragma unroll
    for (int r = 2; r < 10; ++r) {
        const uint64_t r0 = (uint64_t)PHILOX_M0 * c0;
        const uint64_t r1 = (uint64_t)PHILOX_M1 * c2;
        const uint32_t m0 = xor3((uint32_t)(r1 >> 32), c1, s.k0[r]);
        const uint32_t m2 = xor3((uint32_t)(r0 >> 32), c3, s.k1[r]);
        c1 = (uint32_t)r1;
        c3 = (uint32_t)r0;
        c0 = m0;
        c2 = m2;
    }
    return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Separates half-sweeps: within one wave LDS operations execute in order, so a
// compiler fence suffices; a replica spread over several waves needs the
// workgroup barrier.
__device__ __forceinline__ void replica_fence(bool multiwave) {
    if (multiwave) __syncthreads();
    else wave_fence();
}



// Replica layout in LDS: rows -1 .. L of L bytes each; row r at byte (r+1)*L.
// Rows -1 and L are copies of rows L-1 and 0 (periodic halo), kept current by
// the lanes that update rows L-1 and 0.
//
// Fixed L (a power of two) and G lanes per replica (a power of two between
// L/4 and 1024, fewer than a wave for small lattices, several waves for large
// ones): lane g of the replica's G lanes owns dword column
// xd = g mod L/4 and rows y0 + j*RS (y0 = g div L/4, RS = G / (L/4)), so all
// its addresses are the base plus compile-time offsets and its parity per
// unrolled slot is fixed.
template <uint32_t LT, uint32_t GT, bool QSMALL>
__device__ __forceinline__ void sweeps_fixed(uint32_t *lds32, uint32_t g, uint32_t k,
                                             const SweepArgs &a, const Thresholds<false> &thr,
                                             uint32_t theta) {
    constexpr uint32_t L = LT, N = L * L, P = N / 4, DPR = L / 4;
    constexpr uint32_t G = GT;
    constexpr uint32_t PPL = P / G, RS = G / DPR;
    constexpr uint32_t UNR = PPL % 2 == 0 ? 2 : (PPL % 3 == 0 ? 3 : 1);   // pairs interleaved
    static_assert(G % DPR == 0 && P % G == 0 && PPL % UNR == 0, "shape");
    static_assert(PPL == UNR || (RS * UNR) % 2 == 0, "slot parity must not change between iterations");
    const uint32_t xd = g % DPR, y0 = g / DPR;
    const int32_t dl = xd == 0 ? (int32_t)(DPR - 1) : -1;
    const int32_t dr = xd == DPR - 1 ? -(int32_t)(DPR - 1) : 1;
    const uint32_t base = (y0 + 1) * DPR + xd;
    const uint64_t mg = (uint64_t)PHILOX_M0 * g;                    // M0 * first pair
    constexpr uint64_t MSTEP = (uint64_t)PHILOX_M0 * G;              // M0 * pair stride
    const uint32_t qm1 = a.q - 1u;
    const bool top = y0 == 0, bottom = y0 + (PPL - 1) * RS == L - 1;
    for (uint32_t t = 0; t < theta; ++t) {
        #pragma unroll   // both colours in one body: the parity constants stay fixed
        for (uint32_t c = 0; c < 2u; ++c) {
            const SweepKey key = sweep_key(k, a.step, (DOM_SWEEP << 28) | (t << 1) | c, a.key0, a.key1);
            // parity of unrolled slot u (j is a multiple of UNR, and RS * UNR is even
            // unless there is a single iteration)
            PairSel ps[UNR];
            int32_t dx[UNR];
#pragma unroll
            for (uint32_t u = 0; u < UNR; ++u) {
                const uint32_t par = (y0 + u * RS + c) & 1u;
                ps[u] = PairSel(par);
                dx[u] = par ? dr : dl;
            }
            uint64_t P0 = mg;
            for (uint32_t j = 0; j < PPL; j += UNR) {
                uint32_t idx[UNR], D0[UNR], Dx[UNR], U[UNR], Dn[UNR];
                uint4 w[UNR];
#pragma unroll
                for (uint32_t u = 0; u < UNR; ++u) {
                    idx[u] = base + (j + u) * RS * DPR;
                    D0[u] = lds32[idx[u]];
                    Dx[u] = lds32[idx[u] + dx[u]];
                    U[u] = lds32[idx[u] - DPR];
                    Dn[u] = lds32[idx[u] + DPR];
                }
#pragma unroll
                for (uint32_t u = 0; u < UNR; ++u) w[u] = philox_sweep(P0 + u * MSTEP, key);
                P0 += UNR * MSTEP;
#pragma unroll
                for (uint32_t u = 0; u < UNR; ++u) {
                    const uint32_t nw = update_pair<QSMALL, false>(D0[u], Dx[u], U[u], Dn[u], ps[u],
                                                                   w[u], qm1, thr);
                    lds32[idx[u]] = nw;
                    if (j + u == 0 && top) lds32[idx[u] + L * DPR] = nw;
                    if (j + u == PPL - 1 && bottom) lds32[idx[u] - L * DPR] = nw;
                }
            }
            replica_fence(64u % G != 0u);
        }
    }
}

// Any L divisible by 4: pairs visited with an incremental (row, column) walk.
template <bool QSMALL, bool T64>
__device__ __forceinline__ void sweeps_any(uint32_t *lds32, uint32_t g, uint32_t G, uint32_t k,
                                           const SweepArgs &a, const Thresholds<T64> &thr,
                                           uint32_t theta) {
    const uint32_t L = a.L, N = a.N, H = L >> 1, P = N >> 2, DPR = L >> 2;
    const uint32_t step2G = 2u * G;
    const uint32_t dy = step2G / H, dj = step2G % H;
    const uint32_t qm1 = a.q - 1u;
    for (uint32_t t = 0; t < theta; ++t) {
        for (uint32_t c = 0; c < 2u; ++c) {
            const SweepKey key = sweep_key(k, a.step, (DOM_SWEEP << 28) | (t << 1) | c, a.key0, a.key1);
            uint32_t y = (2u * g) / H, j0 = (2u * g) % H;
            for (uint32_t p = g; p < P; p += G) {
                const uint32_t par = (y + c) & 1u;
                const uint32_t xd = j0 >> 1;                       // dword column
                const uint32_t idx = (y + 1) * DPR + xd;
                const uint32_t xo = par ? (xd == DPR - 1 ? idx - (DPR - 1) : idx + 1)
                                        : (xd == 0 ? idx + (DPR - 1) : idx - 1);
                const uint32_t D0 = lds32[idx], Dx = lds32[xo];
                const uint32_t U = lds32[idx - DPR], Dn = lds32[idx + DPR];
                const uint4 w = philox_sweep((uint64_t)PHILOX_M0 * p, key);
                const uint32_t nw = update_pair<QSMALL, T64>(D0, Dx, U, Dn, PairSel(par), w, qm1, thr);
                lds32[idx] = nw;
                if (y == 0) lds32[idx + L * DPR] = nw;
                if (y == L - 1) lds32[idx - L * DPR] = nw;
                j0 += dj;
                if (j0 >= H) { j0 -= H; ++y; }
                y += dy;
            }
            replica_fence(64u % G != 0u);
        }
    }
}

// f(i) for i = g, g + G, ... below n.  With the count and the stride known at
// compile time (NC, GC != 0) the loop has a constant trip count, so that its
// independent iterations (the loads of a gather) issue together.
template <uint32_t NC, uint32_t GC, typename F>
__device__ __forceinline__ void lane_stride(uint32_t g, uint32_t n, uint32_t G, F f) {
    if constexpr (NC != 0 && GC != 0) {
#pragma unroll
        for (uint32_t c = 0; c < (NC + GC - 1) / GC; ++c) {
            const uint32_t i = g + c * GC;
            if (NC % GC == 0 || i < NC) f(i);
        }
    } else {
        for (uint32_t i = g; i < n; i += G) f(i);
    }
}

// Sum over the 64 lanes of a wave (all active), wave-uniform: four DPP adds
// (quad_perm [1,0,3,2] and [2,3,0,1], row_ror 4 and 8) leave every lane of a
// row of 16 with the row's sum; the four row sums are read from lanes 0, 16,
// 32 and 48.
__device__ __forceinline__ uint32_t wave_total(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false);
    return (uint32_t)(__builtin_amdgcn_readlane((int)v, 0) + __builtin_amdgcn_readlane((int)v, 16) +
                      __builtin_amdgcn_readlane((int)v, 32) + __builtin_amdgcn_readlane((int)v, 48));
}

// One workgroup `block` of the sweep launch of one run (a): gather or create
// its replicas in LDS, theta sweeps, energies (and M~), store.  The workgroup
// is the nthreads threads tid = 0 .. nthreads-1 with the LDS at smem: a whole
// workgroup of k_sweep, or, in the persistent batched kernel, one of several
// such groups of waves that share a larger workgroup (PERSIST: every group
// runs the whole body, idle ones without storing, so that all groups meet the
// same workgroup barriers).
template <uint32_t LT, uint32_t GT, bool QSMALL, bool T64, bool PERSIST = false>
__device__ __forceinline__ void sweep_body(const SweepArgs &a, uint32_t block, uint8_t *smem, uint32_t tid,
                                           uint32_t nthreads, const uint32_t *anc, uint32_t anc_first,
                                           uint32_t R_new) {
    // Lanes per replica G: a divisor of 64 (one or several replicas per wave),
    // a multiple of 64 (one replica per block of G/64 waves), or neither
    // (replicas span wave boundaries, several per block: "spanning").  Every
    // replica not inside one wave separates its half-sweeps with barriers.
    const uint32_t G = GT ? GT : a.G;
    const bool multiwave = G > 64 && G % 64u == 0;               // one replica per block
    const bool span = 64u % G != 0 && !multiwave;
    if (tid == 32) reinterpret_cast<uint32_t *>(smem)[24] = 0u;   // energy sum (multi-wave)
    if (tid == 33) reinterpret_cast<uint64_t *>(smem)[13] = 0ull; // digest sum (multi-wave)
    if (a.Mt_out && multiwave) {   // per-state counters of a multi-wave replica, after its rows
        uint32_t *mcnt = reinterpret_cast<uint32_t *>(smem + LDS_HDR + a.N + 2 * a.L);
        for (uint32_t t = tid; t < a.q; t += nthreads) mcnt[t] = 0u;
    }
    if (span) {       // sums of spanning replicas, after all rows
        const uint32_t nr = nthreads / G;
        uint8_t *acc = smem + LDS_HDR + (size_t)nr * (a.N + 2 * a.L);
        const uint32_t words = nr * (3u + (a.Mt_out ? a.q : 0u));
        for (uint32_t t = tid; t < words; t += nthreads) reinterpret_cast<uint32_t *>(acc)[t] = 0u;
    }
    const bool barrier = multiwave || span;
    const uint32_t wave = tid >> 6;
    const uint32_t g = multiwave ? tid : tid % G;
    const uint32_t rpb = multiwave ? 1u : (64u * a.waves_per_block) / G;   // replicas per block

    // the pair threshold table after rows and sums (the host sizes the LDS alike)
    const uint32_t tab = pair_tab_off(sweep_lds_end(a.N, a.L, G, rpb, a.Mt_out ? a.q : 0u));
    load_thresholds<T64>(smem, tab, a.T, tid, nthreads);
    __syncthreads();
    const Thresholds<T64> thr{smem, tab};
    const uint32_t rep = multiwave ? 0u : tid / G;                         // replica within block
    const uint64_t k64 = (uint64_t)block * rpb + rep;
    // idle waves leave; with barriers only a whole idle block may (and in the
    // persistent kernel none)
    const uint64_t first_idle = multiwave ? (uint64_t)block
                                          : (uint64_t)block * rpb + (span ? 0u : (wave * 64u) / G);
    if (!PERSIST && first_idle >= R_new) return;
    const bool live = k64 < R_new;
    // wave-uniform when a wave holds (part of) one replica only
    const uint32_t k = G % 64u == 0 ? __builtin_amdgcn_readfirstlane((uint32_t)k64) : (uint32_t)k64;

    // compile-time shape where the kernel has one (LT != 0): the prologue and
    // epilogue loops then have constant bounds and strides
    const uint32_t L = LT ? LT : a.L, N = LT ? LT * LT : a.N, DPR = L >> 2;
    uint8_t *rep_lds = smem + LDS_HDR + (size_t)rep * (N + 2 * L);
    uint32_t *lds32 = reinterpret_cast<uint32_t *>(rep_lds);
    uint32_t *rows32 = lds32 + DPR;                              // row 0

    // ---- load or create the replica in LDS -----------------------------
    if (a.mode == SWEEP_UPDATE) {
        const uint32_t src = live ? (anc ? anc[k - anc_first] : k) : 0u;
        const uint4 *gsrc = reinterpret_cast<const uint4 *>(a.old_pop + (size_t)src * N);
        uint4 *ldst = reinterpret_cast<uint4 *>(rep_lds + L);
        lane_stride<LT * LT / 16, GT>(g, N / 16u, G, [&](uint32_t o) {
            ldst[o] = live ? gsrc[o] : make_uint4(0, 0, 0, 0);
        });
    } else if (a.mode == SWEEP_INIT_RANDOM) {
        // Site n takes word n mod 4 of Philox(n / 4, k, 0, INIT).
        for (uint32_t dd = g; dd < N / 4u; dd += G) {
            const uint4 w = philox(dd, k, 0u, DOM_INIT << 28, a.key0, a.key1);
            rows32[dd] = mulhi32(w.x, a.q) | (mulhi32(w.y, a.q) << 8) | (mulhi32(w.z, a.q) << 16) |
                         (mulhi32(w.w, a.q) << 24);
        }
    } else {
        // eq. (6): all spins alpha, alpha uniform over the q states.
        const uint4 w = philox(0u, k, 0u, DOM_GROUND << 28, a.key0, a.key1);
        const uint32_t alpha = mulhi32(w.x, a.q) * 0x01010101u;
        lane_stride<LT * LT / 4, GT>(g, N / 4u, G, [&](uint32_t dd) { rows32[dd] = alpha; });
    }
    replica_fence(barrier);
    lane_stride<LT / 4, GT>(g, DPR, G, [&](uint32_t dd) {       // periodic halo rows
        lds32[dd] = rows32[(L - 1) * DPR + dd];
        lds32[(L + 1) * DPR + dd] = rows32[dd];
    });
    replica_fence(barrier);

    // ---- theta checkerboard sweeps --------------------------------------
    const uint32_t theta = (a.mode == SWEEP_UPDATE) ? a.theta : 0u;
    if constexpr (LT != 0) sweeps_fixed<LT, GT, QSMALL>(lds32, g, k, a, thr, theta);
    else sweeps_any<QSMALL, T64>(lds32, g, G, k, a, thr, theta);

    // ---- energy (eq. (3)), store ------------------------------------------
    uint32_t bonds = 0;
    lane_stride<LT * LT / 4, GT>(g, N / 4u, G, [&](uint32_t dd) {
        const uint32_t xd = dd % DPR;
        const uint32_t idx = DPR + dd;
        const uint32_t D = lds32[idx];
        const uint32_t Dr = lds32[xd == DPR - 1 ? idx - (DPR - 1) : idx + 1];
        const uint32_t Dd = lds32[idx + DPR];
        const uint32_t right = __builtin_amdgcn_alignbyte(Dr, D, 1);
        bonds += eq_bytes(D, right) + eq_bytes(D, Dd);
    });
    // per-replica sums of spanning replicas: digest [rpb] u64, bonds [rpb],
    // per-state counts [rpb][q] u32, after all replicas' rows
    uint8_t *acc = smem + LDS_HDR + (size_t)rpb * (N + 2 * L);
    unsigned long long *acc_d = reinterpret_cast<unsigned long long *>(acc);
    uint32_t *acc_e = reinterpret_cast<uint32_t *>(acc + 8u * rpb);
    uint32_t *acc_m = acc_e + rpb;
    if (span) {
        atomicAdd(&acc_e[rep], bonds);
        __syncthreads();
        bonds = acc_e[rep];
    } else {
        if (G % 64u == 0) bonds = wave_total(bonds);
        else for (uint32_t off = G >> 1; off > 0; off >>= 1) bonds += __shfl_xor(bonds, off, 64);
        if (multiwave) {
            uint32_t *sum = reinterpret_cast<uint32_t *>(smem) + 24;
            if ((tid & 63u) == 0) atomicAdd(sum, bonds);
            __syncthreads();
            bonds = *sum;
        }
    }
    // ---- magnetisation (eq. (5)): M~ = the largest number of sites in one state
    uint32_t mt = 0;
    if (a.Mt_out) {
        uint32_t *mcnt = reinterpret_cast<uint32_t *>(rep_lds + N + 2 * L);   // multi-wave only
        for (uint32_t st = 0; st < a.q; ++st) {
            const uint32_t pat = st * 0x01010101u;
            uint32_t c = 0;
            for (uint32_t dd = g; dd < N / 4u; dd += G) c += eq_bytes(rows32[dd], pat);
            if (span) {
                atomicAdd(&acc_m[rep * a.q + st], c);
                continue;
            }
            if (G % 64u == 0) c = wave_total(c);
            else for (uint32_t off = G >> 1; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
            if (!multiwave) mt = max(mt, c);
            else if ((tid & 63u) == 0) atomicAdd(&mcnt[st], c);
        }
        if (multiwave || span) {
            __syncthreads();
            const uint32_t *cnt = span ? acc_m + rep * a.q : mcnt;
            for (uint32_t st = 0; st < a.q; ++st) mt = max(mt, cnt[st]);
        }
    }
    // ---- digest term of the replica (order-free sum over its dwords)
    uint64_t dig = 0;
    if (a.H_out) {
        for (uint32_t dd = g; dd < N / 4u; dd += G) dig += digest_term(dd, k, a.step, rows32[dd], a.key0, a.key1);
        if (span) {
            atomicAdd(&acc_d[rep], (unsigned long long)dig);
            __syncthreads();
            dig = acc_d[rep];
        } else {
            for (uint32_t off = (G < 64 ? G : 64) >> 1; off > 0; off >>= 1) dig += __shfl_xor(dig, off, 64);
        }
        if (multiwave) {
            unsigned long long *sum = reinterpret_cast<unsigned long long *>(smem) + 13;
            if ((tid & 63u) == 0) atomicAdd(sum, (unsigned long long)dig);
            __syncthreads();
            dig = *sum;
        }
    }
    if (live) {
        if (g == 0) {
            const int32_t E = -(int32_t)bonds;
            a.E_out[k] = E;
            if (a.Mt_out) a.Mt_out[k] = mt;
            if (a.H_out) a.H_out[k] = dig;
        }
        // streaming stores: the new population is read back by the next step's
        // gather, not through this kernel's L2, whose write-back at the end of
        // the launch then has little to do
        u32x4 *gdst = reinterpret_cast<u32x4 *>(a.new_pop + (size_t)k * N);
        const u32x4 *lsrc = reinterpret_cast<const u32x4 *>(rep_lds + L);
        lane_stride<LT * LT / 16, GT>(g, N / 16u, G, [&](uint32_t o) {
            __builtin_nontemporal_store(lsrc[o], &gdst[o]);
        });
    }
}

template <uint32_t LT, uint32_t GT, bool QSMALL, bool T64>
__global__ void __launch_bounds__(1024) k_sweep(SweepArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    sweep_body<LT, GT, QSMALL, T64>(a, blockIdx.x, smem, threadIdx.x, blockDim.x, a.anc, 0u, a.R_new);
}

// Index of the segment holding `block`: the last r < n with start[r] <= block
// (start is non-decreasing from start[0] = 0, so segments without workgroups
// are skipped).  Each wave counts the starts not after `block`, 64 per round
// of vector loads, instead of following a chain of dependent loads through a
// binary search; every thread of the workgroup must call it.
__device__ __forceinline__ uint32_t segment_of(const uint32_t *start, uint32_t n, uint32_t block) {
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t count = 0;
    for (uint32_t i0 = 0; i0 < n; i0 += 64u) {
        const uint32_t i = i0 + lane;
        const bool before = i < n && start[i] <= block;
        count += (uint32_t)__popcll(__ballot(before));
    }
    return __builtin_amdgcn_readfirstlane(count - 1u);
}

// Batched form: the workgroups of several runs' sweep launches (same lattice
// class) in one launch; run r owns workgroups start[r] .. start[r+1]-1.
template <uint32_t LT, uint32_t GT, bool QSMALL, bool T64>
__global__ void __launch_bounds__(1024) k_sweep_batch(const SweepArgs *runs, const uint32_t *start,
                                                      uint32_t n) {
    const uint32_t r = segment_of(start, n, blockIdx.x);
    // by reference: a local copy would go to scratch memory (T[] is indexed at run time)
    const SweepArgs &a = runs[r];
    extern __shared__ __align__(16) uint8_t smem[];
    sweep_body<LT, GT, QSMALL, T64>(a, blockIdx.x - start[r], smem, threadIdx.x, blockDim.x, a.anc, 0u, a.R_new);
}

// ---------------------------------------------------------------------------
// Lattices with L = 2 (mod 4): a row of L bytes is not a whole number of
// dwords, and a row holds L/2 sites of each colour, an odd number, so the two
// sites of one Philox block (the m-th and (m+1)-th colour-c sites in row-major
// order, m even) can lie in consecutive rows.  One wave holds a replica in LDS
// byte by byte, without halo rows: lane l updates the pairs p = l, l + 64, ...
// of each half-sweep, site by site, with the same counters, thresholds and
// update rule as the dword kernels (Sec. 2 step 3).  The population size N =
// L^2 is a multiple of 4, so the gather, the initial spins, the digest and the
// store still move whole dwords.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wrap_next(uint32_t v, uint32_t L) { return v + 1u == L ? 0u : v + 1u; }
__device__ __forceinline__ uint32_t wrap_prev(uint32_t v, uint32_t L) { return v == 0u ? L - 1u : v - 1u; }

// Metropolis update of site (y, x) of the replica s (L x L bytes).
__device__ __forceinline__ void byte_site_update(uint8_t *s, uint32_t L, uint32_t y, uint32_t x,
                                                 uint32_t w_prop, uint32_t w_acc, uint32_t qm1,
                                                 const SweepArgs &a) {
    const uint32_t row = y * L;
    const uint32_t cur = s[row + x];
    const uint32_t nb0 = s[row + wrap_prev(x, L)], nb1 = s[row + wrap_next(x, L)];
    const uint32_t nb2 = s[wrap_prev(y, L) * L + x], nb3 = s[wrap_next(y, L) * L + x];
    const uint32_t r = mulhi32(w_prop, qm1);
    const uint32_t prop = r + (r >= cur ? 1u : 0u);
    const int32_t dE = (int32_t)((nb0 == cur) + (nb1 == cur) + (nb2 == cur) + (nb3 == cur)) -
                       (int32_t)((nb0 == prop) + (nb1 == prop) + (nb2 == prop) + (nb3 == prop));
    // T[dE - 1] by selects: a run-time index into the arguments would go
    // through scratch memory
    const uint64_t T = dE == 1 ? a.T[0] : dE == 2 ? a.T[1] : dE == 3 ? a.T[2] : a.T[3];
    if (dE <= 0 || (uint64_t)w_acc < T) s[row + x] = (uint8_t)prop;
}

__device__ __forceinline__ void sweep_bytes_body(const SweepArgs &a, uint32_t block) {
    extern __shared__ __align__(16) uint8_t smem[];
    const uint32_t L = a.L, N = a.N, lane = threadIdx.x & 63u;
    const uint32_t rpb = blockDim.x >> 6;                                  // one replica per wave
    const uint64_t k64 = (uint64_t)block * rpb + (threadIdx.x >> 6);
    if (k64 >= a.R_new) return;              // whole waves only; no workgroup barriers below
    const uint32_t k = __builtin_amdgcn_readfirstlane((uint32_t)k64);
    uint8_t *rep = smem + (size_t)(threadIdx.x >> 6) * ((N + 15u) & ~15u);
    uint32_t *rep32 = reinterpret_cast<uint32_t *>(rep);
    const uint32_t D = N >> 2;                                             // dwords per replica

    if (a.mode == SWEEP_UPDATE) {
        const uint32_t src = a.anc ? a.anc[k] : k;
        const uint32_t *g = reinterpret_cast<const uint32_t *>(a.old_pop + (size_t)src * N);
        for (uint32_t d = lane; d < D; d += 64u) rep32[d] = g[d];
    } else if (a.mode == SWEEP_INIT_RANDOM) {
        // site n takes word n mod 4 of Philox(n / 4, k, 0, INIT)
        for (uint32_t d = lane; d < D; d += 64u) {
            const uint4 w = philox(d, k, 0u, DOM_INIT << 28, a.key0, a.key1);
            rep32[d] = mulhi32(w.x, a.q) | (mulhi32(w.y, a.q) << 8) | (mulhi32(w.z, a.q) << 16) |
                       (mulhi32(w.w, a.q) << 24);
        }
    } else {
        // eq. (6): all spins alpha, alpha uniform over the q states
        const uint4 w = philox(0u, k, 0u, DOM_GROUND << 28, a.key0, a.key1);
        const uint32_t alpha = mulhi32(w.x, a.q) * 0x01010101u;
        for (uint32_t d = lane; d < D; d += 64u) rep32[d] = alpha;
    }
    wave_fence();

    const uint32_t theta = a.mode == SWEEP_UPDATE ? a.theta : 0u;
    const uint32_t half = L >> 1, qm1 = a.q - 1u;
    for (uint32_t t = 0; t < theta; ++t) {
        for (uint32_t c = 0; c < 2u; ++c) {
            const uint32_t c3 = (DOM_SWEEP << 28) | (t << 1) | c;
            for (uint32_t p = lane; p < D; p += 64u) {     // N/4 pairs of colour-c sites
                const uint4 w = philox(p, k, a.step, c3, a.key0, a.key1);
#pragma unroll
                for (uint32_t h = 0; h < 2u; ++h) {
                    const uint32_t m = 2u * p + h;
                    const uint32_t y = m / half;
                    const uint32_t x = 2u * (m - y * half) + ((y + c) & 1u);
                    byte_site_update(rep, L, y, x, h ? w.z : w.x, h ? w.w : w.y, qm1, a);
                }
            }
            wave_fence();
        }
    }

    // energy (eq. (3)): bonds to the right and down neighbours
    uint32_t bonds = 0;
    for (uint32_t n = lane; n < N; n += 64u) {
        const uint32_t y = n / L, x = n - y * L;
        const uint32_t sv = rep[n];
        bonds += (sv == rep[y * L + wrap_next(x, L)]) + (sv == rep[wrap_next(y, L) * L + x]);
    }
    bonds = wave_total(bonds);
    // magnetisation (eq. (5)): the largest number of sites in one state
    uint32_t mt = 0;
    if (a.Mt_out) {
        for (uint32_t st = 0; st < a.q; ++st) {
            uint32_t cnt = 0;
            for (uint32_t n = lane; n < N; n += 64u) cnt += rep[n] == st ? 1u : 0u;
            mt = max(mt, wave_total(cnt));
        }
    }
    uint64_t dig = 0;
    if (a.H_out) {
        for (uint32_t d = lane; d < D; d += 64u) dig += digest_term(d, k, a.step, rep32[d], a.key0, a.key1);
        for (uint32_t off = 32; off > 0; off >>= 1) dig += __shfl_xor(dig, off, 64);
    }
    if (lane == 0) {
        a.E_out[k] = -(int32_t)bonds;
        if (a.Mt_out) a.Mt_out[k] = mt;
        if (a.H_out) a.H_out[k] = dig;
    }
    uint32_t *dst = reinterpret_cast<uint32_t *>(a.new_pop + (size_t)k * N);
    for (uint32_t d = lane; d < D; d += 64u) dst[d] = rep32[d];
}

__global__ void __launch_bounds__(256) k_sweep_bytes(SweepArgs a) { sweep_bytes_body(a, blockIdx.x); }

__global__ void __launch_bounds__(256) k_sweep_bytes_batch(const SweepArgs *runs, const uint32_t *start,
                                                           uint32_t n) {
    const uint32_t r = segment_of(start, n, blockIdx.x);
    sweep_bytes_body(runs[r], blockIdx.x - start[r]);
}

// ---------------------------------------------------------------------------
// Workgroup helpers (1024 threads = 16 waves).  k_post and k_countfill, the
// kernels they serve, always run workgroups of WG_THREADS, so the per-wave
// partials are combined in unrolled loops whose LDS reads issue together.
// ---------------------------------------------------------------------------
constexpr uint32_t WG_THREADS = 1024, WG_WAVES = WG_THREADS / 64;

// Lane moves of a 4- or 8-byte value: DPP pattern CTRL, and one lane's value.
template <uint32_t CTRL, typename T>
__device__ __forceinline__ T dpp_move(T v) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
    } else {
        static_assert(sizeof(T) == 8, "4- or 8-byte values");
        const uint64_t u = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, false);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
        return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
    }
}
template <typename T>
__device__ __forceinline__ T lane_value(T v, int lane) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
    } else {
        const uint64_t u = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
        return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
    }
}

// op over the 64 lanes of a wave (all active; op commutative and
// associative, or, for a floating-point sum, rounded in this fixed order),
// wave-uniform: the DPP steps of wave_total, then the four row results read
// from lanes 0, 16, 32 and 48.  No lane addresses, unlike ds_bpermute
// shuffles.
template <typename T, typename Op>
__device__ __forceinline__ T wave_allreduce(T v, Op op) {
    v = op(v, dpp_move<0xB1>(v));
    v = op(v, dpp_move<0x4E>(v));
    v = op(v, dpp_move<0x124>(v));
    v = op(v, dpp_move<0x128>(v));
    return op(op(lane_value(v, 0), lane_value(v, 16)), op(lane_value(v, 32), lane_value(v, 48)));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Inclusive scan over the 64 lanes of a wave (all active), by DPP: shifts
// right by 1, 2, 4 and 8 lanes within each row of 16 (zero entering), then
// the last lane of row 0 and 2 added to rows 1 and 3 (row_bcast:15) and that
// of row 1 to rows 2 and 3 (row_bcast:31).
template <uint32_t CTRL, uint32_t ROWS, typename T>
__device__ __forceinline__ T dpp_or_zero(T v) {
    if constexpr (sizeof(T) == 4) {
        return (T)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, false);
    } else {
        const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, ROWS, 0xF, false);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, ROWS, 0xF, false);
        return (T)(((uint64_t)hi << 32) | lo);
    }
}
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "4- or 8-byte integers");
    v += dpp_or_zero<0x111, 0xF>(v);   // row_shr:1
    v += dpp_or_zero<0x112, 0xF>(v);   // row_shr:2
    v += dpp_or_zero<0x114, 0xF>(v);   // row_shr:4
    v += dpp_or_zero<0x118, 0xF>(v);   // row_shr:8
    v += dpp_or_zero<0x142, 0xA>(v);   // row_bcast:15 into rows 1, 3
    v += dpp_or_zero<0x143, 0xC>(v);   // row_bcast:31 into rows 2, 3
    return v;
}

// Loops over the 16 wave partials of a workgroup: unrolled, so that their LDS
// reads issue together, or (LEAN) rolled, holding one partial at a time, for
// kernels that must keep few registers.  The results are the same.
template <bool LEAN>
__device__ __forceinline__ uint32_t wave_partials() {
    return LEAN ? (blockDim.x >> 6) : WG_WAVES;
}

// Exclusive offset of this wave's total among the waves of the block (in wave
// order); *total receives the block sum.  scratch holds blockDim/64 entries.
template <bool LEAN = false, typename T>
__device__ __forceinline__ T block_wave_offset(T wave_total, T *scratch, T *total) {
    const uint32_t wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63u) == 0) scratch[wave] = wave_total;
    __syncthreads();
    T off = T(0), tot = T(0);
    const uint32_t nw = wave_partials<LEAN>();
#pragma unroll
    for (uint32_t w = 0; w < nw; ++w) {
        const T x = scratch[w];
        off += w < wave ? x : T(0);
        tot += x;
    }
    *total = tot;
    __syncthreads();
    return off;
}

// Block-wide reduction with `op`; every thread receives the result.
// scratch holds blockDim/64 entries.
template <bool LEAN = false, typename T, typename Op>
__device__ __forceinline__ T block_reduce(T v, Op op, T *scratch) {
    v = wave_allreduce(v, op);
    __syncthreads();
    if ((threadIdx.x & 63u) == 0) scratch[threadIdx.x >> 6] = v;
    __syncthreads();
    T r = scratch[0];
    const uint32_t nw = wave_partials<LEAN>();
#pragma unroll
    for (uint32_t w = 1; w < nw; ++w) r = op(r, scratch[w]);
    return r;
}

// A histogram over levels 0..nb-1 of which only the window lo .. lo+n-1 is
// stored (h[b - lo]); every other level holds zero.
struct HistView {
    const uint32_t *h;
    uint32_t lo, n, nb;
    __device__ __forceinline__ uint32_t at(int64_t b) const {
        return (b >= (int64_t)lo && b < (int64_t)lo + n) ? h[b - lo] : 0u;
    }
};

// Count of bin j (levels j*B .. j*B+B-1); zero outside 0..nc-1.
__device__ __forceinline__ uint64_t bin_count(const HistView &v, uint32_t B, int64_t j) {
    const int64_t nc = ((int64_t)v.nb + B - 1) / B;
    if (j < 0 || j >= nc) return 0;
    const int64_t b0 = j * B, b1 = min(b0 + (int64_t)B, (int64_t)v.nb);
    uint64_t c = 0;
    for (int64_t b = max(b0, (int64_t)v.lo); b < min(b1, (int64_t)v.lo + v.n); ++b) c += v.h[b - v.lo];
    return c;
}

// Integer part of the full width at half maximum (Sec. 4) of the histogram in
// bins of B levels: H, the largest bin count; jl and jr, the outermost bins
// whose count reaches H/2 (2 count >= H); and the counts of bins jl-1, jl, jr
// and jr+1 (zero outside the histogram).  The width is the distance between
// the crossings of H/2 of the straight lines through those counts at the bin
// indices; that interpolation runs on the host.  Whole workgroup; thread 0
// stores out[0..7) = H, jl, jr, h(jl-1), h(jl), h(jr), h(jr+1) (all zero for
// an empty histogram).
template <bool LEAN = false>
__device__ void hist_fwhm_ints(const HistView &v, uint32_t B, uint64_t *scratch, uint64_t *out) {
    const uint32_t j_lo = v.lo / B, j_hi = (v.lo + v.n - 1) / B;   // bins that meet the window
    uint64_t H = 0;
    for (uint32_t j = j_lo + threadIdx.x; j <= j_hi; j += blockDim.x) H = max(H, bin_count(v, B, j));
    H = block_reduce<LEAN>(H, [](uint64_t x, uint64_t y) { return x > y ? x : y; }, scratch);
    uint64_t jl = ~0ull, jr = 0;
    for (uint32_t j = j_lo + threadIdx.x; j <= j_hi; j += blockDim.x)
        if (H && 2 * bin_count(v, B, j) >= H) { jl = min(jl, (uint64_t)j); jr = max(jr, (uint64_t)j); }
    jl = block_reduce<LEAN>(jl, [](uint64_t x, uint64_t y) { return x < y ? x : y; }, scratch);
    jr = block_reduce<LEAN>(jr, [](uint64_t x, uint64_t y) { return x > y ? x : y; }, scratch);
    if (threadIdx.x != 0) return;
    if (H == 0) {
        for (int k = 0; k < 7; ++k) out[k] = 0;
        return;
    }
    out[0] = H;
    out[1] = jl;
    out[2] = jr;
    out[3] = bin_count(v, B, (int64_t)jl - 1);
    out[4] = bin_count(v, B, (int64_t)jl);
    out[5] = bin_count(v, B, (int64_t)jr);
    out[6] = bin_count(v, B, (int64_t)jr + 1);
}

// Calls f(x[j]) for j = 0 .. n-1 (4-byte elements, 16-byte aligned array), in
// no particular order, in tiles of blockDim * V elements (V = 32 unless
// given): each thread issues its V/4 128-bit loads of a tile together, and
// each load of a wave covers 1 KB of consecutive elements.  A partial last
// tile keeps that layout, each 128-bit load bounded on its own, so that it
// costs one memory latency like a full one (with V = 32 a population of up to
// 32768 replicas is read in one round by 1024 threads).
template <uint32_t V = 32, typename T, typename F>
__device__ __forceinline__ void for_each_tiled(const T *x, uint64_t n, F f) {
    static_assert(sizeof(T) == 4, "4-byte elements");
    static_assert(V % 4 == 0, "whole 16-byte loads");
    const uint32_t tile = blockDim.x * V;
    uint64_t base = 0;
    // whole tiles: every load unconditional
    for (; base + tile <= n; base += tile) {
        const uint4 *src = reinterpret_cast<const uint4 *>(x + base) + threadIdx.x;
        T v[V];
#pragma unroll
        for (uint32_t q = 0; q < V / 4; ++q) {
            const uint4 w = src[q * blockDim.x];
            v[4 * q] = (T)w.x; v[4 * q + 1] = (T)w.y; v[4 * q + 2] = (T)w.z; v[4 * q + 3] = (T)w.w;
        }
#pragma unroll
        for (uint32_t q = 0; q < V; ++q) f(v[q]);
    }
    if (base < n) {
        const T *xb = x + base;
        T v[V];
        // element 4 (q blockDim + t) + r of the tile: row q, thread t
        const uint32_t left = (uint32_t)(n - base);
        const uint32_t m4 = left & ~3u;
        bool ok[V / 4];
#pragma unroll
        for (uint32_t q = 0; q < V / 4; ++q) {
            const uint32_t o = 4u * (q * blockDim.x + threadIdx.x);
            ok[q] = o < m4;
            if (ok[q]) {
                const uint4 w = *reinterpret_cast<const uint4 *>(xb + o);
                v[4 * q] = (T)w.x; v[4 * q + 1] = (T)w.y; v[4 * q + 2] = (T)w.z; v[4 * q + 3] = (T)w.w;
            }
        }
        // the last tile's final left mod 4 elements, one by one
        if (threadIdx.x < left - m4) f(xb[m4 + threadIdx.x]);
#pragma unroll
        for (uint32_t q = 0; q < V / 4; ++q)
            if (ok[q]) {
#pragma unroll
                for (uint32_t r = 0; r < 4; ++r) f(v[4 * q + r]);
            }
    }
}

// Sum, minimum and maximum over the workgroup; every thread receives them.
struct SumMinMax { int64_t sum; int32_t mn, mx; };

template <bool LEAN = false>
__device__ SumMinMax block_sum_min_max(int64_t sum, int32_t mn, int32_t mx) {
    __shared__ int64_t s_sum[WG_WAVES];
    __shared__ int32_t s_mn[WG_WAVES], s_mx[WG_WAVES];
    sum = wave_allreduce(sum, [](int64_t x, int64_t y) { return x + y; });
    mn = wave_allreduce(mn, [](int32_t x, int32_t y) { return min(x, y); });
    mx = wave_allreduce(mx, [](int32_t x, int32_t y) { return max(x, y); });
    __syncthreads();
    if ((threadIdx.x & 63u) == 0) { s_sum[threadIdx.x >> 6] = sum; s_mn[threadIdx.x >> 6] = mn; s_mx[threadIdx.x >> 6] = mx; }
    __syncthreads();
    SumMinMax r{s_sum[0], s_mn[0], s_mx[0]};
    const uint32_t nw = wave_partials<LEAN>();
#pragma unroll
    for (uint32_t w = 1; w < nw; ++w) {
        r.sum += s_sum[w]; r.mn = min(r.mn, s_mn[w]); r.mx = max(r.mx, s_mx[w]);
    }
    return r;
}

// Histogram of the n values x[j] + shift (each in 0 .. nb-1) by the whole
// workgroup, with their sum and range.  If all nb levels fit the LDS array
// lds[cap], the values are counted there directly; otherwise a first pass
// finds their range and, if that fits, the window min .. max is counted in
// LDS; failing both, out[0..nb) in global memory is zeroed and counted with
// atomics.  sum (of x, not shifted), mn and mx are valid in every thread.
struct HistBuild { HistView v; int64_t sum; int32_t mn, mx; };

template <uint32_t V = 32, bool LEAN = false, typename T>
__device__ HistBuild build_hist(const T *x, uint64_t n, int32_t shift, uint32_t nb, uint32_t *lds,
                                uint32_t cap, uint32_t *out) {
    HistBuild r;
    if (nb <= cap) {
        // C interleaved copies of every level (lds[level * C + c], the lane
        // picking c), C = 8, 4, 2 or 1 as they fit beside the folded counts
        // at lds[nb * C ..]: a population concentrated on a few energies
        // sends many lanes of a wave to the same level, and LDS atomics on
        // one address serialise.
        const uint32_t C = nb * 9u <= cap ? 8u : nb * 5u <= cap ? 4u : nb * 3u <= cap ? 2u : 1u;
        uint32_t *folded = C > 1u ? lds + nb * C : lds;
        const uint32_t nz = nb * C;
        for (uint32_t b = threadIdx.x; b < nz / 4u; b += blockDim.x)
            reinterpret_cast<uint4 *>(lds)[b] = make_uint4(0u, 0u, 0u, 0u);
        if (threadIdx.x < nz % 4u) lds[nz - 1u - threadIdx.x] = 0u;
        __syncthreads();
        const uint32_t c = threadIdx.x & (C - 1u);
        for_each_tiled<V>(x, n, [&](T e) { atomicAdd(&lds[(uint32_t)((int32_t)e + shift) * C + c], 1u); });
        __syncthreads();
        int64_t sum = 0;
        int32_t mn = 0x7fffffff, mx = (int32_t)0x80000000;
        for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) {
            uint32_t h = 0;
            for (uint32_t k = 0; k < C; ++k) h += lds[b * C + k];
            if (C > 1u) folded[b] = h;
            if (h) {
                const int32_t e = (int32_t)b - shift;
                sum += (int64_t)h * e; mn = min(mn, e); mx = max(mx, e);
            }
        }
        const SumMinMax t = block_sum_min_max<LEAN>(sum, mn, mx);   // synchronises the workgroup first
        r.sum = t.sum; r.mn = t.mn; r.mx = t.mx;
        r.v = HistView{folded, 0u, nb, nb};
        return r;
    }
    int64_t sum = 0;
    int32_t mn = 0x7fffffff, mx = (int32_t)0x80000000;
    for_each_tiled<V>(x, n, [&](T v) { const int32_t e = (int32_t)v; sum += e; mn = min(mn, e); mx = max(mx, e); });
    const SumMinMax t = block_sum_min_max<LEAN>(sum, mn, mx);
    r.sum = t.sum; r.mn = t.mn; r.mx = t.mx;
    const uint32_t lo = (uint32_t)(r.mn + shift), width = (uint32_t)(r.mx - r.mn) + 1u;
    if (width <= cap) {
        for (uint32_t b = threadIdx.x; b < width; b += blockDim.x) lds[b] = 0u;
        __syncthreads();
        for_each_tiled<V>(x, n, [&](T e) { atomicAdd(&lds[(uint32_t)((int32_t)e + shift) - lo], 1u); });
        __syncthreads();
        r.v = HistView{lds, lo, width, nb};
    } else {
        for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) out[b] = 0u;
        __threadfence();
        __syncthreads();
        for_each_tiled<V>(x, n, [&](T e) { atomicAdd(&out[(uint32_t)((int32_t)e + shift)], 1u); });
        __threadfence();
        __syncthreads();
        r.v = HistView{out, 0u, nb, nb};
    }
    return r;
}

// Writes the full histogram (zeros outside the window) to out[0..nb), unless
// it was built there.
__device__ void store_hist(const HistView &v, uint32_t *out) {
    if (v.h == out) return;
    for (uint32_t b = threadIdx.x; b < v.nb; b += blockDim.x) out[b] = v.at(b);
}

constexpr uint32_t POST_LDS_BINS = 14336;   // 56 KB window for the histograms in LDS

constexpr uint32_t SHORT_RUN = 8;   // copies written by their own lane in the slot map

// Multi-workgroup scans: workgroup b of a launch takes the elements
// [b*block, (b+1)*block) in rows of blockDim*4, thread t the four elements
// 4t .. 4t+3 of each row, so that every load and store of a wave covers
// consecutive memory.  The sum over the elements before the block is
// recomputed by each workgroup from the inputs, so that the workgroups need
// no communication.

// C_j = sum_{j' <= j} wf(E_j') for first <= j < last (E 16-byte aligned, C
// 32-byte aligned, first a multiple of 4).
template <typename WF>
__device__ __forceinline__ void weight_block(const int32_t *E, uint32_t first, uint32_t last, WF wf,
                                             uint64_t *C, uint64_t *scratch) {
    uint64_t carry = 0;
    for_each_tiled(E, first, [&](int32_t e) { carry += wf(e); });
    carry = block_reduce(carry, [](uint64_t x, uint64_t y) { return x + y; }, scratch);
    __syncthreads();
    for (uint32_t base = first; base < last; base += blockDim.x * 4u) {
        const uint32_t j = base + threadIdx.x * 4u;
        uint64_t w[4];
        if (j + 4u <= last) {
            const int4 x = *reinterpret_cast<const int4 *>(E + j);
            w[0] = wf(x.x); w[1] = wf(x.y); w[2] = wf(x.z); w[3] = wf(x.w);
        } else {
#pragma unroll
            for (uint32_t v = 0; v < 4; ++v) w[v] = j + v < last ? wf(E[j + v]) : 0ull;
        }
        w[1] += w[0]; w[2] += w[1]; w[3] += w[2];
        const uint64_t incl = wave_inclusive_scan(w[3]);
        uint64_t total;
        const uint64_t off = carry + block_wave_offset(lane_value(incl, 63), scratch, &total) + incl - w[3];
#pragma unroll
        for (uint32_t v = 0; v < 4; ++v) w[v] += off;
        if (j + 4u <= last) {
            ulonglong2 *dst = reinterpret_cast<ulonglong2 *>(C + j);
            dst[0] = make_ulonglong2(w[0], w[1]);
            dst[1] = make_ulonglong2(w[2], w[3]);
        } else {
#pragma unroll
            for (uint32_t v = 0; v < 4; ++v)
                if (j + v < last) C[j + v] = w[v];
        }
        carry += total;
    }
}

// ---------------------------------------------------------------------------
// k_post(i), workgroup 0: the exact integer sums behind the population
// averages of eq. (4) and ln Q_{i+1} of Sec. 2 step 2 / eq. (2) from the energy
// histogram of step i, the magnetisation sum, the integer part of the widths
// and the digest (the averages and the widths themselves are formed on the
// host; FP64 on the device is the ln Q / -beta F chain only).  Workgroups 1, 2, ...: if resampling follows, the integer
// weights W(|E_j - E_ref|) of step i+1 and their inclusive scan C, one block
// of replicas each.
// ---------------------------------------------------------------------------
// V: values per thread and load round of the population passes (the team
// kernel's smaller populations take fewer, and fewer registers).
template <uint32_t V = 32, bool LEAN = false>
__device__ __forceinline__ void post_stats(const PostArgs &a, uint32_t *lds_hist, uint64_t *scratch,
                                           uint32_t lds_cap = POST_LDS_BINS) {
    __shared__ double s_w[WG_WAVES];
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint32_t nb = a.nbins;
    // -beta F of step i, read first: the ln Q_{i+1} chain of thread 0 below
    // would otherwise wait a memory latency for it
    const double mbF_i = (tid == 0 && a.has_next) ? a.mbF[a.step] : 0.0;

    // eq. (4) sums and the energy histogram h[E + 2N] of step i
    const HistBuild he = build_hist<V, LEAN>(a.E, a.R_i, a.two_n, nb, lds_hist, lds_cap, a.hist);
    const int32_t ref = a.dbeta_next >= 0.0 ? he.mn : he.mx;   // E_ref of step i+1
    if (tid == 0) {
        a.E_sum[a.step] = he.sum;
        if (a.has_next) a.E_ref[a.step + 1] = ref;
    }
    // ln Q_{i+1} (Sec. 2 step 2, eq. (2)) from the histogram, and its count
    uint64_t cnt = 0;
    double acc = 0.0;
    for (uint32_t b = tid; b < he.v.n; b += blockDim.x) {
        const uint32_t h = he.v.h[b];
        cnt += h;
        if (a.has_next && h)
            acc += (double)h * exp(-(a.abs_dbeta_next * (double)abs((int32_t)(b + he.v.lo) - a.two_n - ref)));
    }
    acc = wave_allreduce(acc, [](double x, double y) { return x + y; });
    cnt = wave_allreduce(cnt, [](uint64_t x, uint64_t y) { return x + y; });
    if (lane == 0) { s_w[wave] = acc; scratch[wave] = cnt; }
    __syncthreads();
    if (tid == 0) {
        double S = 0.0;
        uint64_t C = 0;
        const uint32_t nw = wave_partials<LEAN>();
#pragma unroll
        for (uint32_t w = 0; w < nw; ++w) { S += s_w[w]; C += scratch[w]; }
        a.count[a.step] = C;
        if (a.has_next) {
            const double lnq = -a.dbeta_next * (double)ref + log(S) - log((double)a.R_i);
            a.lnQ[a.step + 1] = lnq;
            a.mbF[a.step + 1] = mbF_i + lnq;
        }
    }
    __syncthreads();
    if (a.store_hist) store_hist(he.v, a.hist);
    if (a.widths) hist_fwhm_ints<LEAN>(he.v, a.bin_e, scratch, a.fw_e + 8 * (size_t)a.step);
    __syncthreads();

    if (a.H) {
        // digest of the population: the sum of the replicas' terms
        uint64_t dsum = 0;
        for (uint64_t j = tid; j < a.R_i; j += blockDim.x) dsum += a.H[j];
        dsum = block_reduce<LEAN>(dsum, [](uint64_t x, uint64_t y) { return x + y; }, scratch);
        if (tid == 0) a.digest[a.step] = dsum;
        __syncthreads();
    }
    if (a.Mt) {
        // eq. (4)-(5): sum of M~ over the population, M-bar, the M~ histogram
        const HistBuild hm = build_hist<V, LEAN>(a.Mt, a.R_i, 0, a.N + 1, lds_hist, lds_cap, a.mhist);
        if (tid == 0) a.Mt_sum[a.step] = hm.sum;
        if (a.store_hist) store_hist(hm.v, a.mhist);
        if (a.widths) hist_fwhm_ints<LEAN>(hm.v, a.bin_m, scratch, a.fw_m + 8 * (size_t)a.step);
        __syncthreads();
    }

}

// A population of at most 32 blockDim 4-byte values held in registers, in
// the tile layout of for_each_tiled: row q, thread t holds the cnt(q) values
// 4 (q blockDim + t) + r, r < cnt(q) (4 for a whole row).  One round of
// 128-bit loads; the last n mod 4 values are read by the thread whose row
// position they fill.
struct TileRegs {
    static constexpr uint32_t Q = 8;
    int32_t v[4 * Q];
    uint32_t m4, rem, qr;   // n rounded down to a multiple of 4, n mod 4, the row holding m4
    bool own;               // this thread holds the last rem values (in row qr)

    __device__ __forceinline__ uint32_t cnt(uint32_t q) const {
        return 4u * (q * blockDim.x + threadIdx.x) < m4 ? 4u : (own && q == qr ? rem : 0u);
    }
    __device__ __forceinline__ void load(const int32_t *x, uint32_t n) {
        const uint32_t row = 4u * blockDim.x;
        m4 = n & ~3u; rem = n - m4; qr = m4 / row;
        own = rem != 0u && threadIdx.x == (m4 % row) / 4u;
        int32_t er[3] = {0, 0, 0};
        if (own) {
#pragma unroll
            for (uint32_t r = 0; r < 3; ++r) if (r < rem) er[r] = x[m4 + r];
        }
#pragma unroll
        for (uint32_t q = 0; q < Q; ++q) {
            const uint32_t o = 4u * (q * blockDim.x + threadIdx.x);
            if (o < m4) {
                const int4 w = *reinterpret_cast<const int4 *>(x + o);
                v[4 * q] = w.x; v[4 * q + 1] = w.y; v[4 * q + 2] = w.z; v[4 * q + 3] = w.w;
            } else {
                v[4 * q] = er[0]; v[4 * q + 1] = er[1]; v[4 * q + 2] = er[2]; v[4 * q + 3] = 0;
            }
        }
    }
    template <typename F>
    __device__ __forceinline__ void each(F f) const {
#pragma unroll
        for (uint32_t q = 0; q < Q; ++q) {
            const uint32_t c = cnt(q);
#pragma unroll
            for (uint32_t r = 0; r < 4; ++r)
                if (r < c) f(v[4 * q + r]);
        }
    }
};

// weight_block for a population held in TileRegs whose blocks are its rows
// (block b = row b, first = 4 b blockDim): the carry sums the rows before b,
// and row b is scanned and stored as C.
template <typename WF>
__device__ __forceinline__ void weight_row_regs(const TileRegs &tr, uint32_t b, WF wf, uint64_t *C,
                                                uint64_t *scratch) {
    uint64_t carry = 0;
    int32_t e[4] = {0, 0, 0, 0};
    uint32_t c = 0;
#pragma unroll
    for (uint32_t q = 0; q < TileRegs::Q; ++q) {
        if (q < b) {
            const uint32_t cq = tr.cnt(q);
#pragma unroll
            for (uint32_t r = 0; r < 4; ++r) carry += r < cq ? wf(tr.v[4 * q + r]) : 0ull;
        }
        if (q == b) {
            e[0] = tr.v[4 * q]; e[1] = tr.v[4 * q + 1]; e[2] = tr.v[4 * q + 2]; e[3] = tr.v[4 * q + 3];
            c = tr.cnt(q);
        }
    }
    carry = block_reduce(carry, [](uint64_t x, uint64_t y) { return x + y; }, scratch);
    __syncthreads();
    uint64_t w[4];
#pragma unroll
    for (uint32_t r = 0; r < 4; ++r) w[r] = r < c ? wf(e[r]) : 0ull;
    w[1] += w[0]; w[2] += w[1]; w[3] += w[2];
    const uint64_t incl = wave_inclusive_scan(w[3]);
    uint64_t total;
    const uint64_t off = carry + block_wave_offset(lane_value(incl, 63), scratch, &total) + incl - w[3];
#pragma unroll
    for (uint32_t r = 0; r < 4; ++r) w[r] += off;
    const uint32_t j = 4u * (b * blockDim.x + threadIdx.x);
    if (c == 4u) {
        ulonglong2 *dst = reinterpret_cast<ulonglong2 *>(C + j);
        dst[0] = make_ulonglong2(w[0], w[1]);
        dst[1] = make_ulonglong2(w[2], w[3]);
    } else {
#pragma unroll
        for (uint32_t r = 0; r < 4; ++r)
            if (r < c) C[j + r] = w[r];
    }
}

// Weight workgroup b: E_ref of step i+1 (the minimum or maximum energy of the
// population, as the statistics workgroup finds it) and C over block b.  The
// distances that occur are 0 .. max - min; their weights are read from LDS
// when they fit there.  A population of at most 32 blockDim replicas in
// blocks of one row each (R_i <= 32768 with 1024 threads) is read once, into
// registers, for the range, the carry and the block.
__device__ __forceinline__ void post_weights(const PostArgs &a, uint32_t b, uint32_t *lds, uint64_t *scratch) {
    const uint32_t n = (uint32_t)a.R_i, tid = threadIdx.x;
    const uint32_t first = b * a.wblock, last = min(first + a.wblock, n);
    const bool in_regs = n <= 32u * blockDim.x && a.wblock == 4u * blockDim.x;
    TileRegs tr;
    int32_t mn = 0x7fffffff, mx = (int32_t)0x80000000;
    const auto range = [&](int32_t e) { mn = min(mn, e); mx = max(mx, e); };
    if (in_regs) {
        tr.load(a.E, n);
        tr.each(range);
    } else {
        for_each_tiled(a.E, n, range);
    }
    const SumMinMax t = block_sum_min_max(0, mn, mx);
    const int32_t ref = a.dbeta_next >= 0.0 ? t.mn : t.mx;
    const auto weights = [&](auto wf) {
        if (in_regs) weight_row_regs(tr, b, wf, a.C, scratch);
        else weight_block(a.E, first, last, wf, a.C, scratch);
    };
    if (a.w_const) {
        const uint64_t wc = a.w_const;
        weights([=](int32_t) { return wc; });
        return;
    }
    const uint32_t span = (uint32_t)(t.mx - t.mn) + 1u;
    const uint32_t nW = a.D < span ? a.D : span;
    if (nW <= POST_LDS_BINS / 2) {
        uint64_t *Wl = reinterpret_cast<uint64_t *>(lds);
        for (uint32_t d = tid; d < nW; d += blockDim.x) Wl[d] = a.W[d];
        __syncthreads();
        weights([=](int32_t e) {
            const uint32_t d = (uint32_t)abs(e - ref);
            return d < nW ? Wl[d] : 0ull;
        });
    } else {
        const uint64_t *Wg = a.W;
        const uint32_t D = a.D;
        weights([=](int32_t e) {
            const uint32_t d = (uint32_t)abs(e - ref);
            return d < D ? Wg[d] : 0ull;
        });
    }
}

__device__ __forceinline__ void small_resample_body(const SmallResample &st, uint32_t *ancL, uint32_t *ru,
                                                    uint64_t *C, uint64_t *scratch, bool write_out);

__device__ __forceinline__ void post_block(const PostArgs &a, uint32_t b) {
    __shared__ __align__(16) uint32_t lds[POST_LDS_BINS];
    __shared__ uint64_t scratch[17];
    if (b == 0) {
        post_stats(a, lds, scratch);
    } else if (a.small) {
        // the whole resampling into step i+1 (R_prev <= SMALL_RESAMPLE_MAX:
        // counts and cumulative weights take 12 bytes per replica of LDS)
        uint64_t *C = reinterpret_cast<uint64_t *>(lds + ((a.rs.R_prev + 3u) & ~uint64_t(3)));
        // (inlined: the record stays in the kernel arguments)
        small_resample_body(a.rs, nullptr, lds, C, scratch, true);
    } else {
        post_weights(a, b - 1, lds, scratch);
    }
}

__global__ void __launch_bounds__(WG_THREADS) k_post(PostArgs a) { post_block(a, blockIdx.x); }

// Batched form: run r owns workgroups start[r] .. start[r+1]-1.
__global__ void __launch_bounds__(WG_THREADS) k_post_batch(const PostArgs *runs, const uint32_t *start, uint32_t n) {
    const uint32_t r = segment_of(start, n, blockIdx.x);
    const PostArgs a = runs[r];
    post_block(a, blockIdx.x - start[r]);
}

// ---------------------------------------------------------------------------
// Count scan and slot map, workgroup b of the launch: o = exclusive scan of the
// copy numbers r; anc[o_j + c] = j for c < r_j (new population in ancestor
// order, eq. (1)) for the ancestors j of block b; the other parity's counts
// are cleared for the next step.
// ---------------------------------------------------------------------------
__device__ void countfill_block(const SlotmapArgs &a, uint32_t b, uint64_t *scratch) {
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const uint32_t n = (uint32_t)a.R_prev;   // R_prev < 2^32
    const uint32_t first = b * a.block, last = min(first + a.block, n);
    const uint64_t stride = (uint64_t)countfill_blocks(a) * a.block;
    // (c0 is a multiple of the block, 4096, and r_clear 16-byte aligned)
    for (uint64_t c0 = first; c0 < a.clear_n; c0 += stride) {
        const uint64_t c1 = min(c0 + a.block, a.clear_n), n4 = (c1 - c0) / 4u;
        for (uint64_t i = tid; i < n4; i += blockDim.x)
            reinterpret_cast<uint4 *>(a.r_clear + c0)[i] = make_uint4(0u, 0u, 0u, 0u);
        if (tid < (c1 - c0) % 4u) a.r_clear[c1 - 1u - tid] = 0u;
    }
    // the block's rows do not depend on the sum before it: the first row's
    // counts are loaded before that sum, so that the two reads overlap
    auto load_row = [&](uint32_t j, uint32_t r[4]) {
        if (j + 4u <= last) {
            const uint4 x = *reinterpret_cast<const uint4 *>(a.r + j);
            r[0] = x.x; r[1] = x.y; r[2] = x.z; r[3] = x.w;
        } else {
#pragma unroll
            for (uint32_t v = 0; v < 4; ++v) r[v] = j + v < last ? a.r[j + v] : 0u;
        }
    };
    uint32_t r[4];
    load_row(first + tid * 4u, r);
    uint64_t carry = 0;
    // (tiles of 16 per thread: the counts were just written by atomics, and
    // the deeper tiles of 32 measured slower here, 6.7 against 5.9 us at
    // R = 2e4 and 123 against 115 us at R = 2e5)
    for_each_tiled<16>(a.r, first, [&](uint32_t c) { carry += c; });
    carry = block_reduce(carry, [](uint64_t x, uint64_t y) { return x + y; }, scratch);
    __syncthreads();
    for (uint32_t base = first; base < last; base += blockDim.x * 4u) {
        const uint32_t j = base + tid * 4u;
        if (base != first) load_row(j, r);
        // offsets within the row in 32 bits (a row's counts sum to at most the
        // new population, below 2^32)
        const uint32_t sum = r[0] + r[1] + r[2] + r[3];
        const uint32_t incl = wave_inclusive_scan(sum);
        uint32_t total;
        const uint32_t woff = block_wave_offset(lane_value(incl, 63), reinterpret_cast<uint32_t *>(scratch), &total);
        const uint64_t o0 = carry + woff + incl - sum;
        // Short runs of copies are written by their own lane, long ones
        // (strongly skewed weights) by the whole wave.
        uint64_t o = o0;
#pragma unroll
        for (uint32_t v = 0; v < 4; ++v) {
            if (r[v] <= SHORT_RUN)
                for (uint32_t c = 0; c < r[v]; ++c)
                    if (o + c < a.anc_cap) a.anc[o + c] = j + v;
            o += r[v];
        }
        o = o0;
#pragma unroll
        for (uint32_t v = 0; v < 4; ++v) {
            uint64_t todo = __ballot(r[v] > SHORT_RUN);
            while (todo) {
                const uint32_t src = (uint32_t)__ffsll((unsigned long long)todo) - 1u;
                const uint64_t start = ((uint64_t)__shfl((uint32_t)(o >> 32), src, 64) << 32) |
                                       (uint64_t)__shfl((uint32_t)o, src, 64);
                const uint32_t cnt = __shfl(r[v], src, 64);
                const uint32_t who = __shfl(j + v, src, 64);
                for (uint32_t c = lane; c < cnt; c += 64u)
                    if (start + c < a.anc_cap) a.anc[start + c] = who;
                todo &= todo - 1;
            }
            o += r[v];
        }
        if (j + 4u <= last) {
            *reinterpret_cast<uint4 *>(a.counts_last + j) = make_uint4(r[0], r[1], r[2], r[3]);
        } else {
#pragma unroll
            for (uint32_t v = 0; v < 4; ++v)
                if (j + v < last) a.counts_last[j + v] = r[v];
        }
        carry += total;
    }
}

// ---------------------------------------------------------------------------
// k_sample: draw kk picks the first j with C_j > floor(x_kk * S / 2^64) and
// counts it in r_j.
// ---------------------------------------------------------------------------
// Adds one to h[key] for every active lane; lanes of the wave that share the
// key of one of the first few leaders are combined into one atomic (strongly
// skewed weights send many draws of a wave to the same ancestor).
__device__ __forceinline__ void wave_aggregated_inc(uint32_t *h, uint32_t key, bool active) {
    uint64_t todo = __ballot(active);
    // at most four combining rounds (the dominant keys); the rest add one each
    for (int round = 0; round < 4 && todo; ++round) {
        const uint32_t src = (uint32_t)__ffsll((unsigned long long)todo) - 1u;
        const uint32_t k = __shfl(key, src, 64);
        const bool mine = active && key == k;
        const uint64_t same = __ballot(mine);
        if ((threadIdx.x & 63u) == src) atomicAdd(&h[k], (uint32_t)__popcll(same));
        todo &= ~same;
        active = active && !mine;
    }
    if (active) atomicAdd(&h[key], 1u);
}

constexpr uint64_t SAMPLE_WINDOW = 32;   // fastest of 32, 64, 128 at R = 2e4

__device__ __forceinline__ void sample_one(const SampleArgs &a, uint64_t kk) {
    const bool live = kk < a.n_new;
    uint32_t anc = 0;
    if (live) {
        const uint4 w = philox((uint32_t)kk, 0u, a.step, DOM_RESAMPLE << 28, a.key0, a.key1);
        const uint64_t x = ((uint64_t)w.y << 32) | (uint64_t)w.x;
        // The cumulative weights are close to linear in j unless the weights
        // are strongly skewed: the window of SAMPLE_WINDOW replicas either
        // side of x R / 2^64 holds the answer when C_{lo-1} <= u < C_hi, and
        // the search runs there; otherwise over all replicas.  Both ends and
        // S = C_{R-1} are read in one round (unconditionally, C_0 standing in
        // for C_{-1} = 0).
        const uint64_t n = a.R_prev, j0 = __umul64hi(x, n);
        const uint64_t wlo = j0 > SAMPLE_WINDOW ? j0 - SAMPLE_WINDOW : 0;
        const uint64_t whi = j0 + SAMPLE_WINDOW < n ? j0 + SAMPLE_WINDOW : n - 1;
        const uint64_t c_lo_read = a.C[wlo ? wlo - 1 : 0], c_hi = a.C[whi];
        const uint64_t S = a.C[n - 1];
        const uint64_t u = __umul64hi(x, S);
        const uint64_t c_lo = wlo ? c_lo_read : 0ull;
        const bool in_window = c_lo <= u && c_hi > u;
        uint64_t lo = in_window ? wlo : 0, hi = in_window ? whi : n - 1;
        while (lo < hi) {
            const uint64_t mid = lo + ((hi - lo) >> 1);
            if (a.C[mid] > u) hi = mid; else lo = mid + 1;
        }
        anc = (uint32_t)lo;
    }
    wave_aggregated_inc(a.r, anc, live);
}

__global__ void __launch_bounds__(256) k_sample(SampleArgs a) {
    sample_one(a, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Batched form: run r owns workgroups start[r] .. start[r+1]-1.
__global__ void __launch_bounds__(256) k_sample_batch(const SampleArgs *runs, const uint32_t *start,
                                                      uint32_t n) {
    const uint32_t r = segment_of(start, n, blockIdx.x);
    const SampleArgs a = runs[r];
    sample_one(a, (uint64_t)(blockIdx.x - start[r]) * blockDim.x + threadIdx.x);
}

__global__ void __launch_bounds__(WG_THREADS) k_countfill(SlotmapArgs m) {
    __shared__ uint64_t scratch[17];
    countfill_block(m, blockIdx.x, scratch);
}

// Batched form: run r owns workgroups start[r] .. start[r+1]-1.
__global__ void __launch_bounds__(WG_THREADS) k_countfill_batch(const SlotmapArgs *runs, const uint32_t *start,
                                                          uint32_t n) {
    __shared__ uint64_t scratch[17];
    const uint32_t r = segment_of(start, n, blockIdx.x);
    const SlotmapArgs m = runs[r];
    countfill_block(m, blockIdx.x - start[r], scratch);
}

__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Fills and copies of many small buffers in one launch: the workgroup takes
// chunk blockIdx.x - start[r] of record r.
__global__ void __launch_bounds__(256) k_prep_batch(const PrepRec *recs, const uint32_t *start, uint32_t n) {
    const uint32_t r = segment_of(start, n, blockIdx.x);
    const PrepRec e = recs[r];
    const uint64_t lo = (uint64_t)(blockIdx.x - start[r]) * PREP_CHUNK;
    const uint64_t hi = min(e.words, lo + PREP_CHUNK);
    if (e.src)
        for (uint64_t i = lo + threadIdx.x; i < hi; i += 256) e.dst[i] = e.src[i];
    else
        for (uint64_t i = lo + threadIdx.x; i < hi; i += 256) e.dst[i] = e.value;
}

// ---------------------------------------------------------------------------
// Lattices beyond one workgroup's LDS.  A replica stays in HBM as L rows of L
// bytes.  A launch runs a few half-sweeps over (replica, tile of `rows` rows):
// the workgroup copies its rows and the rows around them (periodic) into LDS,
// updates them and writes its own rows to the other buffer, so the tiles of
// one launch are independent.  The first launch of a step reads its rows from
// the ancestor's replica in the previous population (the copy of Sec. 2 step
// 2, fused).  Pair p = y*L/4 + x/4 uses the same Philox counters as in LDS,
// so the result is the same as for a replica held in LDS.
// ---------------------------------------------------------------------------
// Workgroup -> (replica, tile): each XCD takes a contiguous range, so that
// neighbouring tiles of a replica share their halo rows in one L2.
__device__ __forceinline__ void tile_of(uint32_t tiles, uint32_t &k, uint32_t &tile) {
    uint32_t b = blockIdx.x;
    if ((gridDim.x & 7u) == 0) b = (b & 7u) * (gridDim.x >> 3) + (b >> 3);
    k = b / tiles;
    tile = b % tiles;
}

// Copies rows y0-1 .. y0+n (periodic) of replica src (L/4 dwords per row) to
// LDS rows 0 .. n+1; with halo = false only rows y0 .. y0+n (LDS rows 1 .. n+1).
__device__ __forceinline__ void load_tile_rows(uint32_t *lds32, const uint32_t *src32, uint32_t L,
                                               uint32_t y0, uint32_t n, bool above) {
    const uint32_t DPR = L >> 2;
    if ((L & 15u) == 0) {
        // rows of 16-byte multiples: the tile's rows, contiguous in HBM, in 16-byte loads
        const uint4 *src = reinterpret_cast<const uint4 *>(src32 + y0 * DPR);
        uint4 *dst = reinterpret_cast<uint4 *>(lds32 + DPR);
        for (uint32_t i = threadIdx.x; i < n * DPR / 4u; i += blockDim.x) dst[i] = src[i];
    } else {
        for (uint32_t i = threadIdx.x; i < n * DPR; i += blockDim.x) lds32[DPR + i] = src32[y0 * DPR + i];
    }
    const uint32_t ya = (y0 + L - 1) % L, yb = (y0 + n) % L;
    for (uint32_t x = threadIdx.x; x < DPR; x += blockDim.x) {
        if (above) lds32[x] = src32[ya * DPR + x];
        lds32[(n + 1) * DPR + x] = src32[yb * DPR + x];
    }
}

// `a.halves` consecutive half-sweeps (numbers h0, h0+1, ...; half-sweep h is
// sweep h/2, colour h%2) of one tile in one launch.  The tile's rows and
// `halves` rows on each side (periodic) are staged in LDS; half-sweep j of the
// launch updates the tile and halves-1-j rows on each side, so that the last
// one leaves the tile exact.  The side rows are updated redundantly by the
// neighbouring tiles too, with the same counters and hence the same results;
// only the tile is written back.  halves = 0 copies.  The launch must not
// write the buffer it reads (neighbouring tiles would read rows already
// advanced by this launch).
template <bool QSMALL, bool T64>
__global__ void __launch_bounds__(256) k_tiled_half(TiledArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint32_t k, tile;
    tile_of(a.tiles, k, tile);
    const uint32_t tab = pair_tab_off(tiled_lds_end(a.rows, a.halves, a.L, blockDim.x, false));
    load_thresholds<T64>(smem, tab, a.T, threadIdx.x, blockDim.x);
    const uint32_t L = a.L, DPR = L >> 2, S = a.halves;
    const uint32_t y0 = tile * a.rows, n = min(a.rows, L - y0), nl = n + 2 * S;
    uint32_t *lds32 = reinterpret_cast<uint32_t *>(smem + LDS_HDR);
    const uint32_t src = a.anc ? a.anc[k] : k;
    const uint32_t *src32 = reinterpret_cast<const uint32_t *>(a.src + (size_t)src * a.N);
    // local row r holds global row y0 - S + r (periodic)
    for (uint32_t r = threadIdx.x >> 6; r < nl; r += blockDim.x >> 6) {
        const uint32_t gy = (y0 + r + L - S) % L;
        for (uint32_t x = threadIdx.x & 63u; x < DPR; x += 64u) lds32[r * DPR + x] = src32[gy * DPR + x];
    }
    __syncthreads();
    const Thresholds<T64> thr{smem, tab};
    const uint32_t qm1 = a.q - 1u;
    for (uint32_t j = 0; j < S; ++j) {
        const uint32_t h = a.h0 + j, c = h & 1u;
        const SweepKey key = sweep_key(k, a.step, (DOM_SWEEP << 28) | ((h >> 1) << 1) | c, a.key0, a.key1);
        const uint32_t r0 = 1 + j, np = (nl - 2 - 2 * j) * DPR;       // rows r0 .. nl-2-j
        const uint32_t sy = blockDim.x / DPR, sx = blockDim.x % DPR;
        uint32_t yl = r0 + threadIdx.x / DPR, xd = threadIdx.x % DPR;
        for (uint32_t pl = threadIdx.x; pl < np; pl += blockDim.x) {
            uint32_t gy = y0 + yl + L - S;
            gy = gy >= L ? gy - L : gy;
            gy = gy >= L ? gy - L : gy;
            const uint32_t par = (gy + c) & 1u;
            const uint32_t idx = yl * DPR + xd;
            const uint32_t xo = par ? (xd == DPR - 1 ? idx - (DPR - 1) : idx + 1)
                                    : (xd == 0 ? idx + (DPR - 1) : idx - 1);
            const uint32_t D0 = lds32[idx], Dx = lds32[xo];
            const uint32_t U = lds32[idx - DPR], Dn = lds32[idx + DPR];
            const uint4 w = philox_sweep((uint64_t)PHILOX_M0 * (gy * DPR + xd), key);
            lds32[idx] = update_pair<QSMALL, T64>(D0, Dx, U, Dn, PairSel(par), w, qm1, thr);
            xd += sx;
            if (xd >= DPR) { xd -= DPR; ++yl; }
            yl += sy;
        }
        __syncthreads();
    }
    uint32_t *dst32 = reinterpret_cast<uint32_t *>(a.dst + (size_t)k * a.N) + y0 * DPR;
    for (uint32_t i = threadIdx.x; i < n * DPR; i += blockDim.x) dst32[i] = lds32[S * DPR + i];
}

// The same for L a power of two from 512 on: lane layout fixed at compile
// time (each of the NT lanes owns dword columns tid mod L/4 (+ NT c) of every
// RS-th row of the update range), two rows per iteration for independent work.
// Rows beyond the update range are read from RS padding rows and not stored.
template <uint32_t LT, uint32_t NTT, bool QSMALL, bool T64>
__global__ void __launch_bounds__(NTT) k_tiled_fixed(TiledArgs a) {
    constexpr uint32_t L = LT, DPR = L / 4, NT = NTT;
    constexpr uint32_t CPT = DPR > NT ? DPR / NT : 1;     // dword columns per lane
    constexpr uint32_t RS = DPR >= NT ? 1 : NT / DPR;      // rows per pass of the workgroup
    static_assert(RS <= 2, "at most two padding rows");
    extern __shared__ __align__(16) uint8_t smem[];
    uint32_t k, tile;
    tile_of(a.tiles, k, tile);
    const uint32_t tab = pair_tab_off(tiled_lds_end(a.rows, a.halves, L, NT, true));
    load_thresholds<T64>(smem, tab, a.T, threadIdx.x, blockDim.x);
    const uint32_t S = a.halves, y0 = tile * a.rows, n = a.rows, nl = n + 2 * S;
    uint32_t *lds32 = reinterpret_cast<uint32_t *>(smem + LDS_HDR);
    const uint32_t src = a.anc ? a.anc[k] : k;
    const uint32_t *src32 = reinterpret_cast<const uint32_t *>(a.src + (size_t)src * a.N);
    static_assert(DPR % 64 == 0, "whole waves per row");
    for (uint32_t r = threadIdx.x >> 6; r < nl; r += NT / 64) {
        const uint32_t gy = (y0 + r + L - S) & (L - 1);
        if constexpr (DPR % 256 == 0) {
            // 16-byte loads: a wave covers 1 KB of the row per load
            const uint4 *srow = reinterpret_cast<const uint4 *>(src32 + gy * DPR);
            uint4 *lrow = reinterpret_cast<uint4 *>(lds32 + r * DPR);
#pragma unroll
            for (uint32_t c = 0; c < DPR / 256; ++c) {
                const uint32_t x4 = (threadIdx.x & 63u) + 64u * c;
                lrow[x4] = srow[x4];
            }
        } else {
#pragma unroll
            for (uint32_t c = 0; c < DPR / 64; ++c) {
                const uint32_t x = (threadIdx.x & 63u) + 64u * c;
                lds32[r * DPR + x] = src32[gy * DPR + x];
            }
        }
    }
    __syncthreads();
    const Thresholds<T64> thr{smem, tab};
    const uint32_t qm1 = a.q - 1u;
    const uint32_t xd0 = threadIdx.x % DPR, roff = DPR >= NT ? 0u : threadIdx.x / DPR;
    for (uint32_t j = 0; j < S; ++j) {
        const uint32_t h = a.h0 + j, c = h & 1u;
        const SweepKey key = sweep_key(k, a.step, (DOM_SWEEP << 28) | ((h >> 1) << 1) | c, a.key0, a.key1);
        const uint32_t r0 = 1 + j, nr = nl - 2 - 2 * j;
        // A lane's rows of this half-sweep are r0 + roff + 2 RS i + u RS: their
        // parity, hence the pair selectors and the offset of the left or right
        // neighbour dword, stays fixed for each u.
        PairSel ps[2];
        int32_t dxo[2][CPT];
#pragma unroll
        for (uint32_t u = 0; u < 2; ++u) {
            const uint32_t par = (y0 + r0 + roff + u * RS + L - S + c) & 1u;
            ps[u] = PairSel(par);
#pragma unroll
            for (uint32_t cc = 0; cc < CPT; ++cc) {
                const uint32_t xd = xd0 + cc * NT;
                dxo[u][cc] = par ? (xd == DPR - 1 ? -(int32_t)(DPR - 1) : 1)
                                 : (xd == 0 ? (int32_t)(DPR - 1) : -1);
            }
        }
        for (uint32_t rr = roff; rr < nr; rr += 2 * RS) {
            uint32_t idx[2][CPT], D0[2][CPT], Dx[2][CPT], U[2][CPT], Dn[2][CPT];
            uint4 w[2][CPT];
#pragma unroll
            for (uint32_t u = 0; u < 2; ++u) {
                const uint32_t yl = r0 + rr + u * RS;
                const uint32_t gy = (y0 + yl + L - S) & (L - 1);
#pragma unroll
                for (uint32_t cc = 0; cc < CPT; ++cc) {
                    const uint32_t xd = xd0 + cc * NT;
                    idx[u][cc] = yl * DPR + xd;
                    D0[u][cc] = lds32[idx[u][cc]];
                    Dx[u][cc] = lds32[idx[u][cc] + dxo[u][cc]];
                    U[u][cc] = lds32[idx[u][cc] - DPR];
                    Dn[u][cc] = lds32[idx[u][cc] + DPR];
                    w[u][cc] = philox_sweep((uint64_t)PHILOX_M0 * (gy * DPR + xd), key);
                }
            }
#pragma unroll
            for (uint32_t u = 0; u < 2; ++u) {
                const bool in = rr + u * RS < nr;
#pragma unroll
                for (uint32_t cc = 0; cc < CPT; ++cc) {
                    const uint32_t nw = update_pair<QSMALL, T64>(D0[u][cc], Dx[u][cc], U[u][cc], Dn[u][cc],
                                                                 ps[u], w[u][cc], qm1, thr);
                    if (in) lds32[idx[u][cc]] = nw;
                }
            }
        }
        __syncthreads();
    }
    // the tile's rows, contiguous in HBM, in 16-byte stores (rows of L bytes, L a
    // power of two from 512)
    uint4 *dst = reinterpret_cast<uint4 *>(a.dst + (size_t)k * a.N + (size_t)y0 * L);
    const uint4 *lsrc = reinterpret_cast<const uint4 *>(lds32 + S * DPR);
    for (uint32_t i = threadIdx.x; i < n * DPR / 4u; i += NT) dst[i] = lsrc[i];
}

__global__ void __launch_bounds__(256) k_tiled_init(TiledArgs a) {
    uint32_t k, tile;
    tile_of(a.tiles, k, tile);
    const uint32_t DPR = a.L >> 2, y0 = tile * a.rows, n = min(a.rows, a.L - y0);
    uint32_t *dst32 = reinterpret_cast<uint32_t *>(a.dst + (size_t)k * a.N);
    if (a.init == SWEEP_INIT_RANDOM) {
        // site n takes word n mod 4 of Philox(n / 4, k, 0, INIT)
        for (uint32_t dd = y0 * DPR + threadIdx.x; dd < (y0 + n) * DPR; dd += blockDim.x) {
            const uint4 w = philox(dd, k, 0u, DOM_INIT << 28, a.key0, a.key1);
            dst32[dd] = mulhi32(w.x, a.q) | (mulhi32(w.y, a.q) << 8) | (mulhi32(w.z, a.q) << 16) |
                        (mulhi32(w.w, a.q) << 24);
        }
    } else {
        // eq. (6): all spins alpha, alpha uniform over the q states
        const uint4 w = philox(0u, k, 0u, DOM_GROUND << 28, a.key0, a.key1);
        const uint32_t alpha = mulhi32(w.x, a.q) * 0x01010101u;
        for (uint32_t dd = y0 * DPR + threadIdx.x; dd < (y0 + n) * DPR; dd += blockDim.x) dst32[dd] = alpha;
    }
}

// Bonds (eq. (3)) of the tile's rows (right and down neighbours) and, with
// cnt, the number of sites in each state (eq. (5)); added to the replica's
// totals.
__global__ void __launch_bounds__(256) k_tiled_measure(TiledArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ uint32_t s_part[4];
    uint32_t k, tile;
    tile_of(a.tiles, k, tile);
    const uint32_t L = a.L, DPR = L >> 2;
    const uint32_t y0 = tile * a.rows, n = min(a.rows, L - y0);
    uint32_t *lds32 = reinterpret_cast<uint32_t *>(smem);
    uint32_t *scnt = reinterpret_cast<uint32_t *>(smem) + (a.rows + 2) * DPR;   // [q]
    if (a.cnt)
        for (uint32_t s = threadIdx.x; s < a.q; s += blockDim.x) scnt[s] = 0u;
    load_tile_rows(lds32, reinterpret_cast<const uint32_t *>(a.dst + (size_t)k * a.N), L, y0, n, false);
    __syncthreads();
    // Bonds to the right and down of every site of the tile: a lane keeps one
    // dword column (and its right neighbour, periodic) and steps over rows.
    uint32_t bonds = 0;
    auto column = [&](uint32_t x, uint32_t r0, uint32_t rstep) {
        const uint32_t xr = x == DPR - 1 ? 0u : x + 1u;
        for (uint32_t r = r0; r < n; r += rstep) {
            const uint32_t *row = lds32 + (r + 1) * DPR;
            const uint32_t D = row[x];
            bonds += eq_bytes(D, __builtin_amdgcn_alignbyte(row[xr], D, 1)) + eq_bytes(D, row[DPR + x]);
        }
    };
    if (DPR <= blockDim.x) {
        const uint32_t per = blockDim.x / DPR;            // rows per pass of the workgroup
        if (threadIdx.x < per * DPR) column(threadIdx.x % DPR, threadIdx.x / DPR, per);
    } else {
        for (uint32_t x = threadIdx.x; x < DPR; x += blockDim.x) column(x, 0u, 1u);
    }
    bonds = wave_sum(bonds);
    if ((threadIdx.x & 63u) == 0) s_part[threadIdx.x >> 6] = bonds;
    if (a.Hacc) {
        uint64_t dig = 0;
        for (uint32_t i = threadIdx.x; i < n * DPR; i += blockDim.x)
            dig += digest_term(y0 * DPR + i, k, a.step, lds32[DPR + i], a.key0, a.key1);
        dig = wave_sum(dig);
        if ((threadIdx.x & 63u) == 0) atomicAdd(reinterpret_cast<unsigned long long *>(&a.Hacc[k]),
                                                (unsigned long long)dig);
    }
    if (a.cnt) {
        for (uint32_t st = 0; st < a.q; ++st) {
            const uint32_t pat = st * 0x01010101u;
            uint32_t c = 0;
            for (uint32_t i = threadIdx.x; i < n * DPR; i += blockDim.x) c += eq_bytes(lds32[DPR + i], pat);
            c = wave_sum(c);
            if ((threadIdx.x & 63u) == 0 && c) atomicAdd(&scnt[st], c);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t b = 0;
        for (uint32_t w = 0; w < (blockDim.x >> 6); ++w) b += s_part[w];
        atomicAdd(&a.bonds[k], b);
    }
    if (a.cnt)
        for (uint32_t s = threadIdx.x; s < a.q; s += blockDim.x)
            if (scnt[s]) atomicAdd(&a.cnt[(size_t)k * a.q + s], scnt[s]);
}

// Per replica: E = -bonds, M~ = the largest state count; clears both sums.
__global__ void k_tiled_finalize(TiledArgs a) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.R) return;
    a.E_out[k] = -(int32_t)a.bonds[k];
    a.bonds[k] = 0u;
    if (a.Hacc) {
        a.H_out[k] = a.Hacc[k];
        a.Hacc[k] = 0ull;
    }
    if (a.cnt) {
        uint32_t m = 0;
        for (uint32_t s = 0; s < a.q; ++s) {
            m = max(m, a.cnt[(size_t)k * a.q + s]);
            a.cnt[(size_t)k * a.q + s] = 0u;
        }
        if (a.Mt_out) a.Mt_out[k] = m;
    }
}


// ---------------------------------------------------------------------------
// Team kernel (k_team): small runs of one sweep class advanced through all
// their steps in one cooperative launch.  Each run owns a team of workgroups
// of 1024 threads.  Per step i, workgroup 0 of the team forms the statistics of
// step i-1 (the k_post statistics: histogram, sums, ln Q_i, -beta F_i, digest),
// while every other workgroup repeats the whole resampling into step i in its
// LDS from the energies of step i-1 (E_ref, the integer weights and their
// scan, the draws, the copy numbers and their scan: the same integer results as
// k_post, k_sample and k_countfill, since the arithmetic is exact) and then
// sweeps its own contiguous range of new slots, gathering each replica from its
// ancestor.  One team barrier per step separates the steps: energies, digest
// terms and M~ alternate between two buffers by step, so the statistics of
// step i-1 and the sweeps of step i never touch the same buffer.
//
// Barrier: every thread waits for its own stores, the workgroup meets, one
// thread adds to the team counter with agent-scope release and waits for the
// team's count with agent-scope acquire.  The wait is bounded: it ends when
// the host sets the abort word (pinned host memory) or after timeout_ticks of
// the 100 MHz real-time counter, after which it sets the abort word itself, so
// every workgroup leaves normally.
// ---------------------------------------------------------------------------
constexpr uint32_t TEAM_THREADS = 1024;
static_assert(POST_LDS_BINS * 4u <= 65536u, "the statistics' LDS window fits a team workgroup's work area");

__device__ bool team_barrier(uint32_t *ctr, uint32_t target, const TeamCtl &ctl, uint32_t *s_ok) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t ok = 1, spins = 0;
        const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(2);
            if ((++spins & 63u) == 0) {
                if (__hip_atomic_load(ctl.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) { ok = 0; break; }
                if (__builtin_amdgcn_s_memrealtime() - t0 > ctl.timeout_ticks) {
                    __hip_atomic_store(ctl.abort, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    ok = 0;
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

// The resampling into step `st.step` (Sec. 2 step 2, eq. (1)) in one
// workgroup's LDS: the ancestor of every new slot in ancL[0 .. n_new) (if
// ancL is given).  Work areas: E and then the copy numbers in ru[R_prev], the
// cumulative weights and then the offsets in C[R_prev].  With `write_out` the
// ancestors also go to st.anc_out and the copy numbers to st.counts_out.
__device__ __forceinline__ void small_resample_body(const SmallResample &st, uint32_t *ancL, uint32_t *ru,
                                                    uint64_t *C, uint64_t *scratch, bool write_out) {
    const uint32_t tid = threadIdx.x, n = (uint32_t)st.R_prev;
    if (!st.resample) {
        for (uint32_t k = tid; k < (uint32_t)st.n_new; k += blockDim.x) {
            if (ancL) ancL[k] = k;
            if (write_out) st.anc_out[k] = k;
        }
        __syncthreads();
        return;
    }
    // E_ref: the smallest energy (the largest when dbeta < 0)
    int32_t mn = 0x7fffffff, mx = (int32_t)0x80000000;
    for (uint32_t j = tid; j < n; j += blockDim.x) {
        const int32_t e = st.E_prev[j];
        reinterpret_cast<int32_t *>(ru)[j] = e;
        mn = min(mn, e);
        mx = max(mx, e);
    }
    const SumMinMax t = block_sum_min_max<true>(0, mn, mx);
    const int32_t ref = st.ref_max ? t.mx : t.mn;
    // C_j = sum_{j' <= j} W(|E_j' - E_ref|), rows of 4 per thread
    uint64_t carry = 0;
    for (uint32_t base = 0; base < n; base += blockDim.x * 4u) {
        const uint32_t j = base + tid * 4u;
        uint64_t w[4];
#pragma unroll
        for (uint32_t v = 0; v < 4; ++v) {
            uint64_t x = 0;
            if (j + v < n) {
                const uint32_t d = (uint32_t)abs(reinterpret_cast<const int32_t *>(ru)[j + v] - ref);
                x = st.w_const ? st.w_const : (d < st.D ? st.W[d] : 0ull);
            }
            w[v] = x;
        }
        w[1] += w[0]; w[2] += w[1]; w[3] += w[2];
        const uint64_t incl = wave_inclusive_scan(w[3]);
        uint64_t total;
        const uint64_t off = carry + block_wave_offset<true>(lane_value(incl, 63), scratch, &total) + incl - w[3];
#pragma unroll
        for (uint32_t v = 0; v < 4; ++v)
            if (j + v < n) C[j + v] = w[v] + off;
        carry += total;
    }
    __syncthreads();
    // the draws: u = floor(x S / 2^64), ancestor = first j with C_j > u
    const uint64_t S = C[n - 1];
    for (uint32_t j = tid; j < n; j += blockDim.x) ru[j] = 0u;
    __syncthreads();
    for (uint64_t kk = tid; kk < st.n_new; kk += blockDim.x) {
        const uint4 w = philox((uint32_t)kk, 0u, st.step, DOM_RESAMPLE << 28, st.key0, st.key1);
        const uint64_t x = ((uint64_t)w.y << 32) | (uint64_t)w.x;
        const uint64_t u = __umul64hi(x, S);
        uint32_t lo = 0, hi = n - 1;
        while (lo < hi) {
            const uint32_t mid = lo + ((hi - lo) >> 1);
            if (C[mid] > u) hi = mid; else lo = mid + 1;
        }
        atomicAdd(&ru[lo], 1u);
    }
    __syncthreads();
    // offsets o_j = sum_{j' < j} r_j' (in the C area), the copy numbers kept
    uint32_t *o = reinterpret_cast<uint32_t *>(C);
    uint64_t ocarry = 0;
    for (uint32_t base = 0; base < n; base += blockDim.x * 4u) {
        const uint32_t j = base + tid * 4u;
        uint32_t r[4];
#pragma unroll
        for (uint32_t v = 0; v < 4; ++v) r[v] = j + v < n ? ru[j + v] : 0u;
        const uint32_t sum = r[0] + r[1] + r[2] + r[3];
        const uint32_t incl = wave_inclusive_scan(sum);
        uint32_t total;
        const uint32_t woff = block_wave_offset<true>(lane_value(incl, 63), reinterpret_cast<uint32_t *>(scratch), &total);
        uint32_t at = (uint32_t)ocarry + woff + incl - sum;
#pragma unroll
        for (uint32_t v = 0; v < 4; ++v) {
            if (j + v < n) o[j + v] = at;
            at += r[v];
        }
        ocarry += total;
    }
    __syncthreads();
    // the copies of ancestor j fill slots o_j .. o_j + r_j - 1
    for (uint32_t j = tid; j < n; j += blockDim.x) {
        const uint32_t r = ru[j], b = o[j];
        if (ancL)
            for (uint32_t k = b; k < b + r; ++k) ancL[k] = j;
        if (write_out) {
            st.counts_out[j] = r;
            for (uint32_t k = b; k < b + r; ++k) st.anc_out[k] = j;
        }
    }
    __syncthreads();
}

// The same, called (not inlined) from the team kernel so that its registers do
// not add to the sweep's.
__device__ __attribute__((noinline)) void small_resample(const SmallResample &st, uint32_t *ancL, uint32_t *ru,
                                                         uint64_t *C, uint64_t *scratch, bool write_out) {
    small_resample_body(st, ancL, ru, C, scratch, write_out);
}

// The statistics of a step, called (not inlined) from the team kernel so that
// their registers do not add to the sweep's.
__device__ __attribute__((noinline)) void team_stats(const PostArgs &a, uint32_t *lds, uint64_t *scratch,
                                                     uint32_t lds_cap) {
    post_stats<8, true>(a, lds, scratch, lds_cap);
}

template <uint32_t LT, uint32_t GT, bool QSMALL, bool T64>
__global__ void __launch_bounds__(TEAM_THREADS)
k_team(const TeamRun *runs, uint32_t n_runs, const TeamStep *steps, TeamCtl ctl) {
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ uint32_t s_ok, s_next;
    __shared__ uint64_t scratch[17];
    // the run: runs are sorted by their first workgroup
    uint32_t lo = 0, hi = n_runs - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (runs[mid].team0 <= blockIdx.x) lo = mid; else hi = mid - 1;
    }
    const TeamRun &tr = runs[__builtin_amdgcn_readfirstlane(lo)];
    const uint32_t w = blockIdx.x - tr.team0;       // 0: statistics, 1 .. team-1: sweeps
    if (w >= tr.team) return;                        // (not reached: the grid is the teams)
    // LDS: the ancestors of the new slots, then one area used in turn by the
    // resampling (ru, C), the sweep groups and the statistics
    uint32_t *ancL = reinterpret_cast<uint32_t *>(smem);
    uint8_t *work = smem + ctl.anc_bytes;
    uint32_t *ru = reinterpret_cast<uint32_t *>(work);
    uint64_t *C = reinterpret_cast<uint64_t *>(work + ((4u * ctl.r_max + 15u) & ~15u));
    const uint32_t lds_cap = ctl.work_bytes / 4u;
    // sweep groups: a k_sweep workgroup's worth of waves each (64 * waves_per_block
    // threads, which divides 1024 for the classes of this kernel)
    const uint32_t BS = 64u * steps[tr.rec0].w.waves_per_block;
    const uint32_t SUB = TEAM_THREADS / BS;
    const uint32_t rpb = GT > 64u ? 1u : BS / GT;                 // replicas per group
    const uint32_t sub = threadIdx.x / BS, stid = threadIdx.x % BS;
    uint32_t gen = 0;
    for (uint32_t s = 0; s < tr.n_steps; ++s) {
        const TeamStep &st = steps[tr.rec0 + s];
        if (s > 0 && !team_barrier(tr.barrier, ++gen * tr.team, ctl, &s_ok)) return;
        if (w == 0) {
            if (st.stats) team_stats(st.p, reinterpret_cast<uint32_t *>(work), scratch, lds_cap);
            continue;
        }
        // Sweep blocks are taken `unit` at a time from the step's counter,
        // so that workgroups which run faster take more of them; `unit`
        // (at most SUB, one per sweep group) spreads a step's blocks over
        // all the team's sweep workgroups.  The next claim is in flight
        // while the current blocks are swept.
        uint32_t *claim = tr.claims + s;
        const uint32_t nblocks = (uint32_t)((st.w.R_new + rpb - 1) / rpb);
        const uint32_t nsw = tr.team - 1;
        const uint32_t unit = min(SUB, max(1u, (nblocks + nsw - 1) / nsw));
        uint32_t next = 0;
        if (threadIdx.x == 0) next = __hip_atomic_fetch_add(claim, unit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        small_resample(st.r, ancL, ru, C, scratch, w == 1);
        if (threadIdx.x == 0) s_next = next;
        __syncthreads();
        uint32_t b = s_next;
        while (b < nblocks) {
            if (threadIdx.x == 0) next = __hip_atomic_fetch_add(claim, unit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // groups beyond the claim sweep no replica (they still meet the
            // workgroup barriers of the classes that have them)
            const uint32_t blk = sub < unit ? b + sub : nblocks;
            sweep_body<LT, GT, QSMALL, T64, true>(st.w, blk, work + (size_t)sub * ctl.sub_lds, stid, BS,
                                                  ancL, 0u, (uint32_t)st.w.R_new);
            __syncthreads();                     // every group is done with its LDS and s_next
            if (threadIdx.x == 0) s_next = next;
            __syncthreads();
            b = s_next;
        }
    }
    if (!team_barrier(tr.barrier, ++gen * tr.team, ctl, &s_ok)) return;
    if (w == 0 && tr.last_stats) team_stats(tr.last, reinterpret_cast<uint32_t *>(work), scratch, lds_cap);
}

}  // namespace

// Lanes-per-replica candidates of the fixed-shape kernels (first = default,
// chosen by measurement on MI355X; pa_autotune can pick the other).
// Lanes per replica that have a compile-time sweep kernel, per lattice side:
// a lane owns one dword column, so the lanes are a multiple of L/4 and divide
// the L*L/4 pairs.  The first entry is the default.
struct LaneChoice { uint32_t L, lanes[2]; };
static const LaneChoice kLaneChoices[LANE_CHOICE_COUNT] = {
    {4, {4, 4}},
    {8, {16, 8}},
    {12, {36, 12}},       // replicas span waves: 16 per block of 9 or 3 waves
    {16, {64, 32}},
    {20, {20, 10}},       // 16 or 32 replicas per block of 5 waves
    {24, {48, 144}},      // 4 replicas per block of 3 or 9 waves
    {32, {256, 128}},
    {48, {192, 576}},     // three or nine waves per replica
    {64, {512, 1024}},
    {96, {768, 384}},     // twelve or six waves per replica
    {128, {512, 1024}},
    {192, {768, 384}},
    {256, {1024, 512}},
};

int lane_choice_index(uint32_t L) {
    for (int i = 0; i < LANE_CHOICE_COUNT; ++i)
        if (kLaneChoices[i].L == L) return i;
    return -1;
}

uint32_t lane_candidates(uint32_t L, uint32_t *out) {
    const int i = lane_choice_index(L);
    if (i < 0) return 0;
    out[0] = kLaneChoices[i].lanes[0];
    if (kLaneChoices[i].lanes[1] == kLaneChoices[i].lanes[0]) return 1;
    out[1] = kLaneChoices[i].lanes[1];
    return 2;
}

void sweep_shape(uint32_t L, uint32_t lanes, uint32_t *G_out, uint32_t *waves_per_block) {
    uint32_t G = 0;
    if (L & 3u) {
        // byte kernel: one replica per wave, up to four per workgroup, as many
        // as 64 KB of LDS hold (one for larger replicas)
        const uint32_t bytes = ((L * L) + 15u) & ~15u;
        uint32_t wpb = 4;
        while (wpb > 1 && wpb * bytes > 65536u) --wpb;
        *G_out = 64;
        *waves_per_block = wpb;
        return;
    }
    if (lane_choice_index(L) >= 0) {
        uint32_t cand[2];
        const uint32_t n = lane_candidates(L, cand);
        G = cand[0];
        for (uint32_t c = 0; c < n; ++c)
            if (cand[c] == lanes) G = lanes;
    } else {
        // other sizes (generic kernel): two waves per replica from L = 96 on,
        // four from L = 192; below, the largest power of two <= L*L/4 up to 64
        if (L >= 192) G = 256;
        else if (L >= 96) G = 128;
        else { G = 4; while (G < 64 && 2 * G <= (L * L) / 4u) G *= 2; }
    }
    *G_out = G;
    if (G > 64 && G % 64 == 0) {       // one replica per workgroup of G/64 waves
        *waves_per_block = G / 64;
        return;
    }
    if (64 % G != 0) {                 // replicas span waves: lcm(G, 64) lanes per workgroup
        uint32_t w = 1;
        while ((64 * w) % G != 0) ++w;
        *waves_per_block = w;
        return;
    }
    const uint32_t N = L * L;
    const uint32_t rpw = 64u / G;
    uint32_t wpb = 4;
    while (wpb > 1 && (size_t)wpb * rpw * (N + 2 * L) > 32768u) wpb >>= 1;
    *waves_per_block = wpb;
}

uint64_t replicas_per_block(uint32_t G, uint32_t waves_per_block) {
    return (G > 64 && G % 64 == 0) ? 1u : (64u * waves_per_block) / G;
}

size_t sweep_lds_bytes(uint32_t N, uint32_t G, uint32_t waves_per_block, uint32_t q_counters) {
    uint32_t L = 0;
    while (L * L < N) ++L;
    if (L & 3u) return (size_t)waves_per_block * ((N + 15u) & ~15u);   // byte kernel
    const uint64_t rpb = replicas_per_block(G, waves_per_block);
    return pair_tab_off(sweep_lds_end(N, L, G, (uint32_t)rpb, q_counters)) + PAIR_TAB_BYTES;
}

size_t max_lds_per_block(int device) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess)
        return 65536;
    return (size_t)v;
}

hipError_t launch_sweep(const SweepArgs &a, hipStream_t s) {
    const uint64_t per_block = replicas_per_block(a.G, a.waves_per_block);
    const uint64_t blocks = (a.R_new + per_block - 1) / per_block;
    if (blocks == 0) return hipSuccess;
    const size_t lds = sweep_lds_bytes(a.N, a.G, a.waves_per_block, a.Mt_out ? a.q : 0u);
    void *kern = sweep_kernel(sweep_class(a.L, a.q, a.T[3] == 0, a.G), false);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((void (*)(SweepArgs))kern, dim3((uint32_t)blocks), dim3(64u * a.waves_per_block), lds,
                       s, a);
    return hipGetLastError();
}

hipError_t launch_post(const PostArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_post, dim3(post_blocks(a)), dim3(WG_THREADS), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_resample(const SampleArgs &a, const SlotmapArgs &m, hipStream_t s) {
    const uint64_t blocks = (a.n_new + 255) / 256;
    if (blocks) hipLaunchKernelGGL(k_sample, dim3((uint32_t)blocks), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_countfill, dim3(countfill_blocks(m)), dim3(WG_THREADS), 0, s, m);
    return hipGetLastError();
}

// Kernel class: lattice side, lanes per replica, q <= 128, 64-bit thresholds;
// bit 31 marks the byte kernel of L = 2 (mod 4).
constexpr uint32_t CLASS_BYTES = 1u << 31;
uint32_t sweep_class(uint32_t L, uint32_t q, bool t64, uint32_t G) {
    if (L & 3u) return CLASS_BYTES | (L << 16);
    return (L << 16) | (G << 2) | ((q <= 128) ? 2u : 0u) | (t64 ? 1u : 0u);
}

// The instance for a class: fixed-shape when L is a power of two with a
// candidate lane count and the 32-bit threshold form applies, else generic.
void *sweep_kernel(uint32_t cls, bool batch) {
    if (cls & CLASS_BYTES) return batch ? (void *)k_sweep_bytes_batch : (void *)k_sweep_bytes;
    const uint32_t L = (cls >> 16) & 0x7FFFu, G = (cls >> 2) & 0x3FFFu;
    const bool qs = (cls & 2u) != 0, t64 = (cls & 1u) != 0;
#define PA_INST(LV, GV)                                                                       \
    if (L == LV && G == GV)                                                                   \
        return batch ? (qs ? (void *)k_sweep_batch<LV, GV, true, false> : (void *)k_sweep_batch<LV, GV, false, false>) \
                     : (qs ? (void *)k_sweep<LV, GV, true, false> : (void *)k_sweep<LV, GV, false, false>);
    if (!t64) {
        PA_INST(4, 4)
        PA_INST(8, 8) PA_INST(8, 4) PA_INST(8, 16)
        PA_INST(12, 12) PA_INST(12, 36)
        PA_INST(16, 16) PA_INST(16, 8) PA_INST(16, 32) PA_INST(16, 64)
        PA_INST(20, 10) PA_INST(20, 20)
        PA_INST(24, 48) PA_INST(24, 72) PA_INST(24, 144)
        PA_INST(32, 64) PA_INST(32, 32) PA_INST(32, 128) PA_INST(32, 256)
        PA_INST(48, 192) PA_INST(48, 576)
        PA_INST(64, 64) PA_INST(64, 256) PA_INST(64, 128) PA_INST(64, 512) PA_INST(64, 1024)
        PA_INST(96, 192) PA_INST(96, 384) PA_INST(96, 768)
        PA_INST(128, 256) PA_INST(128, 512) PA_INST(128, 128) PA_INST(128, 1024)
        PA_INST(192, 384) PA_INST(192, 768)
        PA_INST(256, 1024) PA_INST(256, 512)
    }
#undef PA_INST
    if (t64)
        return batch ? (qs ? (void *)k_sweep_batch<0, 0, true, true> : (void *)k_sweep_batch<0, 0, false, true>)
                     : (qs ? (void *)k_sweep<0, 0, true, true> : (void *)k_sweep<0, 0, false, true>);
    return batch ? (qs ? (void *)k_sweep_batch<0, 0, true, false> : (void *)k_sweep_batch<0, 0, false, false>)
                 : (qs ? (void *)k_sweep<0, 0, true, false> : (void *)k_sweep<0, 0, false, false>);
}

hipError_t launch_sweep_batch(uint32_t cls, const SweepArgs *runs, const uint32_t *start, uint32_t n,
                              uint32_t blocks, uint32_t threads, size_t lds, hipStream_t s) {
    if (blocks == 0 || n == 0) return hipSuccess;
    void *kern = sweep_kernel(cls, true);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((void (*)(const SweepArgs *, const uint32_t *, uint32_t))kern, dim3(blocks),
                       dim3(threads), lds, s, runs, start, n);
    return hipGetLastError();
}

hipError_t launch_post_batch(const PostArgs *runs, const uint32_t *pstart, uint32_t n, uint32_t blocks,
                             hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_post_batch, dim3(blocks), dim3(WG_THREADS), 0, s, runs, pstart, n);
    return hipGetLastError();
}

hipError_t launch_resample_batch(const SampleArgs *sruns, const uint32_t *start, uint32_t n,
                                 uint32_t blocks, const SlotmapArgs *mruns, const uint32_t *mstart,
                                 uint32_t mblocks, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (blocks) hipLaunchKernelGGL(k_sample_batch, dim3(blocks), dim3(256), 0, s, sruns, start, n);
    hipLaunchKernelGGL(k_countfill_batch, dim3(mblocks), dim3(WG_THREADS), 0, s, mruns, mstart, n);
    return hipGetLastError();
}

// Team kernels: the classes whose k_sweep workgroup (64 * waves_per_block
// threads) divides 1024, with the 32-bit threshold form.
void *team_kernel(uint32_t cls) {
    if (cls & (CLASS_BYTES | 1u)) return nullptr;
    const uint32_t L = (cls >> 16) & 0x7FFFu, G = (cls >> 2) & 0x3FFFu;
    const bool qs = (cls & 2u) != 0;
#define PA_TEAM(LV, GV) \
    if (L == LV && G == GV) return qs ? (void *)k_team<LV, GV, true, false> : (void *)k_team<LV, GV, false, false>;
    PA_TEAM(8, 16) PA_TEAM(8, 8) PA_TEAM(16, 64) PA_TEAM(16, 32) PA_TEAM(32, 256) PA_TEAM(32, 128) PA_TEAM(64, 512)
#undef PA_TEAM
    return nullptr;
}

uint32_t team_threads() { return TEAM_THREADS; }

uint32_t team_capacity(uint32_t cls, size_t lds, int device) {
    void *k = team_kernel(cls);
    int occ = 0, cus = 0;
    if (!k) return 0;
    if (lds > 65536 && hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, TEAM_THREADS, lds) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 0;
    return (uint32_t)(occ > 0 ? occ : 0) * (uint32_t)cus;
}

hipError_t launch_team(uint32_t cls, const TeamRun *runs, uint32_t n_runs, const TeamStep *steps,
                       const TeamCtl &ctl, uint32_t blocks, size_t lds, hipStream_t s) {
    void *k = team_kernel(cls);
    if (!k || blocks == 0) return hipErrorInvalidValue;
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    TeamCtl c = ctl;
    void *args[] = {(void *)&runs, (void *)&n_runs, (void *)&steps, (void *)&c};
    return hipLaunchCooperativeKernel(k, dim3(blocks), dim3(TEAM_THREADS), args, (unsigned)lds, s);
}

bool tiled_path(uint32_t L) { return L > 256; }

uint32_t tiled_rows(uint32_t L) {
    // about 16 KB of rows per tile, at least two
    const uint32_t r = 16384u / L;
    return r < 2u ? 2u : (r > L ? L : r);
}

// Each fused half-sweep beyond the first recomputes two rows per side; two
// per launch measured best for L = 512 .. 4096 (one, three or four: 0-25 %
// slower, taller tiles: slower still).
uint32_t tiled_max_halves(uint32_t L) {
    (void)L;
    return 2u;
}

// Threads per workgroup of the fixed-layout tiled kernel.  At L = 4096 a tile
// holds few rows, so the LDS that limits workgroups per CU is better shared by
// 512 threads (32 waves per CU instead of 16: 589 -> 689 attempts/ns at theta
// 10); at L = 1024 and 2048 512 threads measured slower (-19 % and -2 %).
static uint32_t tiled_threads(uint32_t L) { return L >= 4096 ? 512u : 256u; }

// LDS of a tiled launch: tile and side rows, plus the padding rows the
// fixed-layout kernel reads past the update range (one row per row step of a
// lane: RS = threads / (L/4) rows, at least one).  The budget decides how many
// workgroups share a CU (at L = 4096 two padding rows left room for 3, one
// for 4: 12 or 16 waves).
static size_t tiled_lds_bytes(const TiledArgs &a, bool fixed) {
    const uint32_t nt = fixed ? tiled_threads(a.L) : 256u;
    return pair_tab_off(tiled_lds_end(a.rows, a.halves, a.L, nt, fixed)) + PAIR_TAB_BYTES;
}

template <bool QSMALL, bool T64>
static void *tiled_fixed_kernel(uint32_t L) {
    switch (L) {
        case 512: return (void *)k_tiled_fixed<512, 256, QSMALL, T64>;
        case 1024: return (void *)k_tiled_fixed<1024, 256, QSMALL, T64>;
        case 2048: return (void *)k_tiled_fixed<2048, 256, QSMALL, T64>;
        case 4096: return (void *)k_tiled_fixed<4096, 512, QSMALL, T64>;
        default: return nullptr;
    }
}

hipError_t launch_tiled_half(const TiledArgs &a, hipStream_t s) {
    const uint64_t blocks = (uint64_t)a.R * a.tiles;
    if (blocks == 0) return hipSuccess;
    const bool qsmall = a.q <= 128, t64 = a.T[3] == 0;
    void (*kern)(TiledArgs) = qsmall ? (t64 ? k_tiled_half<true, true> : k_tiled_half<true, false>)
                                     : (t64 ? k_tiled_half<false, true> : k_tiled_half<false, false>);
    bool fixed = false;
    if (a.halves > 0 && a.L % a.rows == 0) {
        void *f = qsmall ? (t64 ? tiled_fixed_kernel<true, true>(a.L) : tiled_fixed_kernel<true, false>(a.L))
                         : (t64 ? tiled_fixed_kernel<false, true>(a.L) : tiled_fixed_kernel<false, false>(a.L));
        if (f) { kern = (void (*)(TiledArgs))f; fixed = true; }
    }
    const uint32_t threads = fixed ? tiled_threads(a.L) : 256u;
    hipLaunchKernelGGL(kern, dim3((uint32_t)blocks), dim3(threads), tiled_lds_bytes(a, fixed), s, a);
    return hipGetLastError();
}

hipError_t launch_tiled_init(const TiledArgs &a, hipStream_t s) {
    const uint64_t blocks = (uint64_t)a.R * a.tiles;
    if (blocks) hipLaunchKernelGGL(k_tiled_init, dim3((uint32_t)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tiled_measure(const TiledArgs &a, hipStream_t s) {
    const uint64_t blocks = (uint64_t)a.R * a.tiles;
    if (blocks == 0) return hipSuccess;
    const size_t lds = (size_t)(a.rows + 2) * a.L + 4 * 256;
    hipLaunchKernelGGL(k_tiled_measure, dim3((uint32_t)blocks), dim3(256), lds, s, a);
    hipLaunchKernelGGL(k_tiled_finalize, dim3((a.R + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_prep_batch(const PrepRec *recs, const uint32_t *start, uint32_t n, uint32_t blocks,
                             hipStream_t s) {
    if (n == 0 || blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_prep_batch, dim3(blocks), dim3(256), 0, s, recs, start, n);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace pa
