// pa_kernels.hip -- gfx950 kernels for population annealing of the 2D q-state
// Potts model (arXiv:1704.01888, Sec. 2-3).
//
//   k_sweep        : initial population (step 1 of Sec. 2) or, per step, the
//                    gather of each new replica from its ancestor (eq. (1)) plus
//                    theta checkerboard Metropolis sweeps (step 3) held in LDS,
//                    then the energy of eq. (3) and the population histogram.
//   k_stats        : population sums for eq. (4), the reference energy and
//                    ln Q of step 2 / eq. (2) in FP64 (one workgroup).
//   k_weights_scan : integer weights W(|E_j - E_ref|) and their inclusive scan.
//   k_sample       : the multinomial draws of the resampling step.
//   k_slotmap      : exclusive scan of the copy numbers -> ancestor of each new slot.
//
// One replica lives inside one wavefront (G = 4..64 lanes of it), so the two
// half-sweeps of a sweep need no workgroup barrier: LDS operations of a wave
// execute in order, and a compiler fence keeps the half-sweeps apart.
#include "pa_device.h"

namespace pa {

namespace {

constexpr uint32_t PHILOX_M0 = 0xD2511F53u;
constexpr uint32_t PHILOX_M1 = 0xCD9E8D57u;
constexpr uint32_t PHILOX_W0 = 0x9E3779B9u;
constexpr uint32_t PHILOX_W1 = 0xBB67AE85u;

// Philox4x32-10 (Salmon et al., SC'11), all in registers.
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
        const uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ uint32_t mulhi32(uint32_t w, uint32_t n) { return __umulhi(w, n); }

// Number of equal bytes between two words.
__device__ __forceinline__ uint32_t eq_bytes(uint32_t a, uint32_t b) {
    const uint32_t x = a ^ b;
    const uint32_t nz = (((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u;
    return 4u - __popc(nz);
}

// Metropolis update of one site (Sec. 2 step 3 with the proposal and
// acceptance arithmetic of the header comment of pa.h).
__device__ __forceinline__ uint32_t update_site(uint32_t s, uint32_t l, uint32_t r, uint32_t u,
                                                uint32_t d, uint32_t w_prop, uint32_t w_acc,
                                                uint32_t qm1, const uint64_t *Ttab) {
    const uint32_t rr = mulhi32(w_prop, qm1);
    const uint32_t sp = rr + (rr >= s ? 1u : 0u);
    const int dE = (int)(l == s) + (int)(r == s) + (int)(u == s) + (int)(d == s)
                 - (int)(l == sp) - (int)(r == sp) - (int)(u == sp) - (int)(d == sp);
    const uint64_t T = Ttab[dE + 4];
    return (T > (uint64_t)w_acc) ? sp : s;
}

__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__global__ void __launch_bounds__(256) k_sweep(SweepArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint64_t *Ttab = reinterpret_cast<uint64_t *>(smem);          // [9], index dE + 4
    if (threadIdx.x < 9) {
        const int dE = (int)threadIdx.x - 4;
        Ttab[threadIdx.x] = dE <= 0 ? (1ull << 32) : a.T[dE - 1];
    }
    __syncthreads();

    const uint32_t G_log2 = a.G_log2;
    const uint32_t G = 1u << G_log2;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    const uint32_t g = lane & (G - 1u);
    const uint32_t rpw = 64u >> G_log2;                          // replicas per wave
    const uint32_t rep = wave * rpw + (lane >> G_log2);          // replica within block
    const uint64_t k64 = (uint64_t)blockIdx.x * a.waves_per_block * rpw + rep;
    const uint64_t first_in_wave = (uint64_t)blockIdx.x * a.waves_per_block * rpw + wave * rpw;
    if (first_in_wave >= a.R_new) return;                        // whole wave idle
    const bool live = k64 < a.R_new;
    const uint32_t k = (uint32_t)k64;

    const uint32_t L = a.L, N = a.N;
    uint8_t *rep_lds = smem + 128 + (size_t)rep * N;
    uint32_t *lds32 = reinterpret_cast<uint32_t *>(rep_lds);

    // ---- load or create the replica in LDS -----------------------------
    if (a.mode == SWEEP_UPDATE) {
        const uint32_t src = live ? (a.anc ? a.anc[k] : k) : 0u;
        const uint4 *gsrc = reinterpret_cast<const uint4 *>(a.old_pop + (size_t)src * N);
        uint4 *ldst = reinterpret_cast<uint4 *>(rep_lds);
        for (uint32_t o = g; o < N / 16u; o += G) ldst[o] = live ? gsrc[o] : make_uint4(0, 0, 0, 0);
    } else if (a.mode == SWEEP_INIT_RANDOM) {
        // Site n takes word n mod 4 of Philox(n / 4, k, 0, INIT).
        for (uint32_t dd = g; dd < N / 4u; dd += G) {
            const uint4 w = philox(dd, k, 0u, DOM_INIT << 28, a.key0, a.key1);
            lds32[dd] = mulhi32(w.x, a.q) | (mulhi32(w.y, a.q) << 8) | (mulhi32(w.z, a.q) << 16) |
                        (mulhi32(w.w, a.q) << 24);
        }
    } else {
        // eq. (6): all spins alpha, alpha uniform over the q states.
        const uint4 w = philox(0u, k, 0u, DOM_GROUND << 28, a.key0, a.key1);
        const uint32_t alpha = mulhi32(w.x, a.q) * 0x01010101u;
        for (uint32_t dd = g; dd < N / 4u; dd += G) lds32[dd] = alpha;
    }
    wave_fence();

    // ---- theta checkerboard sweeps --------------------------------------
    const uint32_t theta = (a.mode == SWEEP_UPDATE) ? a.theta : 0u;
    const uint32_t H = L >> 1;                 // colour-c sites per row
    const uint32_t P = N >> 2;                 // pairs per half-sweep
    const uint32_t step2G = 2u * G;
    const uint32_t dy = step2G / H, dj = step2G % H;
    const uint32_t qm1 = a.q - 1u;
    for (uint32_t t = 0; t < theta; ++t) {
        for (uint32_t c = 0; c < 2u; ++c) {
            const uint32_t c3 = (DOM_SWEEP << 28) | (t << 1) | c;
            uint32_t y = (2u * g) / H, j0 = (2u * g) % H;
            for (uint32_t p = g; p < P; p += G) {
                const uint32_t par = (y + c) & 1u;
                const uint32_t xb = 2u * j0;                       // dword column, x0 = xb + par
                const uint32_t rowY = y * L;
                const uint32_t rowU = (y == 0 ? L - 1u : y - 1u) * L;
                const uint32_t rowD = (y == L - 1u ? 0u : y + 1u) * L;
                const uint32_t xo = par ? (xb + 4u == L ? 0u : xb + 4u) : (xb == 0u ? L - 4u : xb - 4u);
                const uint32_t D0 = lds32[(rowY + xb) >> 2];
                const uint32_t Dx = lds32[(rowY + xo) >> 2];
                const uint32_t U = lds32[(rowU + xb) >> 2];
                const uint32_t Dn = lds32[(rowD + xb) >> 2];

                // bytes x0-1, x0, x0+1, x1 = x0+2 in lo; x1+1 in b4
                const uint32_t lo = par ? D0 : __builtin_amdgcn_alignbyte(D0, Dx, 3);
                const uint32_t b4 = par ? (Dx & 0xFFu) : (D0 >> 24);
                const uint32_t sh = par << 3;
                const uint32_t Us = U >> sh, Ds = Dn >> sh;

                const uint4 w = philox(p, k, a.step, c3, a.key0, a.key1);
                const uint32_t s0 = update_site((lo >> 8) & 0xFFu, lo & 0xFFu, (lo >> 16) & 0xFFu,
                                                Us & 0xFFu, Ds & 0xFFu, w.x, w.y, qm1, Ttab);
                const uint32_t s1 = update_site(lo >> 24, (lo >> 16) & 0xFFu, b4,
                                                (Us >> 16) & 0xFFu, (Ds >> 16) & 0xFFu, w.z, w.w,
                                                qm1, Ttab);
                const uint32_t mask = 0x00FF00FFu << sh;
                const uint32_t val = (s0 | (s1 << 16)) << sh;
                lds32[(rowY + xb) >> 2] = (D0 & ~mask) | val;

                j0 += dj;
                if (j0 >= H) { j0 -= H; ++y; }
                y += dy;
            }
            wave_fence();
        }
    }

    // ---- energy (eq. (3)), histogram, store ------------------------------
    const uint32_t dpr = L >> 2;               // dwords per row
    uint32_t bonds = 0;
    for (uint32_t dd = g; dd < N / 4u; dd += G) {
        const uint32_t y = dd / dpr, xb = (dd - y * dpr) * 4u;
        const uint32_t D = lds32[dd];
        const uint32_t Dr = lds32[(y * L + (xb + 4u == L ? 0u : xb + 4u)) >> 2];
        const uint32_t Dd = lds32[((y == L - 1u ? 0u : y + 1u) * L + xb) >> 2];
        const uint32_t right = __builtin_amdgcn_alignbyte(Dr, D, 1);
        bonds += eq_bytes(D, right) + eq_bytes(D, Dd);
    }
    for (uint32_t off = G >> 1; off > 0; off >>= 1) bonds += __shfl_xor(bonds, off, 64);
    if (live) {
        if (g == 0) {
            const int32_t E = -(int32_t)bonds;
            a.E_out[k] = E;
            atomicAdd(&a.hist[(uint32_t)(E + 2 * (int32_t)N)], 1u);
        }
        uint4 *gdst = reinterpret_cast<uint4 *>(a.new_pop + (size_t)k * N);
        const uint4 *lsrc = reinterpret_cast<const uint4 *>(rep_lds);
        for (uint32_t o = g; o < N / 16u; o += G) gdst[o] = lsrc[o];
    }
}

// ---------------------------------------------------------------------------
// Workgroup helpers (1024 threads = 16 waves).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Exclusive scan of one value per thread over a 1024-thread block; returns the
// exclusive prefix and writes the total to *total.
template <typename T>
__device__ T block_exclusive_scan(T v, T *scratch /*[16]*/, T *total) {
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    T incl = v;
    for (uint32_t off = 1; off < 64; off <<= 1) {
        T n = __shfl_up(incl, off, 64);
        if (lane >= off) incl += n;
    }
    if (lane == 63) scratch[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (uint32_t w = 0; w < (blockDim.x >> 6); ++w) {
            T s = scratch[w];
            scratch[w] = run;
            run += s;
        }
        scratch[16] = run;
    }
    __syncthreads();
    T res = scratch[wave] + incl - v;
    *total = scratch[16];
    __syncthreads();
    return res;
}

// ---------------------------------------------------------------------------
// k_stats: eq. (4) sums and ln Q_{i+1} of Sec. 2 step 2 from the histogram.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_stats(StatsArgs a) {
    __shared__ int64_t s_esum[16];
    __shared__ uint64_t s_cnt[16];
    __shared__ int32_t s_min[16], s_max[16];
    __shared__ double s_w[16];
    __shared__ int32_t s_ref;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint32_t nb = a.nbins;
    const uint32_t chunk = (nb + blockDim.x - 1) / blockDim.x;
    const uint32_t b0 = tid * chunk, b1 = min(nb, b0 + chunk);

    int64_t esum = 0;
    uint64_t cnt = 0;
    int32_t bmin = 0x7fffffff, bmax = -1;
    for (uint32_t b = b0; b < b1; ++b) {
        const uint32_t h = a.hist[b];
        if (h) {
            esum += (int64_t)h * ((int32_t)b - a.two_n);
            cnt += h;
            bmin = min(bmin, (int32_t)b);
            bmax = max(bmax, (int32_t)b);
        }
    }
    esum = wave_sum(esum);
    cnt = wave_sum(cnt);
    for (int off = 32; off > 0; off >>= 1) {
        bmin = min(bmin, __shfl_xor(bmin, off, 64));
        bmax = max(bmax, __shfl_xor(bmax, off, 64));
    }
    if (lane == 0) { s_esum[wave] = esum; s_cnt[wave] = cnt; s_min[wave] = bmin; s_max[wave] = bmax; }
    __syncthreads();
    if (tid == 0) {
        int64_t E = 0; uint64_t C = 0; int32_t mn = 0x7fffffff, mx = -1;
        for (uint32_t w = 0; w < (blockDim.x >> 6); ++w) {
            E += s_esum[w]; C += s_cnt[w]; mn = min(mn, s_min[w]); mx = max(mx, s_max[w]);
        }
        a.E_sum[a.step] = E;
        a.count[a.step] = C;
        a.E_mean[a.step] = (double)E / (double)a.R_i;
        s_ref = (a.dbeta_next >= 0.0 ? mn : mx) - a.two_n;
        if (a.has_next) a.E_ref[a.step + 1] = s_ref;
    }
    __syncthreads();

    if (a.has_next) {
        const int32_t ref = s_ref;
        double acc = 0.0;
        for (uint32_t b = b0; b < b1; ++b) {
            const uint32_t h = a.hist[b];
            if (h) {
                const int32_t dd = abs((int32_t)b - a.two_n - ref);
                acc += (double)h * a.w64_next[dd];
            }
        }
        acc = wave_sum(acc);
        if (lane == 0) s_w[wave] = acc;
        __syncthreads();
        if (tid == 0) {
            double S = 0.0;
            for (uint32_t w = 0; w < (blockDim.x >> 6); ++w) S += s_w[w];
            const double lnq = -a.dbeta_next * (double)ref + log(S) - log((double)a.R_i);
            a.lnQ[a.step + 1] = lnq;
            a.mbF[a.step + 1] = a.mbF[a.step] + lnq;
        }
    }
    if (a.zero_next)
        for (uint32_t b = tid; b < nb; b += blockDim.x) a.zero_next[b] = 0u;
}

// ---------------------------------------------------------------------------
// k_weights_scan: C_j = sum_{j' <= j} W(|E_j' - E_ref|)  (one workgroup).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t weight_of(const WeightsArgs &a, int32_t ref, uint64_t j) {
    const uint32_t dd = (uint32_t)abs(a.E[j] - ref);
    return dd < a.D ? a.W[dd] : 0ull;
}

__global__ void __launch_bounds__(1024) k_weights_scan(WeightsArgs a) {
    __shared__ uint64_t scratch[17];
    const int32_t ref = *a.E_ref;
    const uint64_t n = a.R_prev;
    const uint64_t chunk = (n + blockDim.x - 1) / blockDim.x;
    const uint64_t j0 = (uint64_t)threadIdx.x * chunk, j1 = min(n, j0 + chunk);
    uint64_t local = 0;
    for (uint64_t j = j0; j < j1; ++j) local += weight_of(a, ref, j);
    uint64_t total;
    uint64_t run = block_exclusive_scan<uint64_t>(local, scratch, &total);
    for (uint64_t j = j0; j < j1; ++j) {
        run += weight_of(a, ref, j);
        a.C[j] = run;
    }
}

// ---------------------------------------------------------------------------
// k_sample: draw kk picks the first j with C_j > floor(x_kk * S / 2^64).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_sample(SampleArgs a) {
    const uint64_t kk = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (kk >= a.n_new) return;
    const uint64_t S = a.C[a.R_prev - 1];
    const uint4 w = philox((uint32_t)kk, 0u, a.step, DOM_RESAMPLE << 28, a.key0, a.key1);
    const uint64_t x = ((uint64_t)w.y << 32) | (uint64_t)w.x;
    const uint64_t u = __umul64hi(x, S);
    uint64_t lo = 0, hi = a.R_prev - 1;
    while (lo < hi) {
        const uint64_t mid = lo + ((hi - lo) >> 1);
        if (a.C[mid] > u) hi = mid; else lo = mid + 1;
    }
    atomicAdd(&a.r[lo], 1u);
}

// ---------------------------------------------------------------------------
// k_slotmap: anc[o_j + c] = j for c < r_j, o = exclusive scan of r (one workgroup).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_slotmap(SlotmapArgs a) {
    __shared__ uint64_t scratch[17];
    const uint64_t n = a.R_prev;
    const uint64_t chunk = (n + blockDim.x - 1) / blockDim.x;
    const uint64_t j0 = (uint64_t)threadIdx.x * chunk, j1 = min(n, j0 + chunk);
    uint64_t local = 0;
    for (uint64_t j = j0; j < j1; ++j) local += a.r[j];
    uint64_t total;
    uint64_t o = block_exclusive_scan<uint64_t>(local, scratch, &total);
    for (uint64_t j = j0; j < j1; ++j) {
        const uint32_t rj = a.r[j];
        for (uint32_t c = 0; c < rj; ++c)
            if (o + c < a.anc_cap) a.anc[o + c] = (uint32_t)j;
        o += rj;
        if (a.counts_last) a.counts_last[j] = rj;
        a.r[j] = 0u;
    }
}

__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace

void sweep_shape(uint32_t L, uint32_t *G_log2, uint32_t *waves_per_block) {
    const uint32_t P = (L * L) / 4u;
    uint32_t gl = 2;
    while (gl < 6 && (1u << (gl + 1)) <= P) ++gl;
    *G_log2 = gl;
    const uint32_t N = L * L;
    const uint32_t rpw = 64u >> gl;
    uint32_t wpb = 4;
    while (wpb > 1 && (size_t)wpb * rpw * N > 32768u) wpb >>= 1;
    *waves_per_block = wpb;
}

size_t sweep_lds_bytes(uint32_t N, uint32_t G_log2, uint32_t waves_per_block) {
    return 128u + (size_t)waves_per_block * (64u >> G_log2) * N;
}

size_t max_lds_per_block(int device) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess)
        return 65536;
    return (size_t)v;
}

hipError_t launch_sweep(const SweepArgs &a, hipStream_t s) {
    const uint32_t rpw = 64u >> a.G_log2;
    const uint64_t per_block = (uint64_t)a.waves_per_block * rpw;
    const uint64_t blocks = (a.R_new + per_block - 1) / per_block;
    if (blocks == 0) return hipSuccess;
    const size_t lds = sweep_lds_bytes(a.N, a.G_log2, a.waves_per_block);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sweep),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_sweep, dim3((uint32_t)blocks), dim3(64u * a.waves_per_block), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_stats(const StatsArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_stats, dim3(1), dim3(1024), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_weights_scan(const WeightsArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_weights_scan, dim3(1), dim3(1024), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sample(const SampleArgs &a, hipStream_t s) {
    const uint64_t blocks = (a.n_new + 255) / 256;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sample, dim3((uint32_t)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_slotmap(const SlotmapArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_slotmap, dim3(1), dim3(1024), 0, s, a);
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
