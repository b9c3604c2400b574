// HIP kernels for gfx950 (CDNA4): gate-sweep passes, gather + FP64 path sum.
//
// Pass kernel: one wave64 owns a tile of 64 * 2^R amplitudes (lane bits =
// the 6 lowest extended bits, R register bits = chosen qubits, the rest
// from the tile index).  It loads the tile once, applies a whole list of
// gates (register tier, lane-shuffle tier, bitmask diagonal groups) and
// stores it once, so one HBM round trip covers many gates.  Loads of one
// register index by the 64 lanes are 64 consecutive complex values (512 B
// in complex64), i.e. whole cache lines.
#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_reduce.hpp>
#include <rocprim/device/device_select.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

#include "kernels.hpp"
#include "pass_dev.hpp"

namespace sf {

template <typename T, int R, bool FLIP, bool ZSKIP = false>
__global__ __launch_bounds__(256) SF_PASS_OCCUPANCY void pass_kernel(PassArgs a)
{
    pass_body<T, R, FLIP, ZSKIP>(a, blockIdx.x, gridDim.x);
}

// Two independent passes in one launch (block A's and block B's pass of a tree level): the
// first grid0 workgroups run a0, the rest a1.  The choice is per workgroup, so every wave
// takes one branch.
template <typename T, int R, bool FLIP, bool ZSKIP = false>
__global__ __launch_bounds__(256) SF_PASS_OCCUPANCY void pass_kernel_pair(PassArgs a0, PassArgs a1, uint32_t grid0)
{
    if (blockIdx.x < grid0) pass_body<T, R, FLIP, ZSKIP>(a0, blockIdx.x, grid0);
    else pass_body<T, R, FLIP, ZSKIP>(a1, blockIdx.x - grid0, gridDim.x - grid0);
}

template <typename T, bool FLIP>
static hipError_t launch_pass_pair_t(int R, const PassArgs &a0, unsigned g0, const PassArgs &a1, unsigned g1,
                                     hipStream_t s)
{
    const unsigned grid = g0 + g1;
    switch (R) {
    case 0: pass_kernel_pair<T, 0, FLIP><<<grid, 256, 0, s>>>(a0, a1, g0); break;
    case 1: pass_kernel_pair<T, 1, FLIP><<<grid, 256, 0, s>>>(a0, a1, g0); break;
    case 2: pass_kernel_pair<T, 2, FLIP><<<grid, 256, 0, s>>>(a0, a1, g0); break;
    case 3: pass_kernel_pair<T, 3, FLIP><<<grid, 256, 0, s>>>(a0, a1, g0); break;
    case 4: pass_kernel_pair<T, 4, FLIP><<<grid, 256, 0, s>>>(a0, a1, g0); break;
    case 5: if constexpr (sizeof(T) == 4) { pass_kernel_pair<T, 5, FLIP><<<grid, 256, 0, s>>>(a0, a1, g0); break; }
            return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// The zero-skipping variants exist for the complex64 passes without flips at R = 4 and 5 (the
// widths the tuner uses); other passes ignore the zero list, which only ever saves reads.
static bool zskip_variant(bool zskip, bool fp64, int R, bool flips)
{
    return zskip && !fp64 && !flips && (R == 4 || R == 5);
}

hipError_t launch_pass_pair(bool fp64, int R, bool flips, bool zskip, const PassArgs &a0, unsigned grid0,
                            const PassArgs &a1, unsigned grid1, hipStream_t s)
{
    if (grid0 == 0 || grid1 == 0) return hipErrorInvalidValue;
    if (zskip_variant(zskip, fp64, R, flips)) {
        if (R == 5) pass_kernel_pair<float, 5, false, true><<<grid0 + grid1, 256, 0, s>>>(a0, a1, grid0);
        else pass_kernel_pair<float, 4, false, true><<<grid0 + grid1, 256, 0, s>>>(a0, a1, grid0);
        return hipGetLastError();
    }
    if (flips)
        return fp64 ? launch_pass_pair_t<double, true>(R, a0, grid0, a1, grid1, s)
                    : launch_pass_pair_t<float, true>(R, a0, grid0, a1, grid1, s);
    return fp64 ? launch_pass_pair_t<double, false>(R, a0, grid0, a1, grid1, s)
                : launch_pass_pair_t<float, false>(R, a0, grid0, a1, grid1, s);
}

template <typename T, bool FLIP>
static hipError_t launch_pass_t(int R, const PassArgs &a, unsigned grid, hipStream_t s)
{
    switch (R) {
    case 0: pass_kernel<T, 0, FLIP><<<grid, 256, 0, s>>>(a); break;
    case 1: pass_kernel<T, 1, FLIP><<<grid, 256, 0, s>>>(a); break;
    case 2: pass_kernel<T, 2, FLIP><<<grid, 256, 0, s>>>(a); break;
    case 3: pass_kernel<T, 3, FLIP><<<grid, 256, 0, s>>>(a); break;
    case 4: pass_kernel<T, 4, FLIP><<<grid, 256, 0, s>>>(a); break;
    case 5: if constexpr (sizeof(T) == 4) { pass_kernel<T, 5, FLIP><<<grid, 256, 0, s>>>(a); break; }
            return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pass(bool fp64, int R, bool flips, bool zskip, const PassArgs &a, unsigned grid, hipStream_t s)
{
    if (zskip_variant(zskip, fp64, R, flips)) {
        if (R == 5) pass_kernel<float, 5, false, true><<<grid, 256, 0, s>>>(a);
        else pass_kernel<float, 4, false, true><<<grid, 256, 0, s>>>(a);
        return hipGetLastError();
    }
    if (flips)
        return fp64 ? launch_pass_t<double, true>(R, a, grid, s) : launch_pass_t<float, true>(R, a, grid, s);
    return fp64 ? launch_pass_t<double, false>(R, a, grid, s) : launch_pass_t<float, false>(R, a, grid, s);
}

// ---------------------------------------------------------------- chained passes

// Grid barrier of a cooperative launch.  *count only grows during a call: the barrier after
// phase i of a chain waits until it reaches base + (i + 1) * gridDim.x, base being what the
// call's earlier chains added.  Every thread first makes its stores visible device-wide (a
// release fence at agent scope, which covers the other XCDs' L2s); one thread per workgroup
// arrives and waits; after the wait every thread acquires at agent scope before it reads what
// other workgroups wrote.  The wait is bounded (2^22 polls of at least one sleep each, between
// about 0.2 s and a few seconds): past it *err gets bit 1 and the workgroup goes on, so a
// barrier that cannot complete ends the call with an error instead of hanging it.
__device__ __forceinline__ void chain_barrier(uint64_t *count, uint64_t target, int *err)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(count, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t polls = 0;
        while (__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++polls == (1u << 22)) {
                __hip_atomic_fetch_or(err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// A chain of passes (ChainPhase): the workgroups run phase i's pass (or the two passes of a
// pair, split between them) and meet at a grid barrier before phase i + 1.  pass_body stages each
// program in LDS; the barrier's workgroup syncs keep a phase's staging behind the last reads of
// the one before.
template <typename T, int R, bool FLIP, bool ZSKIP>
__global__ __launch_bounds__(256) SF_PASS_OCCUPANCY void pass_chain_kernel(const PassArgs *__restrict__ args,
                                                         const ChainPhase *__restrict__ phases, uint32_t n_phases,
                                                         uint64_t *__restrict__ count, uint64_t base,
                                                         int *__restrict__ err)
{
    for (uint32_t i = 0; i < n_phases; ++i) {
        const ChainPhase ph = phases[i];
        using Ref = const PassArgs &;
        if (ph.n == 1) pass_body<T, R, FLIP, ZSKIP, Ref>(args[ph.first], blockIdx.x, gridDim.x);
        else if (blockIdx.x < ph.split) pass_body<T, R, FLIP, ZSKIP, Ref>(args[ph.first], blockIdx.x, ph.split);
        else pass_body<T, R, FLIP, ZSKIP, Ref>(args[ph.first + 1], blockIdx.x - ph.split, gridDim.x - ph.split);
        if (i + 1 < n_phases) chain_barrier(count, base + (uint64_t)(i + 1) * gridDim.x, err);
    }
}

// the chain kernel of a variant, or nullptr
static const void *chain_kernel_ptr(bool fp64, int R, bool flips, bool zskip)
{
    if (zskip_variant(zskip, fp64, R, flips))
        return R == 5 ? (const void *)pass_chain_kernel<float, 5, false, true>
                      : (const void *)pass_chain_kernel<float, 4, false, true>;
#define SF_CHAIN_CASES(T, F)                                                    \
    switch (R) {                                                                \
    case 0: return (const void *)pass_chain_kernel<T, 0, F, false>;             \
    case 1: return (const void *)pass_chain_kernel<T, 1, F, false>;             \
    case 2: return (const void *)pass_chain_kernel<T, 2, F, false>;             \
    case 3: return (const void *)pass_chain_kernel<T, 3, F, false>;             \
    case 4: return (const void *)pass_chain_kernel<T, 4, F, false>;             \
    default: break;                                                             \
    }
    if (fp64) {
        if (flips) { SF_CHAIN_CASES(double, true) } else { SF_CHAIN_CASES(double, false) }
        return nullptr;
    }
    if (flips) { SF_CHAIN_CASES(float, true) } else { SF_CHAIN_CASES(float, false) }
#undef SF_CHAIN_CASES
    if (R == 5) return flips ? (const void *)pass_chain_kernel<float, 5, true, false>
                             : (const void *)pass_chain_kernel<float, 5, false, false>;
    return nullptr;
}

bool chain_zskip(bool fp64, int R, bool flips)
{
    return zskip_variant(true, fp64, R, flips);
}

hipError_t chain_max_grid(bool fp64, int R, bool flips, bool zskip, unsigned *grid)
{
    const void *k = chain_kernel_ptr(fp64, R, flips, zskip);
    if (!k) return hipErrorInvalidValue;
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, 0);
    if (e != hipSuccess) return e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    *grid = (unsigned)(per_cu > 0 ? per_cu : 0) * (unsigned)cus;
    return hipSuccess;
}

hipError_t launch_pass_chain(bool fp64, int R, bool flips, bool zskip, const PassArgs *args, const ChainPhase *phases,
                             uint32_t n_phases, uint64_t *count, uint64_t base, int *err, unsigned grid, hipStream_t s)
{
    const void *k = chain_kernel_ptr(fp64, R, flips, zskip);
    if (!k || grid == 0 || n_phases == 0) return hipErrorInvalidValue;
    void *kargs[] = {(void *)&args, (void *)&phases, (void *)&n_phases, (void *)&count, (void *)&base, (void *)&err};
    return hipLaunchCooperativeKernel(k, dim3(grid), dim3(256), kargs, 0, s);
}

// ---------------------------------------------------------------- dense block on matrix cores

typedef float f32x16 __attribute__((ext_vector_type(16)));

// out = U in for every column: a 32x32 real matrix times the real embedding [Re; Im] of
// the 16 block amplitudes of 32 columns, with v_mfma_f32_32x32x2f32 (K = 2 per step).
// Operand layout of that instruction: A[i][k] in lane i + 32k, B[k][j] in lane j + 32k,
// D[i][j] in lane j + 32*((i/4)%2), register 4*(i/8) + i%4.  Lane j + 32h therefore loads
// the complex rows 2r + h (r = 0..7) of column j: for step kk the B value is the real part
// of its row r = kk (kk < 8) or the imaginary part of row r = kk - 8, with no cross-lane
// exchange.  The accumulator holds real rows 8*(r/4) + 4h + r%4: registers 0..7 are real
// parts and 8..15 the imaginary parts of the complex rows 8*(r/4) + 4h + r%4.
__global__ __launch_bounds__(256) void dense_kernel(DenseArgs a)
{
    const unsigned lane = threadIdx.x & 63u;
    const unsigned h = lane >> 5, col = lane & 31u;
    const uint32_t wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * 4u;
    float am[16];
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) am[kk] = a.mat[col * 32u + 2u * kk + h];
    uint64_t bs[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) bs[t] = (uint64_t)1 << a.bpos[t];
    auto rowoff = [&](unsigned r) {
        return ((r & 1u) ? bs[0] : 0u) + ((r & 2u) ? bs[1] : 0u) + ((r & 4u) ? bs[2] : 0u) + ((r & 8u) ? bs[3] : 0u);
    };
    const float sc = (float)a.rescale;
    for (uint64_t g = (uint64_t)blockIdx.x * 4u + wid; g < a.n_groups; g += nwaves) {
        uint64_t et = g << 5;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int p = a.bpos[t];
            et = ((et >> p) << (p + 1)) | (et & (((uint64_t)1 << p) - 1u));
        }
        // 32 columns of padding slots (the 5 lowest extended bits are slot bits when p >= 5)
        if (a.slots_real && (et & ((((uint64_t)1) << a.p) - 1u)) >= a.slots_real) continue;
        const float2 *src = (const float2 *)a.src + et + col;
        float2 v[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r] = src[rowoff(2u * r + h)];
        f32x16 acc = {};
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const float b = kk < 8 ? v[kk].x : v[kk - 8].y;
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(am[kk], b, acc, 0, 0, 0);
        }
        float2 *dst = (float2 *)a.dst + et + col;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const unsigned row = 8u * (r / 4) + 4u * h + (r % 4);
            float2 o;
            o.x = acc[r] * sc;
            o.y = acc[r + 8] * sc;
            dst[rowoff(row)] = o;
        }
    }
}

hipError_t launch_dense(const DenseArgs &a, unsigned grid, hipStream_t s)
{
    dense_kernel<<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- gather + FP64 path sum

// amp[j] += scale * sum_{slot < n_slots} A[x_A(j) * P + slot] * B[x_B(j) * P + slot]
// Lanes of a wave split over slots (L = min(P, 64) lanes per bitstring);
// products and sums are formed in FP64 (a product of two FP32 values is
// exact in FP64).  Each bitstring has one owner, so no atomics are needed.
template <typename T>
__global__ __launch_bounds__(256) void gather_kernel(GatherArgs g)
{
    using C = typename Cplx<T>::type;
    const int lane = threadIdx.x & 63;
    const uint32_t P = 1u << g.p;
    const uint32_t L = P < 64u ? P : 64u;
    const uint32_t G = 64u / L;
    const uint64_t wave = (uint64_t)xcd_block(blockIdx.x, gridDim.x) * 4u + (threadIdx.x >> 6);
    const uint64_t jj = wave * G + (uint32_t)lane / L;
    const uint32_t sl = (uint32_t)lane % L;
    // bitstrings are visited in x_A order when `order` is given, so waves that share a
    // block-A row run close together, on one XCD, and find it in its L2
    const uint64_t j = (jj < g.n_bits && g.order) ? (uint64_t)g.order[jj] : jj;
    double re = 0.0, im = 0.0;
    if (j < g.n_bits) {
        const C *ra = (const C *)g.a + ((uint64_t)g.xa[j] << g.p);
        const C *rb = (const C *)g.b + ((uint64_t)g.xb[j] << g.p);
        for (uint32_t s = sl; s < g.n_slots; s += L) {
            const C x = ra[s], y = rb[s];
            const double xr = x.x, xi = x.y, yr = y.x, yi = y.y;
            re += xr * yr - xi * yi;
            im += xr * yi + xi * yr;
        }
    }
    for (uint32_t m = 1; m < L; m <<= 1) {
        re += __shfl_xor(re, (int)m);
        im += __shfl_xor(im, (int)m);
    }
    if (j < g.n_bits && sl == 0) {
        double *o = g.acc + 2 * j;
        o[0] += g.scale_re * re - g.scale_im * im;
        o[1] += g.scale_re * im + g.scale_im * re;
    }
}

hipError_t launch_gather(bool fp64, const GatherArgs &g, hipStream_t s)
{
    if (g.n_bits == 0) return hipSuccess;
    const uint64_t P = (uint64_t)1 << g.p;
    const uint64_t L = P < 64 ? P : 64;
    const uint64_t per_wave = 64 / L;
    const uint64_t waves = (g.n_bits + per_wave - 1) / per_wave;
    const uint64_t blocks = ((waves + 3) / 4 + 7) / 8 * 8;   // a multiple of 8 (xcd_block)
    if (fp64) gather_kernel<double><<<(unsigned)blocks, 256, 0, s>>>(g);
    else gather_kernel<float><<<(unsigned)blocks, 256, 0, s>>>(g);
    return hipGetLastError();
}

// ---------------------------------------------------------------- x_A ordering of bitstrings

__global__ void iota_kernel(uint32_t *p, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (uint32_t)i;
}

hipError_t sort_by_key_temp_bytes(uint64_t n, size_t *bytes)
{
    *bytes = 0;
    return rocprim::radix_sort_pairs(nullptr, *bytes, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                                     (const uint32_t *)nullptr, (uint32_t *)nullptr, (size_t)n, 0u, 32u);
}

hipError_t launch_order_by_key(const uint32_t *keys, uint32_t *keys_sorted, uint32_t *idx, uint32_t *order,
                               uint64_t n, int key_bits, void *temp, size_t temp_bytes, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    iota_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(idx, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return rocprim::radix_sort_pairs(temp, temp_bytes, keys, keys_sorted, idx, order, (size_t)n, 0u,
                                     (unsigned)(key_bits < 1 ? 1 : key_bits), s);
}

// ---------------------------------------------------------------- small helpers

__device__ __forceinline__ uint32_t pext64(uint64_t x, uint64_t m)
{
    uint32_t r = 0;
    int k = 0;
    while (m) {
        const int q = __ffsll((long long)m) - 1;
        r |= (uint32_t)((x >> q) & 1u) << k;
        ++k;
        m &= m - 1;
    }
    return r;
}

__global__ void pext_kernel(const uint64_t *bits, uint64_t n, uint64_t ma, uint64_t mb, uint64_t all,
                            uint32_t *xa, uint32_t *xb, int *bad)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t x = bits[i];
    if (x & ~all) *bad = 1;
    xa[i] = pext64(x, ma);
    xb[i] = pext64(x, mb);
}

hipError_t launch_pext(const uint64_t *bits, uint64_t n, uint64_t mask_a, uint64_t mask_b,
                       uint64_t all, uint32_t *xa, uint32_t *xb, int *bad, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    pext_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(bits, n, mask_a, mask_b, all, xa, xb, bad);
    return hipGetLastError();
}

// ---------------------------------------------------------------- leaf fold + FP64 path sum

__device__ __forceinline__ uint32_t pext32(uint32_t x, uint32_t m)
{
    uint32_t r = 0;
    int k = 0;
    while (m) {
        const int q = __ffs((int)m) - 1;
        r |= ((x >> q) & 1u) << k;
        ++k;
        m &= m - 1;
    }
    return r;
}

// amp[j] += scale * sum_{slot < n_slots} sum_{i in child_mask[slot]} c_A[i] * WHT(c_B)[i]
// with c_h[i] read from level L-F as described with FoldArgs.  WIDE: one bitstring per wave,
// lanes over slots (P >= 64), so every per-bitstring quantity is wave-uniform; else P lanes per
// bitstring.  Per slot, block B's 2^NB values are formed and transformed first, then block A's
// are streamed against them.  The folded gates are applied in the state precision, the
// products and sums over slots in FP64.
//
// With NB >= 4 there are too many per-bitstring constants (2 x 2^NB entries of V and row
// offsets) to keep in registers: the V entries of each wave's bitstring go to LDS and are read
// back every iteration, and the row offsets are re-added from the per-bit strides every
// iteration (the empty asm statements only hide loop invariance from the compiler).
// At most 4 waves per SIMD (2 with NB >= 4): the register budget then lets the scheduler issue
// every row load of an iteration before the first use (with a tighter budget it serialises them).
template <typename T, int NB, bool WIDE, bool MASKED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, NB >= 4 ? 2 : 4))) void fold_kernel(FoldArgs g)
{
    using C = typename Cplx<T>::type;
    constexpr int V = 1 << NB;
    constexpr bool LDSV = WIDE && NB >= 4;
    __shared__ C sv[LDSV ? 4 * 2 * V : 1];
    const int lane = threadIdx.x & 63;
    const uint32_t wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t P = 1u << g.p;
    const uint32_t L = WIDE ? 64u : P;
    const uint32_t G = 64u / L;
    const uint64_t wave = (uint64_t)xcd_block(blockIdx.x, gridDim.x) * 4u + wid;
    const uint64_t jj = wave * G + (uint32_t)lane / L;
    const uint32_t sl = (uint32_t)lane % L;
    uint64_t j = jj < g.n_bits ? (uint64_t)g.order[jj] : g.n_bits;
    if (WIDE) {
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)j);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(j >> 32));
        j = ((uint64_t)hi << 32) | lo;
    }
    double re = 0.0, im = 0.0;
    if (j < g.n_bits) {
        const C *base[2];             // row (x & ~smask) of each block
        const double *tr[2];          // table row of x_T
        uint32_t xd[2];               // x at the branch qubits outside S, as path bits
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const FoldHalf &f = g.h[h];
            const uint32_t x = h ? g.xb[j] : g.xa[j];
            tr[h] = f.tab + 2 * ((uint64_t)pext32(x, f.tmask) << f.n_s);
            base[h] = (const C *)f.par + ((uint64_t)(x & ~f.smask) << g.p);
            uint32_t d = 0;
#pragma unroll
            for (int u = 0; u < NB; ++u)
                if ((f.dsel >> u) & 1u) d |= ((x >> f.bq[u]) & 1u) << u;
            xd[h] = d;
        }
        // V entry of virtual slot i: zero if i disagrees with x outside S
        auto vval = [&](int h, int i) -> C {
            const FoldHalf &f = g.h[h];
            C v;
            v.x = v.y = T(0);
            if (((uint32_t)i & f.dsel) == xd[h]) {
                uint32_t y = 0;
                for (int u = 0; u < NB; ++u)
                    if (!((f.dsel >> u) & 1u)) y |= (((uint32_t)i >> u) & 1u) << f.ypos[u];
                v.x = (T)tr[h][2 * y];
                v.y = (T)tr[h][2 * y + 1];
            }
            return v;
        };
        C *wv = sv + (LDSV ? wid * 2 * V : 0);
        if (LDSV) {
            if (lane < V) {
                wv[lane] = vval(0, lane);
                wv[V + lane] = vval(1, lane);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        for (uint32_t s = sl; s < g.n_slots; s += L) {
            uint32_t st[2][NB];       // row strides per path bit
            int voff = 0;
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int u = 0; u < NB; ++u) {
                    st[h][u] = g.h[h].sstride[u];
                    if (NB >= 4) asm volatile("" : "+s"(st[h][u]));
                }
            if (LDSV) asm volatile("" : "+v"(voff));
            auto row_of = [&](int h, int i) -> uint64_t {
                uint32_t r = 0;
#pragma unroll
                for (int u = 0; u < NB; ++u)
                    if ((i >> u) & 1) r += st[h][u];
                return (uint64_t)r << g.p;
            };
            // a virtual slot that disagrees with x contributes zero; its row is the row of the
            // slot that agrees (rows depend on the S bits only), so every load is in bounds
            C b[V];
#pragma unroll
            for (int i = 0; i < V; ++i) {
                const C t = base[1][row_of(1, i) + s];
                const C v = LDSV ? wv[V + i + voff] : vval(1, i);
                b[i].x = v.x * t.x - v.y * t.y;
                b[i].y = v.x * t.y + v.y * t.x;
            }
            // block B: the descendant's Z^b signs summed over the input branch bits
#pragma unroll
            for (int stp = 1; stp < V; stp <<= 1)
#pragma unroll
                for (int i = 0; i < V; ++i)
                    if (!(i & stp)) {
                        const C u = b[i], w = b[i | stp];
                        b[i].x = u.x + w.x;
                        b[i].y = u.y + w.y;
                        b[i | stp].x = u.x - w.x;
                        b[i | stp].y = u.y - w.y;
                    }
            const uint32_t m = MASKED ? g.child_mask[s] : 0xffffffffu;
#pragma unroll
            for (int i = 0; i < V; ++i) {
                const C t = base[0][row_of(0, i) + s];
                const C v = LDSV ? wv[i + voff] : vval(0, i);
                const double ar = (double)(v.x * t.x - v.y * t.y), ai = (double)(v.x * t.y + v.y * t.x);
                const double br = b[i].x, bi = b[i].y;
                const double pr = ar * br - ai * bi, pi = ar * bi + ai * br;
                if (MASKED) {
                    const bool use = (m >> i) & 1u;    // a select, not a branch
                    re += use ? pr : 0.0;
                    im += use ? pi : 0.0;
                } else {
                    re += pr;
                    im += pi;
                }
            }
        }
    }
    for (uint32_t mm = 1; mm < L; mm <<= 1) {
        re += __shfl_xor(re, (int)mm);
        im += __shfl_xor(im, (int)mm);
    }
    if (j < g.n_bits && sl == 0) {
        double *o = g.acc + 2 * j;
        o[0] += g.scale_re * re - g.scale_im * im;
        o[1] += g.scale_re * im + g.scale_im * re;
    }
}

template <typename T, int NB>
static void fold_launch(const FoldArgs &g, unsigned blocks, bool wide, hipStream_t s)
{
    if (g.all_children) {
        if (wide) fold_kernel<T, NB, true, false><<<blocks, 256, 0, s>>>(g);
        else fold_kernel<T, NB, false, false><<<blocks, 256, 0, s>>>(g);
    } else {
        if (wide) fold_kernel<T, NB, true, true><<<blocks, 256, 0, s>>>(g);
        else fold_kernel<T, NB, false, true><<<blocks, 256, 0, s>>>(g);
    }
}

hipError_t launch_fold(bool fp64, int nb, const FoldArgs &g, hipStream_t s)
{
    if (g.n_bits == 0) return hipSuccess;
    if (nb < 1 || nb > 5 || g.p < 0 || g.p > 31 || !g.order || !g.child_mask) return hipErrorInvalidValue;
    const uint64_t P = (uint64_t)1 << g.p;
    const bool wide = P >= 64;
    const uint64_t per_wave = wide ? 1 : 64 / P;
    const uint64_t waves = (g.n_bits + per_wave - 1) / per_wave;
    const unsigned blocks = (unsigned)(((waves + 3) / 4 + 7) / 8 * 8);   // a multiple of 8 (xcd_block)
    switch (nb) {
    case 1: fp64 ? fold_launch<double, 1>(g, blocks, wide, s) : fold_launch<float, 1>(g, blocks, wide, s); break;
    case 2: fp64 ? fold_launch<double, 2>(g, blocks, wide, s) : fold_launch<float, 2>(g, blocks, wide, s); break;
    case 3: fp64 ? fold_launch<double, 3>(g, blocks, wide, s) : fold_launch<float, 3>(g, blocks, wide, s); break;
    case 4: fp64 ? fold_launch<double, 4>(g, blocks, wide, s) : fold_launch<float, 4>(g, blocks, wide, s); break;
    default: fp64 ? fold_launch<double, 5>(g, blocks, wide, s) : fold_launch<float, 5>(g, blocks, wide, s); break;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- general fold + FP64 path sum

// amp[j] += scale * sum_{slot < n_slots} sum_{b in child_mask[slot]} w_A[b] * WHT(w_B)[b] with w_h
// formed from 2^|S'| rows of the level the gather reads (GFoldArgs).  WIDE: one bitstring per
// wave, lanes over slots (P >= 64); else P lanes per bitstring, 64 / P bitstrings per wave.  Per
// slot the 2^NB accumulators of block B are formed and transformed, then those of block A; each
// round r loads 2^NB rows, all in flight before their first use.  The column patterns are
// ordered branch bits first, so every accumulator index is a compile-time constant.  Products
// with V and the sums over column patterns run in the state precision (the work of the gates the
// fold replaces), the products c_A c_B and all sums over slots in FP64.
template <typename T, int NB, bool WIDE, bool MASKED, bool DEFER>
__global__ __launch_bounds__(256) void gfold_kernel(GFoldArgs g)
{
    using C = typename Cplx<T>::type;
    constexpr int V = 1 << NB;
    const int lane = threadIdx.x & 63;
    const uint32_t wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t P = 1u << g.p;
    const uint32_t L = WIDE ? 64u : P;
    const uint32_t G = 64u / L;
    const uint64_t wave = (uint64_t)xcd_block(blockIdx.x, gridDim.x) * 4u + wid;
    const uint64_t jj = wave * G + (uint32_t)lane / L;
    const uint32_t sl = (uint32_t)lane % L;
    uint64_t j = jj < g.n_bits ? (uint64_t)g.order[jj] : g.n_bits;
    if (WIDE) {
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)j);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(j >> 32));
        j = ((uint64_t)hi << 32) | lo;
    }
    double re = 0.0, im = 0.0;
    if (j < g.n_bits) {
        const C *base[2];             // row (x & ~smask) of each block
        const C *trow[2];             // table row of x_T'
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const GFoldHalf &f = g.h[h];
            const uint32_t x = h ? g.xb[j] : g.xa[j];
            trow[h] = (const C *)f.tab + ((uint64_t)pext32(x, f.tmask) << f.n_s);
            base[h] = (const C *)f.par + ((uint64_t)(x & ~f.smask) << g.p);
        }
        // deferred block-A level: x_A without S' and the projected qubits, and x at those qubits
        const uint32_t xa_rest = DEFER ? g.xa[j] & ~g.h[0].smask & ~g.h[0].dmask : 0u;
        const uint32_t xa_d = DEFER ? pext32(g.xa[j], g.h[0].dmask) : 0u;
        // w[b] = sum_r V[x_T', b | r << NB] * row(b | r << NB)[slot] for one block; bs points at
        // the slot's row (x & ~smask), consecutive rows are 2^sh elements apart
        auto accumulate = [&](const GFoldHalf &f, const C *bs, int sh, const C *tr, C (&w)[V]) {
#pragma unroll
            for (int b = 0; b < V; ++b) { w[b].x = T(0); w[b].y = T(0); }
            const uint32_t nr = 1u << f.n_rest;
            for (uint32_t r = 0; r < nr; ++r) {
                C t[V];
#pragma unroll
                for (int b = 0; b < V; ++b) t[b] = bs[(uint64_t)f.off[b | (r << NB)] << sh];
#pragma unroll
                for (int b = 0; b < V; ++b) {
                    const C v = tr[b | (r << NB)];
                    w[b].x += v.x * t[b].x - v.y * t[b].y;
                    w[b].y += v.x * t[b].y + v.y * t[b].x;
                }
            }
        };
        for (uint32_t s = sl; s < g.n_slots; s += L) {
            C wb[V], wa[V];
            accumulate(g.h[1], base[1] + s, g.p, trow[1], wb);
            if (DEFER) {
                const GFoldHalf &f = g.h[0];
                const C *bs = (const C *)f.par + ((uint64_t)(xa_rest | f.dsub[s]) << f.p_par) + f.par_slot[s];
                accumulate(f, bs, f.p_par, trow[0], wa);
                const C fac = ((const C *)f.dfac)[((uint64_t)s << f.nd) + xa_d];
#pragma unroll
                for (int b = 0; b < V; ++b) {
                    const T x = wa[b].x, y = wa[b].y;
                    wa[b].x = x * fac.x - y * fac.y;
                    wa[b].y = x * fac.y + y * fac.x;
                }
            } else {
                accumulate(g.h[0], base[0] + s, g.p, trow[0], wa);
            }
            // block B: the descendant's Z^b signs summed over the column patterns' branch bits
#pragma unroll
            for (int stp = 1; stp < V; stp <<= 1)
#pragma unroll
                for (int i = 0; i < V; ++i)
                    if (!(i & stp)) {
                        const C u = wb[i], w = wb[i | stp];
                        wb[i].x = u.x + w.x;
                        wb[i].y = u.y + w.y;
                        wb[i | stp].x = u.x - w.x;
                        wb[i | stp].y = u.y - w.y;
                    }
            const uint32_t m = MASKED ? g.child_mask[s] : 0xffffffffu;
#pragma unroll
            for (int b = 0; b < V; ++b) {
                const double ar = wa[b].x, ai = wa[b].y, br = wb[b].x, bi = wb[b].y;
                const double pr = ar * br - ai * bi, pi = ar * bi + ai * br;
                if (MASKED) {
                    const bool use = (m >> b) & 1u;    // a select, not a branch
                    re += use ? pr : 0.0;
                    im += use ? pi : 0.0;
                } else {
                    re += pr;
                    im += pi;
                }
            }
        }
    }
    for (uint32_t mm = 1; mm < L; mm <<= 1) {
        re += __shfl_xor(re, (int)mm);
        im += __shfl_xor(im, (int)mm);
    }
    if (j < g.n_bits && sl == 0) {
        double *o = g.acc + 2 * j;
        o[0] += g.scale_re * re - g.scale_im * im;
        o[1] += g.scale_re * im + g.scale_im * re;
    }
}

template <typename T, int NB, bool DEFER>
static void gfold_launch_d(const GFoldArgs &g, unsigned blocks, bool wide, hipStream_t s)
{
    if (g.all_children) {
        if (wide) gfold_kernel<T, NB, true, false, DEFER><<<blocks, 256, 0, s>>>(g);
        else gfold_kernel<T, NB, false, false, DEFER><<<blocks, 256, 0, s>>>(g);
    } else {
        if (wide) gfold_kernel<T, NB, true, true, DEFER><<<blocks, 256, 0, s>>>(g);
        else gfold_kernel<T, NB, false, true, DEFER><<<blocks, 256, 0, s>>>(g);
    }
}

template <typename T, int NB>
static void gfold_launch(const GFoldArgs &g, unsigned blocks, bool wide, hipStream_t s)
{
    if (g.h[0].par_slot) gfold_launch_d<T, NB, true>(g, blocks, wide, s);
    else gfold_launch_d<T, NB, false>(g, blocks, wide, s);
}

hipError_t launch_gfold(bool fp64, int nb, const GFoldArgs &g, hipStream_t s)
{
    if (g.n_bits == 0) return hipSuccess;
    if (nb < 1 || nb > kMaxGFoldBits || g.p < 0 || g.p > 31 || !g.order || !g.child_mask) return hipErrorInvalidValue;
    for (int h = 0; h < 2; ++h)
        if (!g.h[h].par || !g.h[h].tab || !g.h[h].off || g.h[h].n_rest < 0 || g.h[h].n_s != nb + g.h[h].n_rest)
            return hipErrorInvalidValue;
    if (g.h[1].par_slot) return hipErrorInvalidValue;   // only block A's level is deferred
    if (g.h[0].par_slot && (!g.h[0].dsub || !g.h[0].dfac || g.h[0].p_par < 0 || g.h[0].p_par > 31 ||
                            g.h[0].nd < 1 || g.h[0].nd > 4 || (g.h[0].dmask & g.h[0].smask)))
        return hipErrorInvalidValue;
    const uint64_t P = (uint64_t)1 << g.p;
    const bool wide = P >= 64;
    const uint64_t per_wave = wide ? 1 : 64 / P;
    const uint64_t waves = (g.n_bits + per_wave - 1) / per_wave;
    const unsigned blocks = (unsigned)(((waves + 3) / 4 + 7) / 8 * 8);   // a multiple of 8 (xcd_block)
    switch (nb) {
    case 1: fp64 ? gfold_launch<double, 1>(g, blocks, wide, s) : gfold_launch<float, 1>(g, blocks, wide, s); break;
    case 2: fp64 ? gfold_launch<double, 2>(g, blocks, wide, s) : gfold_launch<float, 2>(g, blocks, wide, s); break;
    case 3: fp64 ? gfold_launch<double, 3>(g, blocks, wide, s) : gfold_launch<float, 3>(g, blocks, wide, s); break;
    default: fp64 ? gfold_launch<double, 4>(g, blocks, wide, s) : gfold_launch<float, 4>(g, blocks, wide, s); break;
    }
    return hipGetLastError();
}

// amp[j] += scale * sum_{slot < n_slots} sum_{descendants (i, j') requested}
//            V_A(i) row_A(j') V_B(j') row_B(i) i^{popcount(i ^ j')}
// with the terms of FoldIswapArgs.  Per slot, a[i] = V_A(i) row_B(i) and b[j'] = row_A(j') V_B(j')
// are formed (2^G values each, from 2 x 2^G rows); with every descendant requested the double
// sum is a^T (M x ... x M) b with M = [[1, i], [i, 1]] per gate, one butterfly stage per gate.
// Lane layout (WIDE or not) as in fold_kernel; the products and sums are in FP64.
template <typename T, int G, bool WIDE, bool MASKED>
__global__ __launch_bounds__(256) void fold_iswap_kernel(FoldIswapArgs g)
{
    using C = typename Cplx<T>::type;
    constexpr int NI = 1 << G;
    const int lane = threadIdx.x & 63;
    const uint32_t wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t P = 1u << g.p;
    const uint32_t L = WIDE ? 64u : P;
    const uint32_t GB = 64u / L;
    const uint64_t wave = (uint64_t)xcd_block(blockIdx.x, gridDim.x) * 4u + wid;
    const uint64_t jj = wave * GB + (uint32_t)lane / L;
    const uint32_t sl = (uint32_t)lane % L;
    uint64_t j = jj < g.n_bits ? (uint64_t)g.order[jj] : g.n_bits;
    if (WIDE) {
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)j);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(j >> 32));
        j = ((uint64_t)hi << 32) | lo;
    }
    double re = 0.0, im = 0.0;
    if (j < g.n_bits) {
        const C *base[2];
        C vv[2][NI];                  // V_h(t)
        uint32_t off[2][NI];          // row offsets (in rows) of pattern t
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const FoldIswapHalf &f = g.h[h];
            const uint32_t x = h ? g.xb[j] : g.xa[j];
            base[h] = (const C *)f.par + ((uint64_t)(x & ~f.qmask) << g.p);
            const double *tr = f.tab + 2 * ((uint64_t)pext32(x, f.tmask) << f.n_s);
#pragma unroll
            for (int t = 0; t < NI; ++t) {
                bool ok = true;
                uint32_t y = 0, o = 0;
#pragma unroll
                for (int gg = 0; gg < G; ++gg) {
                    const uint32_t b = (uint32_t)(t >> gg) & 1u;
                    if (f.ypos[gg] >= 0) y |= b << f.ypos[gg];
                    else ok = ok && ((x >> f.q[gg]) & 1u) == b;
                    o |= b << f.q[gg];
                }
                vv[h][t].x = ok ? (T)tr[2 * y] : T(0);
                vv[h][t].y = ok ? (T)tr[2 * y + 1] : T(0);
                off[h][t] = o;
            }
        }
        uint32_t vi[NI], vj[NI];      // descendant index bits of an i pattern / a j pattern
#pragma unroll
        for (int t = 0; t < NI; ++t) {
            vi[t] = vj[t] = 0;
#pragma unroll
            for (int gg = 0; gg < G; ++gg) {
                vi[t] |= (uint32_t)((t >> gg) & 1) << (g.u[gg] + 1);
                vj[t] |= (uint32_t)((t >> gg) & 1) << g.u[gg];
            }
        }
        for (uint32_t s = sl; s < g.n_slots; s += L) {
            double ar[NI], ai[NI], br[NI], bi[NI];
#pragma unroll
            for (int t = 0; t < NI; ++t) {
                const C rb = base[1][((uint64_t)off[1][t] << g.p) + s];    // row_B(i = t)
                const C ra = base[0][((uint64_t)off[0][t] << g.p) + s];    // row_A(j = t)
                const C va = vv[0][t], vb = vv[1][t];
                ar[t] = (double)(va.x * rb.x - va.y * rb.y);
                ai[t] = (double)(va.x * rb.y + va.y * rb.x);
                br[t] = (double)(vb.x * ra.x - vb.y * ra.y);
                bi[t] = (double)(vb.x * ra.y + vb.y * ra.x);
            }
            if (!MASKED) {
#pragma unroll
                for (int gg = 0; gg < G; ++gg)
#pragma unroll
                    for (int t = 0; t < NI; ++t)
                        if (!(t & (1 << gg))) {
                            const int t1 = t | (1 << gg);
                            const double r0 = br[t], i0 = bi[t], r1 = br[t1], i1 = bi[t1];
                            br[t] = r0 - i1;  bi[t] = i0 + r1;      // b0 + i b1
                            br[t1] = r1 - i0; bi[t1] = i1 + r0;     // i b0 + b1
                        }
#pragma unroll
                for (int t = 0; t < NI; ++t) {
                    re += ar[t] * br[t] - ai[t] * bi[t];
                    im += ar[t] * bi[t] + ai[t] * br[t];
                }
            } else {
                const uint64_t m = g.child_mask[s];
#pragma unroll
                for (int ti = 0; ti < NI; ++ti)
#pragma unroll
                    for (int tj = 0; tj < NI; ++tj) {
                        double pr = ar[ti] * br[tj] - ai[ti] * bi[tj];
                        double pi = ar[ti] * bi[tj] + ai[ti] * br[tj];
                        const int e = __popc((uint32_t)(ti ^ tj)) & 3;     // times i^e
                        if (e & 1) { const double tmp = pr; pr = -pi; pi = tmp; }
                        if (e & 2) { pr = -pr; pi = -pi; }
                        const bool use = (m >> (vi[ti] | vj[tj])) & 1u;
                        re += use ? pr : 0.0;
                        im += use ? pi : 0.0;
                    }
            }
        }
    }
    for (uint32_t mm = 1; mm < L; mm <<= 1) {
        re += __shfl_xor(re, (int)mm);
        im += __shfl_xor(im, (int)mm);
    }
    if (j < g.n_bits && sl == 0) {
        double *o = g.acc + 2 * j;
        o[0] += g.scale_re * re - g.scale_im * im;
        o[1] += g.scale_re * im + g.scale_im * re;
    }
}

template <typename T, int G>
static void fold_iswap_launch(const FoldIswapArgs &g, unsigned blocks, bool wide, hipStream_t s)
{
    if (g.all_children) {
        if (wide) fold_iswap_kernel<T, G, true, false><<<blocks, 256, 0, s>>>(g);
        else fold_iswap_kernel<T, G, false, false><<<blocks, 256, 0, s>>>(g);
    } else {
        if (wide) fold_iswap_kernel<T, G, true, true><<<blocks, 256, 0, s>>>(g);
        else fold_iswap_kernel<T, G, false, true><<<blocks, 256, 0, s>>>(g);
    }
}

hipError_t launch_fold_iswap(bool fp64, int G, const FoldIswapArgs &g, hipStream_t s)
{
    if (g.n_bits == 0) return hipSuccess;
    if (G < 1 || G > 3 || g.p < 0 || g.p > 31 || !g.order || !g.child_mask) return hipErrorInvalidValue;
    const uint64_t P = (uint64_t)1 << g.p;
    const bool wide = P >= 64;
    const uint64_t per_wave = wide ? 1 : 64 / P;
    const uint64_t waves = (g.n_bits + per_wave - 1) / per_wave;
    const unsigned blocks = (unsigned)(((waves + 3) / 4 + 7) / 8 * 8);   // a multiple of 8 (xcd_block)
    switch (G) {
    case 1: fp64 ? fold_iswap_launch<double, 1>(g, blocks, wide, s) : fold_iswap_launch<float, 1>(g, blocks, wide, s); break;
    case 2: fp64 ? fold_iswap_launch<double, 2>(g, blocks, wide, s) : fold_iswap_launch<float, 2>(g, blocks, wide, s); break;
    default: fp64 ? fold_iswap_launch<double, 3>(g, blocks, wide, s) : fold_iswap_launch<float, 3>(g, blocks, wide, s); break;
    }
    return hipGetLastError();
}

// key[i] = pext(x[i], mask): visiting key of the leaf fold (bitstrings that share their block-A
// bits outside the fold's S qubits read the same parent rows)
__global__ void key_kernel(const uint32_t *x, uint64_t n, uint32_t mask, uint32_t *key)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) key[i] = pext32(x[i], mask);
}

hipError_t launch_key(const uint32_t *x, uint64_t n, uint32_t mask, uint32_t *key, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    key_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, n, mask, key);
    return hipGetLastError();
}

// *count += number of i with i == 0 or keys[i] != keys[i - 1] (distinct values of a sorted array)
__global__ void count_runs_kernel(const uint32_t *keys, uint64_t n, int *count)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool first = i < n && (i == 0 || keys[i] != keys[i - 1]);
    const uint64_t b = __ballot(first);      // one atomic per wave
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(count, (int)__popcll(b));
}

hipError_t launch_count_runs(const uint32_t *keys, uint64_t n, int *count, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    count_runs_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(keys, n, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------- rejection sampling

// Candidate j of a batch (Algorithms 1 and 2 of the rejection-sampling section): p = re^2 + im^2,
// t = p * scale (scale = 2^n / M), u = (output j of SplitMix64(seed) >> 11) * 2^-53.  Algorithm 2
// accepts when u < t; Algorithm 1 (basic) removes t > 1 first.  excess[j] = p when t > 1.
// Every product and sum is rounded on its own (no contraction), so the decision is the same FP64
// computation on any device.
__global__ void accept_kernel(const double *amps, uint64_t n, double scale, uint64_t seed, int basic,
                              uint8_t *flag, double *excess)
{
#pragma clang fp contract(off)
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double re = amps[2 * j], im = amps[2 * j + 1];
    const double rr = re * re;
    const double ii = im * im;
    const double p = rr + ii;
    const double t = p * scale;
    uint64_t z = seed + (j + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const double u = (double)(z >> 11) * 0x1p-53;
    const bool acc = basic ? (t <= 1.0 && u < t) : (u < t);
    flag[j] = acc ? 1 : 0;
    excess[j] = t > 1.0 ? p : 0.0;
}

hipError_t reject_temp_bytes(uint64_t n, size_t *bytes)
{
    size_t a = 0, b = 0;
    hipError_t e = rocprim::select(nullptr, a, rocprim::counting_iterator<uint32_t>(0), (const uint8_t *)nullptr,
                                   (uint32_t *)nullptr, (uint64_t *)nullptr, (size_t)n);
    if (e != hipSuccess) return e;
    e = rocprim::reduce(nullptr, b, (const double *)nullptr, (double *)nullptr, (size_t)n, rocprim::plus<double>());
    *bytes = a > b ? a : b;
    return e;
}

hipError_t launch_accept(const double *amps, uint64_t n, double scale, uint64_t seed, int basic, uint8_t *flag,
                         double *excess, uint32_t *accepted, uint64_t *n_accepted, double *excess_sum,
                         void *temp, size_t temp_bytes, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    accept_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(amps, n, scale, seed, basic, flag, excess);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t tb = temp_bytes;
    e = rocprim::select(temp, tb, rocprim::counting_iterator<uint32_t>(0), (const uint8_t *)flag, accepted, n_accepted,
                        (size_t)n, s);
    if (e != hipSuccess) return e;
    tb = temp_bytes;
    return rocprim::reduce(temp, tb, (const double *)excess, excess_sum, (size_t)n, rocprim::plus<double>(), s);
}

// ---------------------------------------------------------------- validation: overlaps

// Per-block partial sums over n FP64 complex pairs: Re sum conj(a) b, Im sum conj(a) b,
// sum |a|^2, sum |b|^2 (b == NULL: only sum |a|^2 is meaningful).  Grid-stride, then a fixed
// tree over the block, so a launch's result does not depend on timing.
__global__ __launch_bounds__(256) void overlap_kernel(const double *a, const double *b, uint64_t n, double *partial)
{
    __shared__ double sh[4][256];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
        const double ar = a[2 * i], ai = a[2 * i + 1];
        s2 += ar * ar + ai * ai;
        if (b) {
            const double br = b[2 * i], bi = b[2 * i + 1];
            s0 += ar * br + ai * bi;
            s1 += ar * bi - ai * br;
            s3 += br * br + bi * bi;
        }
    }
    sh[0][threadIdx.x] = s0;
    sh[1][threadIdx.x] = s1;
    sh[2][threadIdx.x] = s2;
    sh[3][threadIdx.x] = s3;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 4; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) partial[4 * (uint64_t)blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

hipError_t launch_overlap(const double *a, const double *b, uint64_t n, double *partial, unsigned blocks,
                          hipStream_t s)
{
    if (n == 0 || blocks == 0) return hipSuccess;
    overlap_kernel<<<blocks, 256, 0, s>>>(a, b, n, partial);
    return hipGetLastError();
}

// Row masks of the passes that write the level the path sum reads (PassArgs::row_mask): bitstring
// i reads the rows (x_i & ~vary) | m of a block for every m inside the vary mask (the qubits its
// fold varies; none for a plain gather); the tile holding a row has the row's qubit bits with the
// qubits inside a tile cleared.  keep = ~(vary | inside) over the block's qubits; each thread
// marks the 2^|vary & ~inside| tiles one bitstring reads.
__global__ void mark_rows_kernel(const uint32_t *__restrict__ xh, uint64_t n, uint32_t keep, uint32_t spread,
                                 uint32_t *bitmap)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t base = xh[i] & keep;
    const int nv = __popc(spread);
    for (uint32_t s = 0; s < (1u << nv); ++s) {
        // deposit the bits of s at the positions of spread
        uint32_t m = 0, rest = spread;
        for (int b = 0; b < nv; ++b) {
            const uint32_t low = rest & (0u - rest);
            if ((s >> b) & 1u) m |= low;
            rest ^= low;
        }
        const uint32_t r = base | m;
        atomicOr(&bitmap[r >> 5], 1u << (r & 31u));
    }
}

// Number of set bits in n words (one atomic add per workgroup).
__global__ void count_bits_kernel(const uint32_t *__restrict__ words, uint64_t n, unsigned long long *count)
{
    __shared__ unsigned long long part[256];
    unsigned long long c = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        c += (unsigned long long)__popc(words[i]);
    part[threadIdx.x] = c;
    __syncthreads();
    for (unsigned w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(count, part[0]);
}

hipError_t launch_mark_rows(const uint32_t *xh, uint64_t n, uint32_t keep, uint32_t spread, uint32_t *bitmap,
                            hipStream_t s)
{
    if (!n) return hipSuccess;
    if (__builtin_popcount(spread) > 8) return hipErrorInvalidValue;
    mark_rows_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(xh, n, keep, spread, bitmap);
    return hipGetLastError();
}

hipError_t launch_count_bits(const uint32_t *words, uint64_t n, unsigned long long *count, hipStream_t s)
{
    if (!n) return hipSuccess;
    const unsigned grid = (unsigned)std::min<uint64_t>((n + 255) / 256, 4096);
    count_bits_kernel<<<grid, 256, 0, s>>>(words, n, count);
    return hipGetLastError();
}

// Streaming read of reps x n16 16-byte words of a buffer of n16 (a power of two) words: thread
// index i (grid-stride) reads word i mod n16, eight independent loads in flight per thread
// whatever the buffer size, so a buffer that fits a cache level (the XCDs' L2s, the Infinity
// Cache) is read from it at that level's rate.  The sum is stored only in an impossible case,
// which keeps the loads.
__global__ __launch_bounds__(256) void read_probe_kernel(const float4 *__restrict__ buf, uint64_t n16, uint32_t reps,
                                                         float *sink)
{
    const uint64_t stride = (uint64_t)gridDim.x * 256u;
    const uint64_t total = (uint64_t)reps * n16, mask = n16 - 1;
    float acc = 0.f;
    uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    for (; i + 7 * stride < total; i += 8 * stride) {
        float4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = buf[(i + u * stride) & mask];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u].x + v[u].y + v[u].z + v[u].w;
    }
    for (; i < total; i += stride) acc += buf[i & mask].x;
    if (acc == -1.2345e30f) sink[0] = acc;
}

hipError_t launch_read_probe(const void *buf, uint64_t bytes, uint32_t reps, unsigned grid, float *sink, hipStream_t s)
{
    if (!buf || !sink || bytes < 16 || (bytes & (bytes - 1)) || grid == 0) return hipErrorInvalidValue;
    read_probe_kernel<<<grid, 256, 0, s>>>((const float4 *)buf, bytes / 16, reps, sink);
    return hipGetLastError();
}

__global__ void fill_zero_kernel(double *p, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

__global__ void fill_zero_i32_kernel(int *p, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

hipError_t launch_fill_zero(double *p, uint64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    fill_zero_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_fill_zero_i32(int *p, uint64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    fill_zero_i32_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

}  // namespace sf
