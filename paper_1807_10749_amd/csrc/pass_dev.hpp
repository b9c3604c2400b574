// Device code of the gate-sweep passes, shared by the library's own kernels (kernels.hip) and
// by the pass kernels compiled at run time for one pass program each (hiprtc, jit.cpp): it
// depends on sf_device.hpp and the HIP device builtins only.
#pragma once
#include "sf_device.hpp"

namespace sf {

template <bool B> struct BoolC {
    static constexpr bool value = B;
};
template <int I> struct IntC {
    static constexpr int value = I;
};
template <typename X, typename Y> struct IsSame {
    static constexpr bool value = false;
};
template <typename X> struct IsSame<X, X> {
    static constexpr bool value = true;
};

// the pass program in PassArgs, staged in LDS (see pass_body)
struct LdsProgram {};

template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };

// Workgroups are dispatched to the 8 XCDs round-robin, and each XCD has its own L2.  For a grid
// that is a multiple of 8, this maps the hardware block index to a logical one so that XCD x runs
// the contiguous logical range [x * n / 8, (x + 1) * n / 8): neighbouring bitstrings in the
// visiting order (which share rows) then meet in one L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t n)
{
    return (b & 7u) * (n >> 3) + (b >> 3);
}

template <typename T>
__device__ __forceinline__ T inv_sqrt2() { return T(0.70710678118654752440084436210485); }

// a * b + c, one rounding
__device__ __forceinline__ float fma1(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma1(double a, double b, double c) { return __builtin_fma(a, b, c); }

// x with its sign bit XORed with bit 31 of s (s is 0 or 1 << 31)
__device__ __forceinline__ float flip_sign(float x, uint32_t s) { return __uint_as_float(__float_as_uint(x) ^ s); }
__device__ __forceinline__ double flip_sign(double x, uint32_t s)
{
    return __longlong_as_double((long long)((unsigned long long)__double_as_longlong(x) ^ ((unsigned long long)s << 32)));
}

// ---------------------------------------------------------------- register tier

template <int K, int R, typename C>
__device__ __forceinline__ void reg_gate(int kind, C (&v)[1 << R])
{
    constexpr int N = 1 << R;
    constexpr int B = 1 << K;
    if (kind == GK_H) {
#pragma unroll
        for (int j = 0; j < N; ++j) {
            if (j & B) continue;
            C a = v[j], b = v[j | B];
            v[j].x = a.x + b.x; v[j].y = a.y + b.y;
            v[j | B].x = a.x - b.x; v[j | B].y = a.y - b.y;
        }
    } else if (kind == GK_X) {
        // [[1,-i],[-i,1]]: a' = a - i b, b' = b - i a
#pragma unroll
        for (int j = 0; j < N; ++j) {
            if (j & B) continue;
            C a = v[j], b = v[j | B];
            v[j].x = a.x + b.y; v[j].y = a.y - b.x;
            v[j | B].x = b.x + a.y; v[j | B].y = b.y - a.x;
        }
    } else {
        // [[1,-1],[1,1]]: a' = a - b, b' = a + b
#pragma unroll
        for (int j = 0; j < N; ++j) {
            if (j & B) continue;
            C a = v[j], b = v[j | B];
            v[j].x = a.x - b.x; v[j].y = a.y - b.y;
            v[j | B].x = a.x + b.x; v[j | B].y = a.y + b.y;
        }
    }
}

template <int R, typename C>
__device__ __forceinline__ void reg_dispatch(int k, int kind, C (&v)[1 << R])
{
    switch (k) {
    case 0: if constexpr (R > 0) reg_gate<0, R>(kind, v); break;
    case 1: if constexpr (R > 1) reg_gate<1, R>(kind, v); break;
    case 2: if constexpr (R > 2) reg_gate<2, R>(kind, v); break;
    case 3: if constexpr (R > 3) reg_gate<3, R>(kind, v); break;
    case 4: if constexpr (R > 4) reg_gate<4, R>(kind, v); break;
    default: break;
    }
}

// ---------------------------------------------------------------- lane tier

template <int R, typename C>
__device__ __forceinline__ void lane_gate(int b, int kind, int lane, C (&v)[1 << R])
{
    constexpr int N = 1 << R;
    using T = decltype(v[0].x);
    const int m = 1 << b;
    const bool hi = (lane & m) != 0;
    // H:  lo' = lo + hi, hi' = lo - hi  ->  self' = sg * self + other, sg = -1 on the hi lanes
    // Y:  lo' = lo - hi, hi' = lo + hi  ->  self' = self + sg * other, sg = -1 on the lo lanes
    // (multiplying by +-1 is exact, so each is one rounded operation as an add would be)
    const T sg = (kind == GK_H) == hi ? T(-1) : T(1);
    if (kind == GK_X) {
        // both halves: self' = self - i * other
#pragma unroll
        for (int j = 0; j < N; ++j) {
            C o = v[j];
            C t;
            t.x = __shfl_xor(o.x, m);
            t.y = __shfl_xor(o.y, m);
            v[j].x = o.x + t.y;
            v[j].y = o.y - t.x;
        }
    } else if (kind == GK_H) {
#pragma unroll
        for (int j = 0; j < N; ++j) {
            C o = v[j];
            C t;
            t.x = __shfl_xor(o.x, m);
            t.y = __shfl_xor(o.y, m);
            v[j].x = fma1(o.x, sg, t.x);
            v[j].y = fma1(o.y, sg, t.y);
        }
    } else {
#pragma unroll
        for (int j = 0; j < N; ++j) {
            C o = v[j];
            C t;
            t.x = __shfl_xor(o.x, m);
            t.y = __shfl_xor(o.y, m);
            v[j].x = fma1(t.x, sg, o.x);
            v[j].y = fma1(t.y, sg, o.y);
        }
    }
}

// ---------------------------------------------------------------- per-path flips

// Swap the pairs of register qubit K where f (this lane's slot) is set.  The empty asm statement
// with K as an operand ends every case of reg_flip_dispatch with an instruction the compiler
// cannot merge across cases; otherwise it sinks the cases' identical selects into one access of
// v with a computed index, which moves v out of registers into scratch memory.
template <int K, int R, typename C>
__device__ __forceinline__ void reg_flip(bool f, C (&v)[1 << R])
{
    constexpr int N = 1 << R;
    constexpr int B = 1 << K;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        if (j & B) continue;
        const C a = v[j], b = v[j | B];
        v[j].x = f ? b.x : a.x; v[j].y = f ? b.y : a.y;
        v[j | B].x = f ? a.x : b.x; v[j | B].y = f ? a.y : b.y;
    }
    asm volatile("; reg_flip %0" :: "n"(K));
}

template <int R, typename C>
__device__ __forceinline__ void reg_flip_dispatch(int k, bool f, C (&v)[1 << R])
{
    switch (k) {
    case 0: if constexpr (R > 0) reg_flip<0, R>(f, v); break;
    case 1: if constexpr (R > 1) reg_flip<1, R>(f, v); break;
    case 2: if constexpr (R > 2) reg_flip<2, R>(f, v); break;
    case 3: if constexpr (R > 3) reg_flip<3, R>(f, v); break;
    case 4: if constexpr (R > 4) reg_flip<4, R>(f, v); break;
    default: break;
    }
}

// Flip lane bit b where f is set.  The target is a qubit bit (above the slot bits), so the
// partner lane holds the same slot and takes the same decision.
template <int R, typename C>
__device__ __forceinline__ void lane_flip(int b, bool f, C (&v)[1 << R])
{
    constexpr int N = 1 << R;
    const int m = 1 << b;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const C o = v[j];
        C t;
        t.x = __shfl_xor(o.x, m);
        t.y = __shfl_xor(o.y, m);
        v[j].x = f ? t.x : o.x;
        v[j].y = f ? t.y : o.y;
    }
}

// ---------------------------------------------------------------- iSWAP inside a block

// iSWAP (Section 7) on two qubits of the tile: the amplitudes with the qubits' bits (0, 1) and
// (1, 0) trade places, each multiplied by i; (0, 0) and (1, 1) are kept.  Selects, shuffles and
// sign flips only.

// Both qubits in registers KA < KB.  The empty asm statement keeps the cases of the dispatch
// apart (see reg_flip).
template <int KA, int KB, int R, typename C>
__device__ __forceinline__ void reg_iswap(C (&v)[1 << R])
{
    constexpr int N = 1 << R;
    constexpr int A = 1 << KA, B = 1 << KB;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        if ((j & A) || !(j & B)) continue;          // j holds (a, b) = (0, 1)
        constexpr int X = A | B;
        const C x = v[j], y = v[j ^ X];
        v[j].x = -y.y; v[j].y = y.x;                // (0, 1) <- i (1, 0)
        v[j ^ X].x = -x.y; v[j ^ X].y = x.x;        // (1, 0) <- i (0, 1)
    }
    asm volatile("; reg_iswap %0 %1" :: "n"(KA), "n"(KB));
}

template <int R, typename C>
__device__ __forceinline__ void reg_iswap_dispatch(int ka, int kb, C (&v)[1 << R])
{
    if (ka > kb) { const int t = ka; ka = kb; kb = t; }
    switch (ka * 8 + kb) {
    case 0 * 8 + 1: if constexpr (R > 1) reg_iswap<0, 1, R>(v); break;
    case 0 * 8 + 2: if constexpr (R > 2) reg_iswap<0, 2, R>(v); break;
    case 0 * 8 + 3: if constexpr (R > 3) reg_iswap<0, 3, R>(v); break;
    case 0 * 8 + 4: if constexpr (R > 4) reg_iswap<0, 4, R>(v); break;
    case 1 * 8 + 2: if constexpr (R > 2) reg_iswap<1, 2, R>(v); break;
    case 1 * 8 + 3: if constexpr (R > 3) reg_iswap<1, 3, R>(v); break;
    case 1 * 8 + 4: if constexpr (R > 4) reg_iswap<1, 4, R>(v); break;
    case 2 * 8 + 3: if constexpr (R > 3) reg_iswap<2, 3, R>(v); break;
    case 2 * 8 + 4: if constexpr (R > 4) reg_iswap<2, 4, R>(v); break;
    case 3 * 8 + 4: if constexpr (R > 4) reg_iswap<3, 4, R>(v); break;
    default: break;
    }
}

// One qubit in register K, the other in lane bit b: each lane trades with its partner across
// lane bit b.  A lane with the lane qubit 1 takes i times its partner's register j|A into its
// register j (bits (0, 1) <- (1, 0)); a lane with it 0 takes i times the partner's register j
// into its register j|A ((1, 0) <- (0, 1)).
template <int K, int R, typename C>
__device__ __forceinline__ void reg_lane_iswap(int b, int lane, C (&v)[1 << R])
{
    constexpr int N = 1 << R;
    constexpr int A = 1 << K;
    const int m = 1 << b;
    const bool hi = (lane & m) != 0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        if (j & A) continue;
        const C x0 = v[j], x1 = v[j | A];
        C t0, t1;
        t0.x = __shfl_xor(x0.x, m);
        t0.y = __shfl_xor(x0.y, m);
        t1.x = __shfl_xor(x1.x, m);
        t1.y = __shfl_xor(x1.y, m);
        v[j].x = hi ? -t1.y : x0.x;
        v[j].y = hi ? t1.x : x0.y;
        v[j | A].x = hi ? x1.x : -t0.y;
        v[j | A].y = hi ? x1.y : t0.x;
    }
    asm volatile("; reg_lane_iswap %0" :: "n"(K));
}

template <int R, typename C>
__device__ __forceinline__ void reg_lane_iswap_dispatch(int k, int b, int lane, C (&v)[1 << R])
{
    switch (k) {
    case 0: if constexpr (R > 0) reg_lane_iswap<0, R>(b, lane, v); break;
    case 1: if constexpr (R > 1) reg_lane_iswap<1, R>(b, lane, v); break;
    case 2: if constexpr (R > 2) reg_lane_iswap<2, R>(b, lane, v); break;
    case 3: if constexpr (R > 3) reg_lane_iswap<3, R>(b, lane, v); break;
    case 4: if constexpr (R > 4) reg_lane_iswap<4, R>(b, lane, v); break;
    default: break;
    }
}

// Both qubits in lane bits ba, bb: a lane whose two bits differ takes i times the value of the
// lane with both bits flipped; the others keep theirs.
template <int R, typename C>
__device__ __forceinline__ void lane_iswap(int ba, int bb, int lane, C (&v)[1 << R])
{
    constexpr int N = 1 << R;
    const int m = (1 << ba) | (1 << bb);
    const bool sel = (((lane >> ba) ^ (lane >> bb)) & 1) != 0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const C o = v[j];
        C t;
        t.x = __shfl_xor(o.x, m);
        t.y = __shfl_xor(o.y, m);
        v[j].x = sel ? -t.y : o.x;
        v[j].y = sel ? t.x : o.y;
    }
}

// ---------------------------------------------------------------- diagonal groups

__device__ __forceinline__ int tab_entry(const uint64_t (&tab)[4], int j)
{
    return (int)((tab[j >> 4] >> ((j & 15) * 4)) & 15u);
}

struct RtGroup {
    uint32_t f, ps;
    uint64_t tab[4];
    __device__ __forceinline__ uint32_t flags() const { return f; }
    __device__ __forceinline__ uint32_t pset() const { return ps; }
    __device__ __forceinline__ int t(int j) const { return tab_entry(tab, j); }
};

template <uint32_t F, uint32_t PS, uint64_t T0, uint64_t T1, uint64_t T2, uint64_t T3>
struct CtGroup {
    __device__ static constexpr uint32_t flags() { return F; }
    __device__ static constexpr uint32_t pset() { return PS; }
    __device__ static constexpr int t(int j)
    {
        return (int)(((j < 16 ? T0 : j < 32 ? T1 : j < 48 ? T2 : T3) >> ((j & 15) * 4)) & 15u);
    }
};

// Register part of a diagonal group (the lane part gives mB, cmask, keep and the path bits pval
// of the projected register qubits).  G supplies flags(), pset() (register qubits with a
// projector) and t(j) (the weight of the register-only terms at register index j): from a
// DiagGroup read at run time (RtGroup), or compile-time constants (CtGroup, the passes compiled
// for one program), where every choice below that depends on them is made by the compiler.
template <int R, typename T, typename G, typename C>
__device__ __forceinline__ void diag_regs(const G &g, int mB, uint32_t cmask, bool keep, uint32_t pval,
                                          C (&v)[1 << R])
{
    constexpr int N = 1 << R;
    const bool has_proj = (g.flags() & 2u) != 0;
    // The phase of amplitude (lane, j) is omega^m, m = mB + t(j) + 4 parity(j & cmask) (mod 8):
    // mB and cmask depend on the lane (its lane and tile bits, its slot's path bits), t(j) (the
    // terms on register qubits only) is the same for every lane.  The parity sign is kept in the
    // sign-bit word sg, updated with one XOR per register because the registers are visited in
    // Gray-code order (consecutive j differ in one bit); the sign is applied by flipping sign bits.
    // bit k of cmask moved to the sign bit
    auto cbit = [&](int k) { return (cmask << (31 - k)) & 0x80000000u; };
    if (!(g.flags() & 1u)) {
        // every weight is a multiple of 4: the phase is a sign
        auto run = [&](auto with_proj) {
            uint32_t sg = (uint32_t)((mB >> 2) & 1) << 31;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int j = i ^ (i >> 1);
                if (i) sg ^= cbit(__builtin_ctz(i));
                const uint32_t su = sg ^ ((uint32_t)((g.t(j) >> 2) & 1) << 31);
                T x = flip_sign(v[j].x, su), y = flip_sign(v[j].y, su);
                if (decltype(with_proj)::value) {
                    const bool k = keep && (((uint32_t)j & g.pset()) == pval);
                    x = k ? x : T(0);
                    y = k ? y : T(0);
                }
                v[j].x = x;
                v[j].y = y;
            }
        };
        if (has_proj) run(BoolC<true>{});
        else run(BoolC<false>{});
    } else {
        // per lane: f0 = omega^mB and f1 = omega^(mB+1); per register the uniform t(j) picks f0
        // or f1 (bit 0), then times i (bit 1) and -1 (bit 2, joined to the sign): one complex
        // product per amplitude
        const T r = inv_sqrt2<T>();
        auto omega = [&](int m, T &c, T &sn) {
            const bool odd = (m & 1) != 0;
            T c1 = odd ? r : T(1), s1 = odd ? r : T(0);
            if (m & 2) { const T t = c1; c1 = -s1; s1 = t; }
            if (m & 4) { c1 = -c1; s1 = -s1; }
            c = c1;
            sn = s1;
        };
        T c0, s0, c1, s1;
        omega(mB & 7, c0, s0);
        omega((mB + 1) & 7, c1, s1);
        // FULL: registers pick f0 or f1 and may turn by i; otherwise every register takes f0
        auto run = [&](auto with_proj, auto full) {
            uint32_t sg = 0;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int j = i ^ (i >> 1);
                if (i) sg ^= cbit(__builtin_ctz(i));
                const int t = g.t(j);
                const T x = v[j].x, y = v[j].y;
                T nx, ny;
                if (decltype(full)::value) {
                    const T c = (t & 1) ? c1 : c0, sn = (t & 1) ? s1 : s0;
                    const T px = x * c - y * sn, py = x * sn + y * c;
                    // times i: (px, py) -> (-py, px)
                    nx = (t & 2) ? -py : px;
                    ny = (t & 2) ? px : py;
                } else {
                    nx = x * c0 - y * s0;
                    ny = x * s0 + y * c0;
                }
                const uint32_t su = sg ^ ((uint32_t)((t >> 2) & 1) << 31);
                nx = flip_sign(nx, su);
                ny = flip_sign(ny, su);
                if (decltype(with_proj)::value) {
                    const bool k = keep && (((uint32_t)j & g.pset()) == pval);
                    nx = k ? nx : T(0);
                    ny = k ? ny : T(0);
                }
                v[j].x = nx;
                v[j].y = ny;
            }
        };
        const bool full = (g.flags() & 12u) != 0;
        if (has_proj) {
            if (full) run(BoolC<true>{}, BoolC<true>{});
            else run(BoolC<true>{}, BoolC<false>{});
        } else {
            if (full) run(BoolC<false>{}, BoolC<true>{});
            else run(BoolC<false>{}, BoolC<false>{});
        }
    }
}

template <int R, typename T, typename C>
__device__ __forceinline__ void apply_diag(const DiagGroup *gp, const uint8_t *terms, uint64_t eB,
                                           uint64_t sp, C (&v)[1 << R])
{
    const DiagGroup g = *gp;
    const uint8_t *t = terms + 2 * (size_t)g.term_off;
    int mB = 0;
    uint32_t cmask = 0;
    bool keep = true;
    uint32_t pset = 0, pval = 0;
    for (int i = 0; i < g.n_lin_b; ++i, t += 2) mB += t[1] * (int)((eB >> t[0]) & 1u);
    for (int i = 0; i < g.n_quad_bb; ++i, t += 2) mB += 4 * (int)((eB >> t[0]) & (eB >> t[1]) & 1u);
    for (int i = 0; i < g.n_quad_br; ++i, t += 2) cmask ^= ((uint32_t)(eB >> t[0]) & 1u) << t[1];
    for (int i = 0; i < g.n_zs_b; ++i, t += 2) mB += 4 * (int)((eB >> t[0]) & (sp >> t[1]) & 1u);
    for (int i = 0; i < g.n_zs_r; ++i, t += 2) cmask ^= ((uint32_t)(sp >> t[1]) & 1u) << t[0];
    for (int i = 0; i < g.n_proj_b; ++i, t += 2) keep = keep && (((eB >> t[0]) & 1u) == ((sp >> t[1]) & 1u));
    for (int i = 0; i < g.n_proj_r; ++i, t += 2) {
        const uint32_t bit = 1u << t[0];
        const uint32_t s = (uint32_t)((sp >> t[1]) & 1u) << t[0];
        if ((pset & bit) && ((pval & bit) != s)) keep = false;
        pset |= bit;
        pval |= s;
    }
    diag_regs<R, T>(RtGroup{g.flags, pset, {g.tab[0], g.tab[1], g.tab[2], g.tab[3]}}, mB, cmask, keep, pval, v);
}

// ---------------------------------------------------------------- pass kernel

template <int R>
__device__ __forceinline__ uint64_t reg_offset(const int32_t (&pos)[6], int j, int shift_down, int shift_up)
{
    uint64_t o = 0;
#pragma unroll
    for (int k = 0; k < R; ++k)
        if (j & (1 << k)) o += (uint64_t)1 << (pos[k] - shift_down + shift_up);
    return o;
}

// One pass for workgroup `block` of `nblocks` (see PassArgs).  P: where the pass program comes
// from: LdsProgram = the program in PassArgs, staged in LDS and interpreted per tile; otherwise
// a type whose apply<R, T>(v, lane, eB, sp) is the program compiled for this pass alone (the
// compiled passes), with every gate's kind and position a constant.  FLIP: the program may hold
// per-path flips (crossing iSWAPs); passes without them run the variant that has no code for
// them, whose register allocation they do not affect.  ZSKIP: registers (and lanes) that the
// source's zero subspace (PassArgs::n_zero) says are zero are set to zero instead of loaded;
// where a whole cache line is zero its bytes are never fetched.
//
// A (the way the arguments arrive): PassArgs by value for a kernel's own arguments, which then
// stay in the kernel-argument segment and scalar registers; const PassArgs & for the chained
// kernel's arguments in device memory, which a local copy would put in scratch memory (the
// arrays in PassArgs are indexed with run-time indices).
template <typename T, int R, bool FLIP, bool ZSKIP = false, typename A = PassArgs, typename P = LdsProgram>
__device__ __forceinline__ void pass_body(A a, uint32_t block, uint32_t nblocks)
{
    constexpr bool kLds = IsSame<P, LdsProgram>::value;
    using C = typename Cplx<T>::type;
    constexpr int N = 1 << R;
    const unsigned lane = threadIdx.x & 63u;
    const uint64_t nwaves = (uint64_t)nblocks * 4u;
    int32_t pos[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) pos[k] = a.reg_pos[k];
    const uint64_t pmask_dst = ((uint64_t)1 << a.p_dst) - 1u;

    // stage the pass program in LDS (a compiled program has none)
    __shared__ __align__(16) uint32_t s_prog[kLds ? kMaxProgWords : 1];
    const PassOp *ops = nullptr;
    const DiagGroup *groups = nullptr;
    const uint8_t *terms = nullptr;
    if constexpr (kLds) {
        for (uint32_t i = threadIdx.x; i < a.prog_words; i += blockDim.x) s_prog[i] = a.prog[i];
        __syncthreads();
        ops = (const PassOp *)s_prog;
        groups = (const DiagGroup *)(s_prog + a.groups_word);
        terms = (const uint8_t *)(s_prog + a.terms_word);
    }

    // the wave index is uniform across a wave; say so, so tile arithmetic stays in scalar registers
    const uint32_t wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool fan = a.src_mode == SRC_FANOUT;
    const uint32_t pmax = (1u << a.p_src) - 1u;
    // this lane's part of the extended index: the lane number, or its low bits plus bit 5 at
    // lane_qpos (and bit 4 at lane_qpos4)
    const bool lq = a.lane_qpos > 0, lq4 = lq && a.lane_qpos4 > 0;
    const int lane_bits = lq4 ? 4 : lq ? 5 : 6;
    const uint64_t lx = !lq ? (uint64_t)lane
                            : ((uint64_t)(lane & ((1u << lane_bits) - 1u)) | ((uint64_t)(lane >> 5) << a.lane_qpos) |
                               (lq4 ? (uint64_t)((lane >> 4) & 1u) << a.lane_qpos4 : 0));
    auto tile_base = [&](uint64_t tile) {
        // wave-uniform part of the extended index: the low tile bits go to low_pos, the rest
        // is spread around the register and low positions
        uint64_t et = (tile >> a.n_low) << lane_bits;
        for (int k = 0; k < a.n_skip; ++k) {
            const int p = a.skip_pos[k];
            et = ((et >> p) << (p + 1)) | (et & (((uint64_t)1 << p) - 1u));
        }
        for (int k = 0; k < a.n_low; ++k) et |= ((tile >> k) & 1u) << a.low_pos[k];
        return et;
    };
    // per-lane slot tables of a tile are fetched one tile ahead, so the data loads of a
    // fan-out pass do not wait behind a dependent table load
    uint64_t tile = (uint64_t)block * 4u + wid;
    uint64_t nx_sp = 0;
    uint32_t nx_par = 0;
    if (tile < a.n_tiles) {
        const uint64_t slot = (tile_base(tile) | lx) & pmask_dst;
        nx_sp = a.slot_path[slot];
        if (fan) nx_par = a.slot_parent[slot];
    }
    for (; tile < a.n_tiles; tile += nwaves) {
        const uint64_t et = tile_base(tile);
        bool skip = a.slots_real && (et & pmask_dst) >= a.slots_real;
        if (!skip && a.row_mask) {
            const uint64_t qb = et >> a.p_dst;
            skip = ((a.row_mask[qb >> 5] >> (qb & 31u)) & 1u) == 0;
        }
        if (skip) {
            // every slot of the tile is padding (the lane bits hold the 4 to 6 lowest slot bits),
            // or no amplitude of it is read by the path sum: only fetch the next tile's tables
            const uint64_t nt = tile + nwaves;
            if (nt < a.n_tiles) {
                const uint64_t slot = (tile_base(nt) | lx) & pmask_dst;
                nx_sp = a.slot_path[slot];
                if (fan) nx_par = a.slot_parent[slot];
            }
            continue;
        }
        const uint64_t eB = et | lx;                 // this lane's amplitude with register bits 0
        const uint64_t sp = nx_sp;
        const uint32_t par = nx_par;

        // zero subspace of the source: register j of this lane can be non-zero only if
        // (j & z_m) == z_v, and none of them if a lane or tile bit disagrees with its path bit
        bool z_lane = true;
        uint32_t z_m = 0, z_v = 0;
        if (ZSKIP) {
            for (int k = 0; k < a.n_zero; ++k) {
                const uint32_t sb = (uint32_t)(sp >> a.zero_bit[k]) & 1u;
                const int r = a.zero_reg[k];
                if (r >= 0) {
                    if (((z_m >> r) & 1u) && (((z_v >> r) & 1u) != sb)) z_lane = false;
                    z_m |= 1u << r;
                    z_v |= sb << r;
                } else if (((uint32_t)(eB >> a.zero_pos[k]) & 1u) != sb) {
                    z_lane = false;
                }
            }
        }
        auto live = [&](int j) { return !ZSKIP || (z_lane && (((uint32_t)j & z_m) == z_v)); };

        C v[N];
        if (a.src_mode == SRC_INIT) {
#pragma unroll
            for (int j = 0; j < N; ++j) {
                const uint64_t ej = eB + reg_offset<R>(pos, j, 0, 0);
                v[j].x = (ej & a.init_zero_mask) ? T(0) : T(1);
                v[j].y = T(0);
            }
        } else if (fan) {
            // parent slot inside the source batch; clamped so padded slots stay in bounds
            uint32_t ps = par - a.slot_parent_base;
            ps = ps > pmax ? pmax : ps;
            // source index = ((et >> p_dst) << p_src) + ((lx >> p_dst) << p_src) + ps: the first
            // term is wave-uniform (et has zeros at the lane bits), the rest a per-lane offset
            const uint64_t su = (et >> a.p_dst) << a.p_src;
            const uint64_t sl = ((lx >> a.p_dst) << a.p_src) + ps;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                const C *row = (const C *)a.src + (su + reg_offset<R>(pos, j, a.p_dst, a.p_src));   // uniform
                if (live(j)) {
                    v[j] = row[sl];
                } else {
                    v[j].x = T(0);
                    v[j].y = T(0);
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < N; ++j) {
                const C *row = (const C *)a.src + (et + reg_offset<R>(pos, j, 0, 0));   // uniform
                if (live(j)) {
                    v[j] = row[lx];
                } else {
                    v[j].x = T(0);
                    v[j].y = T(0);
                }
            }
        }
        {
            const uint64_t nt = tile + nwaves;
            if (nt < a.n_tiles) {
                const uint64_t slot = (tile_base(nt) | lx) & pmask_dst;
                nx_sp = a.slot_path[slot];
                if (fan) nx_par = a.slot_parent[slot];
            }
        }

        if constexpr (!kLds) P::template apply<R, T>(v, (int)lane, eB, sp);
        for (uint32_t i = 0; kLds && i < a.n_ops; ++i) {
            const PassOp op = ops[i];
            if (op.type == PO_REG) {
                reg_dispatch<R>(op.target, op.kind, v);
            } else if (op.type == PO_LANE) {
                lane_gate<R>(op.target, op.kind, (int)lane, v);
            } else if (!FLIP || op.type == PO_DIAG) {
                apply_diag<R, T>(groups + op.group, terms, eB, sp, v);
            } else if (op.type == PO_ISWAP) {
                const int t0 = op.target, t1 = (int)(op.group & 0xffu);
                if (op.kind == 0) reg_iswap_dispatch<R>(t0, t1, v);
                else if (op.kind == 3) lane_iswap<R>(t0, t1, (int)lane, v);
                else if (op.kind == 1) reg_lane_iswap_dispatch<R>(t1, t0, (int)lane, v);
                else reg_lane_iswap_dispatch<R>(t0, t1, (int)lane, v);
            } else {
                const bool f = (((sp >> op.group) ^ (sp >> (op.group + 1))) & 1u) != 0;
                if (op.type == PO_PFLIP_REG) reg_flip_dispatch<R>(op.target, f, v);
                else lane_flip<R>(op.target, f, v);
                // times i where the slot flips (selects: a branch here costs registers everywhere)
                const bool fi = op.kind && f;
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    const T x = v[j].x, y = v[j].y;
                    v[j].x = fi ? -y : x;
                    v[j].y = fi ? x : y;
                }
            }
        }

        if (a.rescale != 1.0) {
            const T sc = (T)a.rescale;
#pragma unroll
            for (int j = 0; j < N; ++j) { v[j].x *= sc; v[j].y *= sc; }
        }
        // streaming stores: nothing reads the destination before the next pass or the path sum
        using V2 = T __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int j = 0; j < N; ++j) {
            C *row = (C *)a.dst + (et + reg_offset<R>(pos, j, 0, 0));   // uniform
            const V2 val = {v[j].x, v[j].y};
            __builtin_nontemporal_store(val, (V2 *)(row + lx));
        }
    }
}

// The pass kernels keep at least three waves per SIMD resident (at most 168 VGPRs): the
// sweeps alternate whole-tile loads, register work and stores, and fewer waves leave the SIMDs
// idle while a tile's loads are in flight.
#define SF_PASS_OCCUPANCY __attribute__((amdgpu_waves_per_eu(3)))

}  // namespace sf
