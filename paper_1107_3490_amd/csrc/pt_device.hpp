// pt_device.hpp -- device arithmetic of the replica-exchange polymer kernels
// (Gross, Janke, Bachmann, arXiv:1107.3490) for gfx950.
//
// All FP64 routines here follow the operation order fixed in include/pt.h so
// that their results are identical, bit for bit, to any other implementation
// of that order on IEEE hardware.  This file must be compiled with
// -ffp-contract=off: every fused multiply-add is written out.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pt_internal.hpp"

namespace pt {

// ---------------------------------------------------------------- Philox --
// Philox4x32-10 of Salmon, Moraes, Dror and Shaw (SC'11): ten rounds of two
// 32x32->64 multiplications with the round multipliers, the high halves
// xored with the other counter words and the round key, the key bumped by the
// Weyl constants between rounds.
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox10(U4 c, uint64_t seed) {
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t a = 0xD2511F53u, b = 0xCD9E8D57u;
        uint32_t hi0 = __umulhi(a, c.x), lo0 = a * c.x;
        uint32_t hi1 = __umulhi(b, c.z), lo1 = b * c.z;
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// SplitMix64 finaliser (Steele, Lea and Flood, OOPSLA'14): the mixing step of
// the running 64-bit digests of decisions.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// (w + 1/2) 2^-32: a uniform deviate in (0, 1), exact in FP64.
__device__ __forceinline__ double unit_open(uint32_t w) {
    return ((double)w + 0.5) * 0x1p-32;
}

// ------------------------------------------------------------------ log --
// Natural logarithm from IEEE operations only.  x = 2^e m with m reduced to
// [sqrt(1/2), sqrt(2)); f = m - 1 (exact); s = f/(2+f);
// log m = 2 atanh(s) = 2s + s z Q(z), z = s^2, Q(z) = sum_{k=1..10} 2/(2k+1) z^(k-1)
// (Horner with fma); log x = e ln2_hi + fma(e, ln2_lo, log m).  Straight-line
// code: subnormals are scaled by 2^54 first, and zero, infinity, negative and
// NaN arguments are patched at the end (-inf, +inf, NaN, NaN).
__device__ __forceinline__ double det_log(double x) {
    const uint64_t b0 = (uint64_t)__double_as_longlong(x);
    const bool sub = (b0 >> 52) == 0;
    const double xs = sub ? x * 0x1p54 : x;
    const uint64_t bits = (uint64_t)__double_as_longlong(xs);
    int ex = (int)((bits >> 52) & 0x7FF) - 1023 - (sub ? 54 : 0);
    double m = __longlong_as_double((long long)((bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
    const bool hi = m >= 0x1.6a09e667f3bcdp+0;
    m = hi ? m * 0.5 : m;
    ex += hi ? 1 : 0;
    const double f = m - 1.0;
    const double s = f / (2.0 + f);
    const double z = s * s;
    double q = 2.0 / 21.0;
    q = __builtin_fma(q, z, 2.0 / 19.0);
    q = __builtin_fma(q, z, 2.0 / 17.0);
    q = __builtin_fma(q, z, 2.0 / 15.0);
    q = __builtin_fma(q, z, 2.0 / 13.0);
    q = __builtin_fma(q, z, 2.0 / 11.0);
    q = __builtin_fma(q, z, 2.0 / 9.0);
    q = __builtin_fma(q, z, 2.0 / 7.0);
    q = __builtin_fma(q, z, 2.0 / 5.0);
    q = __builtin_fma(q, z, 2.0 / 3.0);
    const double lm = __builtin_fma(s * z, q, 2.0 * s);
    const double de = (double)ex;
    double r = de * 0x1.62e42fee00000p-1 + __builtin_fma(de, 0x1.a39ef35793c76p-33, lm);
    r = (x == 0.0) ? -__builtin_inf() : r;
    r = (x == __builtin_inf()) ? x : r;
    r = (x >= 0.0) ? r : __builtin_nan("");
    return r;
}

// ------------------------------------------------------- pair / bond terms --
__device__ __forceinline__ double sq3(double dx, double dy, double dz) {
    return __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
}

// Truncated, shifted Lennard-Jones term of Eqs. (1)-(2) from r^2, FP64 order.
__device__ __forceinline__ double lj64(const Consts &k, double r2) {
    const double s2 = k.sig2 / r2;
    const double s6 = (s2 * s2) * s2;
    const double e = __builtin_fma(k.four_eps, s6 * (s6 - 1.0), -k.e_rc);
    return (r2 < k.rc2) ? e : 0.0;
}

// FENE term of Eq. (3) from r^2; +inf at or beyond r0 +- R.
__device__ __forceinline__ double fene64(const Consts &k, double r2) {
    const double r = __builtin_sqrt(r2);
    const double x = (r - k.r0) / k.R;
    const double y = __builtin_fma(-x, x, 1.0);
    const double v = k.fene_cf * det_log(y);
    return (y > 0.0) ? v : __builtin_inf();
}

// FP32 Lennard-Jones bracket g = s6 (s6 - 1), s6 = (sigma^2/r^2)^3, from an
// r^2 formed in FP64 and rounded to FP32 once, with r^2 clamped to the cutoff:
// the term of Eqs. (1)-(2) is 4 eps g(min(r^2, rc^2)) - E_LJ(rc), so the
// difference of a pair's new and old terms is 4 eps times the difference of
// their brackets (the shift cancels exactly), a far pair gives the same
// bracket twice and an exact zero, and the kernels sum bracket differences in
// FP32 and scale the sum by 4 eps once.  Error, with u = 2^-24, relative
// errors to first order and b = s6^2 + s6 (>= |g|): r^2 is within 1.01u (FP64
// r^2 rounded to FP32); v_rcp_f32 (1 ulp, 2u), the conversion of sigma^2 and the
// product give s2 within 5u; s4 11u; s6 17u; fma(s6, s6, -s6) is within
// (|2 s6 - 1| 17u s6 + u |g|) <= 35u b; the FP32 difference of the new and old
// brackets adds u (b_new + b_old).  A pair whose FP32 r^2 lands on the other
// side of the cutoff than the exact one is within 2u rc^2 of it, where
// |E_mod| <= |dE/dr^2|(rc) 2u rc^2 <= c_win u (4 eps) b_rc (c_win is taken for
// a 6u window; b >= b_rc = s6(rc)(1 + s6(rc)) inside the cutoff).  The pairwise
// FP32 sum of a move (in-lane tree, butterfly, tree over wavefronts: depth
// <= 11) adds at most 11.01u sum |t| <= 11.01u sum (b_new + b_old), and the
// scaling by 4 eps is exact for a power of two (else one FP64 rounding, inside
// the decision's relative slack).  Per pair the kernels accumulate
// b' = S^2 + S with S = s6_new + s6_old (>= b_new + b_old), and use
// kbound sum b' with kbound = kappa u (4 eps)(1 + 2^-8), kappa >= 128 and
// >= 1.25 (62 + c_erc + c_win), plus 24 for the sum: the terms need
// 37 + c_win, so the margin is more than a factor two.
struct Lj32 {
    float g;   // bracket s6 (s6 - 1)
    float s6;  // (sigma^2 / r^2)^3 of the (clamped) FP32 r^2
};

__device__ __forceinline__ Lj32 lj32(const Consts &k, double r2d) {
    const float r2 = __builtin_fminf((float)r2d, k.rc2_f);
    const float q = __builtin_amdgcn_rcpf(r2);
    const float s2 = k.sig2_f * q;
    const float s6 = (s2 * s2) * s2;
    Lj32 o;
    o.g = __builtin_fmaf(s6, s6, -s6);
    o.s6 = s6;
    return o;
}

// ------------------------------------------------------ wave reductions --
// Pairwise tree over the 64 lanes, all in registers.  Level L adds the value
// of the partner lane block of size 2^(L-1): quad permutations for levels 1-2,
// the half-row and row mirrors for levels 3-4 (after level 2 every lane of a
// quad holds the quad's sum, so a mirror reaches the partner quad; likewise
// for 8-lane groups), and the gfx950 row-swap instructions for levels 5-6
// (v_permlane16_swap / v_permlane32_swap applied to two copies of the value
// leave the lower and the upper block's sums in the two outputs).  Every node
// is (lower block + upper block) up to operand order, and IEEE addition
// commutes: the result is the pairwise tree, the same in every lane.
__device__ __forceinline__ uint32_t dpp_qp1(uint32_t v) { return __builtin_amdgcn_update_dpp(0u, v, 0xB1, 0xF, 0xF, false); }
__device__ __forceinline__ uint32_t dpp_qp2(uint32_t v) { return __builtin_amdgcn_update_dpp(0u, v, 0x4E, 0xF, 0xF, false); }
__device__ __forceinline__ uint32_t dpp_hmir(uint32_t v) { return __builtin_amdgcn_update_dpp(0u, v, 0x141, 0xF, 0xF, false); }
__device__ __forceinline__ uint32_t dpp_mir(uint32_t v) { return __builtin_amdgcn_update_dpp(0u, v, 0x140, 0xF, 0xF, false); }

template <uint32_t (*OP)(uint32_t)>
__device__ __forceinline__ double dpp64(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = OP((uint32_t)b), hi = OP((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ double join64(uint32_t lo, uint32_t hi) {
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ double wave_tree(double v) {
    v = v + dpp64<dpp_qp1>(v);
    v = v + dpp64<dpp_qp2>(v);
    v = v + dpp64<dpp_hmir>(v);
    v = v + dpp64<dpp_mir>(v);
    {
        const uint64_t b = (uint64_t)__double_as_longlong(v);
        const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)b, (uint32_t)b, false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(b >> 32), (uint32_t)(b >> 32), false, false);
        v = join64(lo[0], hi[0]) + join64(lo[1], hi[1]);
    }
    {
        const uint64_t b = (uint64_t)__double_as_longlong(v);
        const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)b, (uint32_t)b, false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(b >> 32), (uint32_t)(b >> 32), false, false);
        v = join64(lo[0], hi[0]) + join64(lo[1], hi[1]);
    }
    return v;
}

__device__ __forceinline__ float wave_tree(float v) {
    v = v + __uint_as_float(dpp_qp1(__float_as_uint(v)));
    v = v + __uint_as_float(dpp_qp2(__float_as_uint(v)));
    v = v + __uint_as_float(dpp_hmir(__float_as_uint(v)));
    v = v + __uint_as_float(dpp_mir(__float_as_uint(v)));
    {
        const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
        v = __uint_as_float(p[0]) + __uint_as_float(p[1]);
    }
    {
        const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
        v = __uint_as_float(p[0]) + __uint_as_float(p[1]);
    }
    return v;
}

// In-lane pairwise tree over a static power-of-two range of leaves.
template <int LO, int HI, class Leaf>
__device__ __forceinline__ auto lane_tree(const Leaf &leaf) {
    if constexpr (HI - LO == 1) {
        return leaf(LO);
    } else {
        constexpr int MID = (LO + HI) / 2;
        auto a = lane_tree<LO, MID>(leaf);
        auto b = lane_tree<MID, HI>(leaf);
        return a + b;
    }
}

// Orders the LDS accesses of one wavefront around a point where lanes read
// what other lanes of the same wavefront wrote.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int read_lane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ uint32_t read_lane(uint32_t v, int l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __forceinline__ double read_lane(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

}  // namespace pt
