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

// (w + 1/2) 2^-32: a uniform deviate in (0, 1), exact in FP64.
__device__ __forceinline__ double unit_open(uint32_t w) {
    return ((double)w + 0.5) * 0x1p-32;
}

// ------------------------------------------------------------------ log --
// Natural logarithm from IEEE operations only.  x = 2^e m with m reduced to
// [sqrt(1/2), sqrt(2)); f = m - 1 (exact); s = f/(2+f);
// log m = 2 atanh(s) = 2s + s z Q(z), z = s^2, Q(z) = sum_{k=1..10} 2/(2k+1) z^(k-1)
// (Horner with fma); log x = e ln2_hi + fma(e, ln2_lo, log m).
__device__ __forceinline__ double det_log(double x) {
    if (!(x >= 0.0)) return __builtin_nan("");
    if (x == 0.0) return -__builtin_inf();
    if (x == __builtin_inf()) return x;
    uint64_t bits = (uint64_t)__double_as_longlong(x);
    int ex = 0;
    if ((bits >> 52) == 0) {
        x = x * 0x1p54;
        bits = (uint64_t)__double_as_longlong(x);
        ex = -54;
    }
    ex += (int)(bits >> 52) - 1023;
    double m = __longlong_as_double((long long)((bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
    if (m >= 0x1.6a09e667f3bcdp+0) {
        m = m * 0.5;
        ex += 1;
    }
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
    return de * 0x1.62e42fee00000p-1 + __builtin_fma(de, 0x1.a39ef35793c76p-33, lm);
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
    if (!(y > 0.0)) return __builtin_inf();
    return k.fene_cf * det_log(y);
}

// FP32 Lennard-Jones term from an FP64 separation, and b = s6^2 + s6 that
// bounds its error.  With u = 2^-24 and relative errors to first order: the
// conversions and the three roundings of r^2 give 5u; v_rcp_f32 (1 ulp, 2u),
// the conversion of sigma^2 and the product give s2 within 9u; s4 19u; s6 29u;
// fma(s6, s6, -s6) is within (|2 s6 - 1| 29u s6 + u |g|) <= 59u b; the final
// fma and the conversions of 4 eps and E_LJ(rc) bring the term within
// 61u (4 eps) b + 2u |E_LJ(rc)|, and the later FP32 difference of the new and
// old terms adds u (4 eps) b + u |E_LJ(rc)| per term.  For a pair inside the
// cutoff b >= b_rc = s6(rc)(1 + s6(rc)), so the |E_LJ(rc)| parts are below
// c_erc u (4 eps) b, c_erc = 3 |E_LJ(rc)| / (4 eps b_rc).  A pair whose FP32
// r^2 lands on the other side of the cutoff than the FP64 one is within 6u
// rc^2 of it, where |E_mod| <= |dE/dr^2|(rc) 6u rc^2 = c_win u (4 eps) b_rc.
// The host sets kbound = kappa u (4 eps)(1 + 2^-8), kappa >= 62 + c_erc +
// c_win with a margin (at least 128), and the kernels accumulate b over both
// evaluations of every pair, inside or outside the cutoff.
struct Lj32 {
    float e;  // term
    float b;  // s6^2 + s6
};

__device__ __forceinline__ Lj32 lj32(const Consts &k, double dx, double dy, double dz) {
    const float fx = (float)dx, fy = (float)dy, fz = (float)dz;
    const float r2 = __builtin_fmaf(fz, fz, __builtin_fmaf(fy, fy, fx * fx));
    const float q = __builtin_amdgcn_rcpf(r2);
    const float s2 = k.sig2_f * q;
    const float s6 = (s2 * s2) * s2;
    const float e = __builtin_fmaf(k.four_eps_f, __builtin_fmaf(s6, s6, -s6), -k.e_rc_f);
    Lj32 o;
    o.e = (r2 < k.rc2_f) ? e : 0.0f;
    o.b = __builtin_fmaf(s6, s6, s6);
    return o;
}

// ------------------------------------------------------ wave reductions --
// Butterfly over the 64 lanes: after level L every lane holds the sum of its
// aligned block of 2^L lanes, each node formed as (left + right) in either
// operand order (IEEE addition commutes), i.e. the pairwise tree over lanes.
__device__ __forceinline__ double wave_tree(double v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v = v + __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ float wave_tree(float v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v = v + __shfl_xor(v, m, 64);
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
