// Device-side modular arithmetic and launch-parameter structs for gfx950.
//
// All residues are 32-bit words mod 30-bit primes q (q < 2^30, so 4q < 2^32 and
// the lazy ranges [0, 2q) / [0, 4q) of Harvey's butterflies fit a word).
// Products by a fixed operand use Shoup's precomputed quotient
// w' = floor(w 2^32 / q): a*w - umulhi(a, w')*q lies in [0, 2q) for any a < 2^32.
// Sums of products of two residues are accumulated in 64 bits
// (v_mad_u64_u32) and reduced once per <= 16 terms (16 q^2 < 2^64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define HE_MAX_LIMBS 8

struct LimbConst {
    uint32_t q;        // prime
    uint32_t q2;       // 2q
    uint32_t delta;    // Delta mod q
    uint32_t delta_sh; // Shoup companion of delta
    uint32_t r32;      // 2^32 mod q
    uint32_t r32_sh;   // Shoup companion of r32
    uint32_t bar;      // floor(2^32 / q): Shoup companion of 1
    uint32_t ninv;     // N^-1 mod q
    uint32_t ninv_sh;  // Shoup companion of ninv
    uint32_t t_mod;    // t (plaintext modulus), repeated per limb for convenience
};

struct LimbConsts {
    LimbConst l[HE_MAX_LIMBS];
};

__device__ __forceinline__ uint32_t csub(uint32_t a, uint32_t m) { return a >= m ? a - m : a; }

// a * w mod q in [0, 2q), for any a < 2^32, w < q, wsh = floor(w 2^32 / q).
__device__ __forceinline__ uint32_t shoup_lazy(uint32_t a, uint32_t w, uint32_t wsh, uint32_t q) {
    uint32_t hi = __umulhi(a, wsh);
    return a * w - hi * q;
}

// x mod q in [0, q) for any 64-bit x.
__device__ __forceinline__ uint32_t reduce64(uint64_t x, const LimbConst &c) {
    uint32_t hi = (uint32_t)(x >> 32);
    uint32_t lo = (uint32_t)x;
    uint32_t a = shoup_lazy(hi, c.r32, c.r32_sh, c.q);   // hi * 2^32 mod q, [0, 2q)
    uint32_t b = lo - __umulhi(lo, c.bar) * c.q;         // lo mod q, [0, 2q)
    uint32_t s = a + b;                                   // [0, 4q)
    s = csub(s, c.q2);
    return csub(s, c.q);
}

// Cooley-Tukey butterfly with lazy reduction: inputs and outputs in [0, 4q).
__device__ __forceinline__ void ct_bfly(uint32_t &x, uint32_t &y, uint32_t w, uint32_t wsh,
                                        uint32_t q, uint32_t q2) {
    uint32_t u = csub(x, q2);                 // [0, 2q)
    uint32_t v = shoup_lazy(y, w, wsh, q);    // [0, 2q)
    x = u + v;
    y = u - v + q2;
}

// Gentleman-Sande butterfly with lazy reduction: inputs and outputs in [0, 2q).
__device__ __forceinline__ void gs_bfly(uint32_t &x, uint32_t &y, uint32_t w, uint32_t wsh,
                                        uint32_t q, uint32_t q2) {
    uint32_t u = x + y;
    uint32_t d = x - y + q2;                  // (0, 4q)
    x = csub(u, q2);
    y = shoup_lazy(d, w, wsh, q);
}
