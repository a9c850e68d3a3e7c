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

__device__ __forceinline__ uint32_t addmod(uint32_t a, uint32_t b, uint32_t q) { return csub(a + b, q); }

// Accumulate four slots of rows J in [0, Juse) for one image.  Rows are taken
// MAC_ROWS at a time with every load of the group issued before the products,
// so a thread keeps 2 * MAC_ROWS 16-byte loads in flight; rows past Juse
// contribute zero.  The sums are folded below q after every 3 groups
// (12 products: 12 q^2 + q < 2^64).
constexpr int MAC_ROWS = 4;

__device__ __forceinline__ void mac4(const uint32_t *__restrict__ x, size_t xstride,
                                     const uint32_t *__restrict__ op, size_t opstride, uint32_t Juse,
                                     const LimbConst &c, uint32_t (&r)[4]) {
    uint64_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    uint32_t groups = 0;
    for (uint32_t J0 = 0; J0 < Juse; J0 += MAC_ROWS) {
        uint4 xv[MAC_ROWS], ov[MAC_ROWS];
#pragma unroll
        for (int u = 0; u < MAC_ROWS; ++u) {
            const uint32_t J = J0 + u < Juse ? J0 + u : Juse - 1;
            xv[u] = *reinterpret_cast<const uint4 *>(x + (size_t)J * xstride);
            ov[u] = *reinterpret_cast<const uint4 *>(op + (size_t)J * opstride);
        }
#pragma unroll
        for (int u = 0; u < MAC_ROWS; ++u) {
            if (J0 + u < Juse) {
                a0 += (uint64_t)xv[u].x * ov[u].x;
                a1 += (uint64_t)xv[u].y * ov[u].y;
                a2 += (uint64_t)xv[u].z * ov[u].z;
                a3 += (uint64_t)xv[u].w * ov[u].w;
            }
        }
        if (++groups == 3) {
            a0 = reduce64(a0, c);
            a1 = reduce64(a1, c);
            a2 = reduce64(a2, c);
            a3 = reduce64(a3, c);
            groups = 0;
        }
    }
    r[0] = reduce64(a0, c);
    r[1] = reduce64(a1, c);
    r[2] = reduce64(a2, c);
    r[3] = reduce64(a3, c);
}

// Workgroup ids are dealt to the 8 XCDs round robin.  Remap so that XCD x runs the
// contiguous logical range [x per, (x + 1) per), per = ceil(total / 8): neighbouring logical
// workgroups, which write neighbouring words of one line, then share an L2 and their partial
// writes merge there.  Launch 8 per workgroups; false for the padding ones (the whole
// workgroup, so it may return before any barrier).
__device__ __forceinline__ bool xcd_logical(uint32_t w, uint32_t total, uint32_t &logical) {
    const uint32_t per = (total + 7u) >> 3;
    logical = (w & 7u) * per + (w >> 3);
    return logical < total;
}

inline uint32_t xcd_grid(uint32_t total) { return ((total + 7u) >> 3) << 3; }
