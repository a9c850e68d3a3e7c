// Device-side building blocks of the negacyclic NTT / INTT, shared by the kernels of
// kernels_ntt.hip and the fused layer kernel (kernels_fused.hip).
//
// One workgroup (or T threads of it) transforms one limb-polynomial of 2^LOGN words held in
// LDS (2^LOGN + 2^LOGN/32 words with one pad word per 32 to spread strided accesses over the
// banks).  Each of the T = 2^(LOGN-LOGR) threads keeps 2^LOGR words in registers and runs LOGR
// radix-2 stages on them per pass, with one LDS exchange between passes.
//
// Forward (Cooley-Tukey, natural -> bit-reversed order): stage s (0-based) pairs indices
// differing in bit LOGN-1-s and multiplies by psi^brv(2^s + i), i the block index; the output
// at position k is a(psi^(2 brv(k) + 1)).  Inverse (Gentleman-Sande, bit-reversed -> natural):
// stage k pairs indices differing in bit k with twiddle psi^-brv(N/2^(k+1) + i), unscaled.
// Lazy reduction keeps forward values in [0, 4q) and inverse values in [0, 2q).
#pragma once

#include "he_device.h"

namespace {

__device__ __forceinline__ uint32_t lpad(uint32_t i) { return i + (i >> 5); }

template <int LOGN, int LO, int RP>
__device__ __forceinline__ uint32_t gidx(uint32_t F, uint32_t vv) {
    return ((F >> LO) << (LO + RP)) | (vv << LO) | (F & ((1u << LO) - 1u));
}

// Twiddles of the leading passes, fetched into registers at kernel entry.  A
// pass of RP radix-2 stages needs 2^RP - 1 twiddle pairs per register group;
// fetching them up front overlaps their latency with the first data load
// instead of paying it after every barrier.  Passes beyond the register budget
// of the launch shape (TPB threads per workgroup) read their twiddles in place.
template <int LOGN, int LOGR, int TPB>
struct PassTw {
    static constexpr int NP = (LOGN + LOGR - 1) / LOGR;
    static constexpr int rp(int P) { return LOGN - P * LOGR < LOGR ? LOGN - P * LOGR : LOGR; }
    static constexpr int cnt(int P) { return ((1 << LOGR) >> rp(P)) * ((1 << rp(P)) - 1); }
    static constexpr int off(int P) { return P == 0 ? 0 : off(P - 1) + cnt(P - 1); }
    static constexpr int waves_per_simd = TPB >= 512 ? TPB / 256 : 1;
    static constexpr int limit = 512 / waves_per_simd < 256 ? 512 / waves_per_simd : 256;
    static constexpr int budget = limit - (1 << LOGR) - 48;
    static constexpr int pf(int P, int used) {
        return (P < NP && used + 2 * cnt(P) <= budget) ? pf(P + 1, used + 2 * cnt(P)) : P;
    }
    static constexpr int PF = pf(0, 0);
    static constexpr int TOTAL = off(PF) > 0 ? off(PF) : 1;
    uint32_t w[TOTAL], ws[TOTAL];
};

// PassTw sizes its prefetch for the workgroup size it is given.  At this size the register
// budget leaves nothing to prefetch for radix 8 and up: each pass then reads its twiddles from
// cache, which keeps registers for occupancy in launches of many rows.
constexpr int TW_IN_PASS = 2048;


// Forward pass P, stage k, group g: the pair (vv, vv + half) uses twiddle
// psi^brv(tb 2^(S0+k) + ((F >> LO) << k) + (vv >> (RP - k))), slot (2^k - 1) + (vv >> (RP - k)).
// tb = 1 for a whole transform.  Sub-block j of size 2^LOGN of a 2^(LOGN+K)-point transform,
// after its first K stages, is a 2^LOGN-point transform with tb = 2^K + j: its stage s pairs
// use psi^brv(2^(s+K) + j 2^s + local block), the whole transform's twiddles.
template <int LOGN, int LOGR, int TPB, int P>
__device__ __forceinline__ void fwd_tw_load(PassTw<LOGN, LOGR, TPB> &tw, uint32_t tid, const uint32_t *__restrict__ W,
                                            const uint32_t *__restrict__ Wsh, uint32_t tb = 1) {
    using PT = PassTw<LOGN, LOGR, TPB>;
    if constexpr (P < PT::PF) {
        constexpr int T = 1 << (LOGN - LOGR);
        constexpr int S0 = P * LOGR;
        constexpr int RP = PT::rp(P);
        constexpr int LO = LOGN - S0 - RP;
        constexpr int G = (1 << LOGR) >> RP;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint32_t hi = (tid + g * T) >> LO;
#pragma unroll
            for (int k = 0; k < RP; ++k)
#pragma unroll
                for (int top = 0; top < (1 << k); ++top) {
                    const uint32_t ti = (tb << (S0 + k)) + (hi << k) + top;
                    const int slot = PT::off(P) + g * ((1 << RP) - 1) + (1 << k) - 1 + top;
                    tw.w[slot] = W[ti];
                    tw.ws[slot] = Wsh[ti];
                }
        }
        fwd_tw_load<LOGN, LOGR, TPB, P + 1>(tw, tid, W, Wsh, tb);
    }
}

// Inverse pass P, stage kk, group g: the pair (vv, vv + 2^kk) uses twiddle
// psi^-brv(2^(LOGN-S0-kk-1) + ((F >> S0) << (RP-kk-1)) + (vv >> (kk+1))),
// slot (2^(RP-kk-1) - 1) + (vv >> (kk+1)).
template <int LOGN, int LOGR, int TPB, int P>
__device__ __forceinline__ void inv_tw_load(PassTw<LOGN, LOGR, TPB> &tw, uint32_t tid, const uint32_t *__restrict__ W,
                                            const uint32_t *__restrict__ Wsh) {
    using PT = PassTw<LOGN, LOGR, TPB>;
    if constexpr (P < PT::PF) {
        constexpr int T = 1 << (LOGN - LOGR);
        constexpr int S0 = P * LOGR;
        constexpr int RP = PT::rp(P);
        constexpr int G = (1 << LOGR) >> RP;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint32_t hi = (tid + g * T) >> S0;
#pragma unroll
            for (int kk = 0; kk < RP; ++kk)
#pragma unroll
                for (int u = 0; u < (1 << (RP - kk - 1)); ++u) {
                    const uint32_t ti = (1u << (LOGN - S0 - kk - 1)) + (hi << (RP - kk - 1)) + u;
                    const int slot = PT::off(P) + g * ((1 << RP) - 1) + (1 << (RP - kk - 1)) - 1 + u;
                    tw.w[slot] = W[ti];
                    tw.ws[slot] = Wsh[ti];
                }
        }
        inv_tw_load<LOGN, LOGR, TPB, P + 1>(tw, tid, W, Wsh);
    }
}

// ------------------------------------------------------------------ forward
template <int LOGN, int LOGR, int TPB, int P>
__device__ __forceinline__ void fwd_stages(uint32_t (&v)[1 << LOGR], const PassTw<LOGN, LOGR, TPB> &tw, uint32_t tid,
                                           const uint32_t *__restrict__ W, const uint32_t *__restrict__ Wsh,
                                           uint32_t q, uint32_t q2, uint32_t tb = 1) {
    using PT = PassTw<LOGN, LOGR, TPB>;
    constexpr int T = 1 << (LOGN - LOGR);
    constexpr int S0 = P * LOGR;
    constexpr int RP = PT::rp(P);
    constexpr int LO = LOGN - S0 - RP;
    constexpr int G = (1 << LOGR) >> RP;
#pragma unroll
    for (int k = 0; k < RP; ++k) {
        const int s = S0 + k;
        const int half = 1 << (RP - 1 - k);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint32_t F = tid + g * T;
#pragma unroll
            for (int vv = 0; vv < (1 << RP); ++vv) {
                if (vv & half) continue;
                uint32_t w, wsh;
                if constexpr (P < PT::PF) {
                    const int slot = PT::off(P) + g * ((1 << RP) - 1) + (1 << k) - 1 + (vv >> (RP - k));
                    w = tw.w[slot];
                    wsh = tw.ws[slot];
                } else {
                    const uint32_t idx = gidx<LOGN, LO, RP>(F, vv);
                    const uint32_t ti = (tb << s) + (idx >> (LOGN - s));
                    w = W[ti];
                    wsh = Wsh[ti];
                }
                ct_bfly(v[g * (1 << RP) + vv], v[g * (1 << RP) + vv + half], w, wsh, q, q2);
            }
        }
    }
}

// The value at position sub 2^LS + i after the first K stages of a 2^(LS+K)-point forward
// transform, from the 2^K inputs x[i + j 2^LS] it depends on (x: the whole row).
template <int K>
__device__ __forceinline__ uint32_t fwd_lead(const uint32_t *__restrict__ x, uint32_t i, uint32_t ns, uint32_t sub,
                                             const uint32_t *__restrict__ W, const uint32_t *__restrict__ Wsh,
                                             uint32_t q, uint32_t q2) {
    static_assert(K == 1 || K == 2, "one or two leading stages");
    if constexpr (K == 1) {
        uint32_t a = x[i], b = x[i + ns];
        ct_bfly(a, b, W[1], Wsh[1], q, q2);          // stage 0: (i, i + N/2)
        return sub ? b : a;
    } else {
        uint32_t a0 = x[i], a1 = x[i + ns], a2 = x[i + 2 * ns], a3 = x[i + 3 * ns];
        ct_bfly(a0, a2, W[1], Wsh[1], q, q2);        // stage 0: (i, i + N/2), (i + N/4, i + 3N/4)
        ct_bfly(a1, a3, W[1], Wsh[1], q, q2);
        uint32_t x0 = sub < 2 ? a0 : a2, x1 = sub < 2 ? a1 : a3;
        const uint32_t ti = 2u + (sub >> 1);         // stage 1: block sub / 2, pair (i, i + N/4)
        ct_bfly(x0, x1, W[ti], Wsh[ti], q, q2);
        return (sub & 1u) ? x1 : x0;
    }
}

// K = 0: a whole transform of the row `in`.  K > 0: sub-block `sub` of a 2^(LOGN+K)-point
// transform of the row `in` (its leading K stages formed on load), twiddle base tb = 2^K + sub.
template <int LOGN, int LOGR, int TPB, int P, int K = 0>
__device__ __forceinline__ void fwd_pass(uint32_t (&v)[1 << LOGR], const PassTw<LOGN, LOGR, TPB> &tw, uint32_t *lds,
                                         uint32_t tid, const uint32_t *__restrict__ in,
                                         const uint32_t *__restrict__ W, const uint32_t *__restrict__ Wsh, uint32_t q,
                                         uint32_t q2, uint32_t tb = 1, uint32_t sub = 0) {
    constexpr int T = 1 << (LOGN - LOGR);
    constexpr int S0 = P * LOGR;
    constexpr int RP = (LOGN - S0 < LOGR) ? (LOGN - S0) : LOGR;
    constexpr int LO = LOGN - S0 - RP;
    constexpr int G = (1 << LOGR) >> RP;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const uint32_t F = tid + g * T;
#pragma unroll
        for (int vv = 0; vv < (1 << RP); ++vv) {
            const uint32_t idx = gidx<LOGN, LO, RP>(F, vv);
            if constexpr (P > 0)
                v[g * (1 << RP) + vv] = lds[lpad(idx)];
            else if constexpr (K == 0)
                v[g * (1 << RP) + vv] = in[idx];
            else
                v[g * (1 << RP) + vv] = fwd_lead<K>(in, idx, 1u << LOGN, sub, W, Wsh, q, q2);
        }
    }
    fwd_stages<LOGN, LOGR, TPB, P>(v, tw, tid, W, Wsh, q, q2, tb);
    if (P > 0) __syncthreads();   // every read of this pass is done before any write
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const uint32_t F = tid + g * T;
#pragma unroll
        for (int vv = 0; vv < (1 << RP); ++vv) {
            const uint32_t idx = gidx<LOGN, LO, RP>(F, vv);
            lds[lpad(idx)] = v[g * (1 << RP) + vv];
        }
    }
    __syncthreads();
    if constexpr (S0 + RP < LOGN) fwd_pass<LOGN, LOGR, TPB, P + 1, K>(v, tw, lds, tid, in, W, Wsh, q, q2, tb, sub);
}

// ------------------------------------------------------------------ inverse
template <int LOGN, int LOGR, int TPB, int P>
__device__ __forceinline__ void inv_stages(uint32_t (&v)[1 << LOGR], const PassTw<LOGN, LOGR, TPB> &tw, uint32_t tid,
                                           const uint32_t *__restrict__ W, const uint32_t *__restrict__ Wsh,
                                           uint32_t q, uint32_t q2) {
    using PT = PassTw<LOGN, LOGR, TPB>;
    constexpr int T = 1 << (LOGN - LOGR);
    constexpr int S0 = P * LOGR;
    constexpr int RP = PT::rp(P);
    constexpr int LO = S0;
    constexpr int G = (1 << LOGR) >> RP;
#pragma unroll
    for (int kk = 0; kk < RP; ++kk) {
        const int k = S0 + kk;          // pairs differ in bit k
        const int half = 1 << kk;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint32_t F = tid + g * T;
#pragma unroll
            for (int vv = 0; vv < (1 << RP); ++vv) {
                if (vv & half) continue;
                uint32_t w, wsh;
                if constexpr (P < PT::PF) {
                    const int slot = PT::off(P) + g * ((1 << RP) - 1) + (1 << (RP - kk - 1)) - 1 + (vv >> (kk + 1));
                    w = tw.w[slot];
                    wsh = tw.ws[slot];
                } else {
                    const uint32_t idx = gidx<LOGN, LO, RP>(F, vv);
                    const uint32_t ti = (1u << (LOGN - k - 1)) + (idx >> (k + 1));
                    w = W[ti];
                    wsh = Wsh[ti];
                }
                gs_bfly(v[g * (1 << RP) + vv], v[g * (1 << RP) + vv + half], w, wsh, q, q2);
            }
        }
    }
}

// Threads with act == false take part in the barriers only (a workgroup wider
// than the transform's T threads).
template <int LOGN, int LOGR, int TPB, int P>
__device__ __forceinline__ void inv_pass(uint32_t (&v)[1 << LOGR], const PassTw<LOGN, LOGR, TPB> &tw, uint32_t *lds,
                                         uint32_t tid, const uint32_t *__restrict__ W,
                                         const uint32_t *__restrict__ Wsh, uint32_t q, uint32_t q2,
                                         const bool act = true) {
    constexpr int T = 1 << (LOGN - LOGR);
    constexpr int S0 = P * LOGR;
    constexpr int RP = (LOGN - S0 < LOGR) ? (LOGN - S0) : LOGR;
    constexpr int LO = S0;
    constexpr int G = (1 << LOGR) >> RP;
    constexpr bool LAST = (S0 + RP >= LOGN);
    if (act) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint32_t F = tid + g * T;
#pragma unroll
            for (int vv = 0; vv < (1 << RP); ++vv) {
                const uint32_t idx = gidx<LOGN, LO, RP>(F, vv);
                v[g * (1 << RP) + vv] = lds[lpad(idx)];
            }
        }
        inv_stages<LOGN, LOGR, TPB, P>(v, tw, tid, W, Wsh, q, q2);
    }
    if constexpr (!LAST) {
        __syncthreads();
        if (act) {
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const uint32_t F = tid + g * T;
#pragma unroll
                for (int vv = 0; vv < (1 << RP); ++vv) {
                    const uint32_t idx = gidx<LOGN, LO, RP>(F, vv);
                    lds[lpad(idx)] = v[g * (1 << RP) + vv];
                }
            }
        }
        __syncthreads();
        inv_pass<LOGN, LOGR, TPB, P + 1>(v, tw, lds, tid, W, Wsh, q, q2, act);
    }
}

// Index of register i after the last inverse pass.
template <int LOGN, int LOGR>
__device__ __forceinline__ uint32_t inv_final_idx(uint32_t tid, int i) {
    constexpr int T = 1 << (LOGN - LOGR);
    constexpr int NP = (LOGN + LOGR - 1) / LOGR;
    constexpr int S0 = (NP - 1) * LOGR;
    constexpr int RP = LOGN - S0;
    constexpr int LO = S0;
    const int g = i >> RP;
    const int vv = i & ((1 << RP) - 1);
    return gidx<LOGN, LO, RP>(tid + g * T, vv);
}

__device__ __forceinline__ uint32_t mul_delta_msg(uint32_t m, const LimbConst &c) {
    // Delta * m mod q, m < t < q
    return csub(shoup_lazy(m, c.delta, c.delta_sh, c.q), c.q);
}

}  // namespace
