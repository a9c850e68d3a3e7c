// Negacyclic NTT / INTT kernels for gfx950.
//
// One workgroup transforms one limb-polynomial of N = 2^LOGN words held in LDS
// (N + N/32 words with one pad word per 32 to spread strided accesses over the
// banks).  Each of the T = N / R threads keeps R = 2^LOGR words in registers
// and runs LOGR radix-2 stages on them per pass, so a transform is
// ceil(LOGN / LOGR) passes with one LDS exchange between passes.
//
// Forward (Cooley-Tukey, natural -> bit-reversed order): stage s (0-based)
// pairs indices differing in bit LOGN-1-s and multiplies by psi^brv(2^s + i),
// i the block index; the output at position k is a(psi^(2 brv(k) + 1)).
// Inverse (Gentleman-Sande, bit-reversed -> natural): stage k pairs indices
// differing in bit k with twiddle psi^-brv(N/2^(k+1) + i).  Unscaled: N^-1 is
// folded into the resident operands, or applied by the EPI_STORE epilogue.
// Lazy reduction keeps forward values in [0, 4q) and inverse values in [0, 2q).

#include "he_kernels.h"

namespace {

__device__ __forceinline__ uint32_t lpad(uint32_t i) { return i + (i >> 5); }

template <int LOGN, int LO, int RP>
__device__ __forceinline__ uint32_t gidx(uint32_t F, uint32_t vv) {
    return ((F >> LO) << (LO + RP)) | (vv << LO) | (F & ((1u << LO) - 1u));
}

// ------------------------------------------------------------------ forward
template <int LOGN, int LOGR, int S0, int RP>
__device__ __forceinline__ void fwd_stages(uint32_t (&v)[1 << LOGR], uint32_t tid, const uint32_t *__restrict__ W,
                                           const uint32_t *__restrict__ Wsh, uint32_t q, uint32_t q2) {
    constexpr int T = 1 << (LOGN - LOGR);
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
                const uint32_t idx = gidx<LOGN, LO, RP>(F, vv);
                const uint32_t ti = (1u << s) + (idx >> (LOGN - s));
                ct_bfly(v[g * (1 << RP) + vv], v[g * (1 << RP) + vv + half], W[ti], Wsh[ti], q, q2);
            }
        }
    }
}

template <int LOGN, int LOGR, int P>
__device__ __forceinline__ void fwd_pass(uint32_t (&v)[1 << LOGR], uint32_t *lds, uint32_t tid,
                                         const uint32_t *__restrict__ in, const uint32_t *__restrict__ W,
                                         const uint32_t *__restrict__ Wsh, uint32_t q, uint32_t q2) {
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
            v[g * (1 << RP) + vv] = (P == 0) ? in[idx] : lds[lpad(idx)];
        }
    }
    fwd_stages<LOGN, LOGR, S0, RP>(v, tid, W, Wsh, q, q2);
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
    if constexpr (S0 + RP < LOGN) fwd_pass<LOGN, LOGR, P + 1>(v, lds, tid, in, W, Wsh, q, q2);
}

template <int LOGN, int LOGR>
__global__ void __launch_bounds__(1 << (LOGN - LOGR))
k_ntt_fwd(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst, RowMap map,
          const uint32_t *__restrict__ tw, const uint32_t *__restrict__ twsh, LimbConsts lc) {
    constexpr int N = 1 << LOGN;
    constexpr int T = 1 << (LOGN - LOGR);
    __shared__ uint32_t lds[N + (N >> 5)];
    const uint32_t tid = threadIdx.x;
    const uint32_t r = blockIdx.x;
    const uint32_t l = r % map.L;
    const uint32_t jb = r / map.L;
    const uint32_t j = jb % map.J;
    const uint32_t b = jb / map.J;
    const uint32_t *in = src + b * map.src_b + j * map.src_j + l * map.src_l;
    uint32_t *out = dst + b * map.dst_b + j * map.dst_j + l * map.dst_l;
    const uint32_t q = lc.l[l].q, q2 = lc.l[l].q2;
    uint32_t v[1 << LOGR];
    fwd_pass<LOGN, LOGR, 0>(v, lds, tid, in, tw + (size_t)l * N, twsh + (size_t)l * N, q, q2);
#pragma unroll
    for (int i = 0; i < (1 << LOGR); ++i) {
        const uint32_t idx = tid + i * T;
        uint32_t x = lds[lpad(idx)];
        x = csub(x, q2);
        out[idx] = csub(x, q);
    }
}

// ------------------------------------------------------------------ inverse
template <int LOGN, int LOGR, int S0, int RP>
__device__ __forceinline__ void inv_stages(uint32_t (&v)[1 << LOGR], uint32_t tid, const uint32_t *__restrict__ W,
                                           const uint32_t *__restrict__ Wsh, uint32_t q, uint32_t q2) {
    constexpr int T = 1 << (LOGN - LOGR);
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
                const uint32_t idx = gidx<LOGN, LO, RP>(F, vv);
                const uint32_t ti = (1u << (LOGN - k - 1)) + (idx >> (k + 1));
                gs_bfly(v[g * (1 << RP) + vv], v[g * (1 << RP) + vv + half], W[ti], Wsh[ti], q, q2);
            }
        }
    }
}

template <int LOGN, int LOGR, int P>
__device__ __forceinline__ void inv_pass(uint32_t (&v)[1 << LOGR], uint32_t *lds, uint32_t tid,
                                         const uint32_t *__restrict__ W, const uint32_t *__restrict__ Wsh,
                                         uint32_t q, uint32_t q2) {
    constexpr int T = 1 << (LOGN - LOGR);
    constexpr int S0 = P * LOGR;
    constexpr int RP = (LOGN - S0 < LOGR) ? (LOGN - S0) : LOGR;
    constexpr int LO = S0;
    constexpr int G = (1 << LOGR) >> RP;
    constexpr bool LAST = (S0 + RP >= LOGN);
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const uint32_t F = tid + g * T;
#pragma unroll
        for (int vv = 0; vv < (1 << RP); ++vv) {
            const uint32_t idx = gidx<LOGN, LO, RP>(F, vv);
            v[g * (1 << RP) + vv] = lds[lpad(idx)];
        }
    }
    inv_stages<LOGN, LOGR, S0, RP>(v, tid, W, Wsh, q, q2);
    if constexpr (!LAST) {
        __syncthreads();
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
        inv_pass<LOGN, LOGR, P + 1>(v, lds, tid, W, Wsh, q, q2);
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

template <int LOGN, int LOGR, int EPI>
__global__ void __launch_bounds__(1 << (LOGN - LOGR))
k_ntt_inv(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst, RowMap map,
          const uint32_t *__restrict__ twi, const uint32_t *__restrict__ twish, LimbConsts lc, EpiParams ep) {
    constexpr int N = 1 << LOGN;
    constexpr int T = 1 << (LOGN - LOGR);
    __shared__ uint32_t lds[N + (N >> 5)];
    const uint32_t tid = threadIdx.x;
    const uint32_t r = blockIdx.x;
    const uint32_t l = r % map.L;
    const LimbConst c = lc.l[l];
    const uint32_t q = c.q, q2 = c.q2;

    const uint32_t *in = nullptr;
    uint32_t *outp = nullptr;
    const uint32_t *shp = nullptr;
    uint32_t cls_lo = 0, cls_w = 0, own = 0;      // EPI_CONV_CLASS
    const int32_t *biasp = nullptr;               // EPI_FC_PREFIX
    if (EPI == EPI_STORE) {
        const uint32_t jb = r / map.L;
        const uint32_t j = jb % map.J;
        const uint32_t b = jb / map.J;
        in = src + b * map.src_b + j * map.src_j + l * map.src_l;
        outp = dst + b * map.dst_b + j * map.dst_j + l * map.dst_l;
    } else if (EPI == EPI_CONV_CLASS) {
        // rows (b, g, n', l), l fastest
        const uint32_t rr = r / map.L;
        const uint32_t np = rr % ep.g_o;
        const uint32_t g = (rr / ep.g_o) % ep.K_out;
        const uint32_t b = rr / (ep.g_o * ep.K_out);
        const uint32_t n = g * ep.g_o + np;
        const uint32_t s = 1u << ep.s_log;
        cls_w = s / ep.g_o;
        cls_lo = np * cls_w;
        own = (n < ep.c_o);
        in = own ? src + ((size_t)(b * ep.c_o + n) * map.L + l) * N : nullptr;
        outp = ep.out + ((size_t)(b * ep.K_out + g) * map.L + l) * N;
        shp = ep.sh_next ? ep.sh_next + (size_t)(b * ep.K_out + g) * N : nullptr;
        if (!own) {
            // missing channel of a ragged last group: its class range holds only Delta sh'
            for (uint32_t idx = tid; idx < (uint32_t)N; idx += T) {
                const uint32_t cc = idx & (s - 1);
                if (cc >= cls_lo && cc < cls_lo + cls_w)
                    outp[idx] = shp ? mul_delta_msg(shp[idx], c) : 0u;
            }
            return;
        }
    } else {
        // rows (b, blk, l)
        const uint32_t rr = r / map.L;
        const uint32_t blk = rr % ep.blocks;
        const uint32_t b = rr / ep.blocks;
        in = src + ((size_t)(b * ep.blocks + blk) * map.L + l) * N;
        outp = ep.out + ((size_t)(b * ep.blocks + blk) * map.L + l) * ep.n_o_p;
        shp = ep.sh_next ? ep.sh_next + (size_t)(b * ep.blocks + blk) * ep.n_o_p : nullptr;
        biasp = ep.bias + (size_t)blk * ep.n_o_p;
    }

    // coalesced load into LDS
#pragma unroll
    for (int i = 0; i < (1 << LOGR); ++i) {
        const uint32_t idx = tid + i * T;
        lds[lpad(idx)] = in[idx];
    }
    __syncthreads();
    uint32_t v[1 << LOGR];
    inv_pass<LOGN, LOGR, 0>(v, lds, tid, twi + (size_t)l * N, twish + (size_t)l * N, q, q2);

#pragma unroll
    for (int i = 0; i < (1 << LOGR); ++i) {
        const uint32_t idx = inv_final_idx<LOGN, LOGR>(tid, i);
        uint32_t x = v[i];                                        // [0, 2q)
        if (EPI == EPI_STORE) {
            x = ep.scale ? shoup_lazy(x, c.ninv, c.ninv_sh, q) : x;
            outp[idx] = csub(x, q);
        } else if (EPI == EPI_CONV_CLASS) {
            const uint32_t cc = idx & ((1u << ep.s_log) - 1u);
            if (cc >= cls_lo && cc < cls_lo + cls_w) {
                uint32_t val = (cc == cls_lo) ? csub(x, q) : 0u;
                if (shp) val = csub(val + mul_delta_msg(shp[idx], c), q);
                outp[idx] = val;
            }
        } else {
            if (idx < ep.n_o_p) {
                const int32_t d = biasp[idx];
                const int64_t t = (int64_t)c.t_mod;
                int64_t m = (int64_t)d + (shp ? (int64_t)shp[idx] : 0);
                m %= t;
                if (m < 0) m += t;
                outp[idx] = csub(csub(x, q) + mul_delta_msg((uint32_t)m, c), q);
            }
        }
    }
}

template <int LOGN>
struct NttCfg {
    static constexpr int LOGR = (LOGN <= 12) ? 4 : 5;
    static constexpr int T = 1 << (LOGN - LOGR);
};

template <int LOGN>
hipError_t fwd_dispatch(const uint32_t *src, uint32_t *dst, const RowMap &map, uint32_t rows,
                        const uint32_t *tw, const uint32_t *twsh, const LimbConsts &lc, hipStream_t st) {
    using C = NttCfg<LOGN>;
    hipLaunchKernelGGL((k_ntt_fwd<LOGN, C::LOGR>), dim3(rows), dim3(C::T), 0, st, src, dst, map, tw, twsh, lc);
    return hipGetLastError();
}

template <int LOGN>
hipError_t inv_dispatch(const uint32_t *src, uint32_t *dst, const RowMap &map, uint32_t rows,
                        const uint32_t *twi, const uint32_t *twish, const LimbConsts &lc, int epi,
                        const EpiParams &ep, hipStream_t st) {
    using C = NttCfg<LOGN>;
    if (epi == EPI_STORE)
        hipLaunchKernelGGL((k_ntt_inv<LOGN, C::LOGR, EPI_STORE>), dim3(rows), dim3(C::T), 0, st, src, dst, map, twi,
                           twish, lc, ep);
    else if (epi == EPI_CONV_CLASS)
        hipLaunchKernelGGL((k_ntt_inv<LOGN, C::LOGR, EPI_CONV_CLASS>), dim3(rows), dim3(C::T), 0, st, src, dst, map,
                           twi, twish, lc, ep);
    else
        hipLaunchKernelGGL((k_ntt_inv<LOGN, C::LOGR, EPI_FC_PREFIX>), dim3(rows), dim3(C::T), 0, st, src, dst, map,
                           twi, twish, lc, ep);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_ntt_fwd(int logn, const uint32_t *src, uint32_t *dst, const RowMap &map, uint32_t rows,
                          const uint32_t *tw, const uint32_t *twsh, const LimbConsts &lc, hipStream_t st) {
    if (rows == 0) return hipSuccess;
    switch (logn) {
        case 8: return fwd_dispatch<8>(src, dst, map, rows, tw, twsh, lc, st);
        case 9: return fwd_dispatch<9>(src, dst, map, rows, tw, twsh, lc, st);
        case 10: return fwd_dispatch<10>(src, dst, map, rows, tw, twsh, lc, st);
        case 11: return fwd_dispatch<11>(src, dst, map, rows, tw, twsh, lc, st);
        case 12: return fwd_dispatch<12>(src, dst, map, rows, tw, twsh, lc, st);
        case 13: return fwd_dispatch<13>(src, dst, map, rows, tw, twsh, lc, st);
        case 14: return fwd_dispatch<14>(src, dst, map, rows, tw, twsh, lc, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_ntt_inv(int logn, const uint32_t *src, uint32_t *dst, const RowMap &map, uint32_t rows,
                          const uint32_t *twi, const uint32_t *twish, const LimbConsts &lc, int epi,
                          const EpiParams &ep, hipStream_t st) {
    if (rows == 0) return hipSuccess;
    switch (logn) {
        case 8: return inv_dispatch<8>(src, dst, map, rows, twi, twish, lc, epi, ep, st);
        case 9: return inv_dispatch<9>(src, dst, map, rows, twi, twish, lc, epi, ep, st);
        case 10: return inv_dispatch<10>(src, dst, map, rows, twi, twish, lc, epi, ep, st);
        case 11: return inv_dispatch<11>(src, dst, map, rows, twi, twish, lc, epi, ep, st);
        case 12: return inv_dispatch<12>(src, dst, map, rows, twi, twish, lc, epi, ep, st);
        case 13: return inv_dispatch<13>(src, dst, map, rows, twi, twish, lc, epi, ep, st);
        case 14: return inv_dispatch<14>(src, dst, map, rows, twi, twish, lc, epi, ep, st);
        default: return hipErrorInvalidValue;
    }
}
