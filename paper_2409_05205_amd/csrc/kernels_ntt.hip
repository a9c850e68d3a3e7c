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
k_ntt_fwd(FwdJobs jobs, const uint32_t *__restrict__ tw, const uint32_t *__restrict__ twsh, LimbConsts lc) {
    constexpr int N = 1 << LOGN;
    constexpr int T = 1 << (LOGN - LOGR);
    __shared__ uint32_t lds[N + (N >> 5)];
    const uint32_t tid = threadIdx.x;
    uint32_t r = blockIdx.x;
    const int js = r < jobs.rows0 ? 0 : 1;       // rows of job 0 first, then job 1
    if (js) r -= jobs.rows0;
    const RowMap &map = jobs.map[js];
    const uint32_t l = r % map.L;
    const uint32_t jb = r / map.L;
    const uint32_t j = jb % map.J;
    const uint32_t b = jb / map.J;
    const uint32_t *in = jobs.src[js] + b * map.src_b + j * map.src_j + l * map.src_l;
    uint32_t *out = jobs.dst[js] + b * map.dst_b + j * map.dst_j + l * map.dst_l;
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

// Threads per row T = N / 2^LOGR; a variant is valid when 1 <= T <= 1024.
constexpr bool valid_variant(int logn, int logr) { return logr >= 2 && logr <= 5 && logr <= logn && logn - logr <= 10; }

// Default register radix: enough rows to fill the chip -> 2^5 words per thread
// (fewer, longer threads); a handful of rows -> more threads per row.
inline int default_logr(int logn, uint32_t rows) {
    if (rows >= 128) return logn <= 12 ? 4 : 5;
    const int lr = logn - 10 > 3 ? logn - 10 : 3;   // up to 1024 threads per row
    return lr < logn ? lr : logn;
}

template <int LOGN, int LOGR>
hipError_t fwd_launch(const FwdJobs &jobs, uint32_t rows, const uint32_t *tw, const uint32_t *twsh,
                      const LimbConsts &lc, hipStream_t st, const LaunchEv *ev) {
    if constexpr (valid_variant(LOGN, LOGR)) {
        HE_LAUNCH(ev, (k_ntt_fwd<LOGN, LOGR>), dim3(rows), dim3(1 << (LOGN - LOGR)), 0, st, jobs, tw, twsh, lc);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

template <int LOGN, int LOGR>
hipError_t inv_launch(const uint32_t *src, uint32_t *dst, const RowMap &map, uint32_t rows, const uint32_t *twi,
                      const uint32_t *twish, const LimbConsts &lc, int epi, const EpiParams &ep, hipStream_t st,
                      const LaunchEv *ev) {
    if constexpr (valid_variant(LOGN, LOGR)) {
        constexpr int T = 1 << (LOGN - LOGR);
        if (epi == EPI_STORE)
            HE_LAUNCH(ev, (k_ntt_inv<LOGN, LOGR, EPI_STORE>), dim3(rows), dim3(T), 0, st, src, dst, map, twi, twish,
                      lc, ep);
        else if (epi == EPI_CONV_CLASS)
            HE_LAUNCH(ev, (k_ntt_inv<LOGN, LOGR, EPI_CONV_CLASS>), dim3(rows), dim3(T), 0, st, src, dst, map, twi,
                      twish, lc, ep);
        else
            HE_LAUNCH(ev, (k_ntt_inv<LOGN, LOGR, EPI_FC_PREFIX>), dim3(rows), dim3(T), 0, st, src, dst, map, twi,
                      twish, lc, ep);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------ residue-class tail
// Rows are channel vectors h[b][n][l][0..M) with M = N/s.  A workgroup of TPW
// threads holds RW = TPW / T rows (T = M / R threads per row) of consecutive
// channels n' of one output group (b, g, l); it inverts each row in registers
// (unscaled Gentleman-Sande, twiddles = the first M entries of the N-point
// inverse table), then writes the span of residue classes its channels own:
// out_g[s m + c] for c in [c_lo, c_lo + RW s / g_o), every m < M.
template <int LOGM, int LOGR>
__global__ void __launch_bounds__(1024)
k_tail_rows(const uint32_t *__restrict__ h, uint32_t *__restrict__ out, const uint32_t *__restrict__ sh_next,
            uint32_t c_o, uint32_t g_o, uint32_t K_out, uint32_t L, uint32_t logN, uint32_t s_log, uint32_t RW,
            const uint32_t *__restrict__ twi, const uint32_t *__restrict__ twish, LimbConsts lc) {
    constexpr int M = 1 << LOGM;
    constexpr int T = 1 << (LOGM - LOGR);
    constexpr int MP = M + (M >> 5);
    extern __shared__ uint32_t lds[];
    const uint32_t tid = threadIdx.x;
    const uint32_t row = tid / T;               // row within the workgroup
    const uint32_t t = tid % T;
    const uint32_t chunks = g_o / RW;
    uint32_t w = blockIdx.x;
    const uint32_t chunk = w % chunks;
    w /= chunks;
    const uint32_t l = w % L;
    w /= L;
    const uint32_t g = w % K_out;
    const uint32_t b = w / K_out;
    const LimbConst c = lc.l[l];
    const uint32_t N = 1u << logN;
    const uint32_t np0 = chunk * RW;             // first channel slot of this workgroup within the group
    uint32_t *my = lds + row * MP;
    const bool active = row < RW;
    const uint32_t n = g * g_o + np0 + row;
    const bool exists = active && n < c_o;
    if (active) {
        const uint32_t *src = h + ((size_t)(b * c_o + (exists ? n : 0)) * L + l) * M;
#pragma unroll
        for (int i = 0; i < (1 << LOGR); ++i) {
            const uint32_t idx = t + i * T;
            my[lpad(idx)] = exists ? src[idx] : 0u;
        }
    }
    __syncthreads();
    uint32_t v[1 << LOGR];
    inv_pass<LOGM, LOGR, 0>(v, my, t, twi + (size_t)l * N, twish + (size_t)l * N, c.q, c.q2);
    __syncthreads();
    if (active) {
#pragma unroll
        for (int i = 0; i < (1 << LOGR); ++i) my[lpad(inv_final_idx<LOGM, LOGR>(t, i))] = csub(v[i], c.q);
    }
    __syncthreads();
    // g_o, RW and s are powers of two: class width, span and indices by shifts
    const uint32_t cw_log = s_log - (31u - __clz(g_o));
    const uint32_t span_log = (31u - __clz(RW)) + cw_log;
    const uint32_t c_lo = np0 << cw_log;
    uint32_t *o = out + ((size_t)(b * K_out + g) * L + l) * N;
    const uint32_t *sh = sh_next ? sh_next + (size_t)(b * K_out + g) * N : nullptr;
    const uint32_t total = (uint32_t)M << span_log;
    for (uint32_t e = tid; e < total; e += blockDim.x) {
        const uint32_t m = e >> span_log;
        const uint32_t off = e & ((1u << span_log) - 1u);
        const uint32_t r = off >> cw_log;
        uint32_t val = 0;
        if ((off & ((1u << cw_log) - 1u)) == 0 && g * g_o + np0 + r < c_o) val = lds[r * MP + lpad(m)];
        const uint32_t k = (m << s_log) + c_lo + off;
        if (sh) val = csub(val + mul_delta_msg(sh[k], c), c.q);
        o[k] = val;
    }
}

template <int LOGM, int LOGR>
hipError_t tail_launch(const uint32_t *h, uint32_t *out, const uint32_t *sh_next, uint32_t B, uint32_t c_o,
                       uint32_t g_o, uint32_t K_out, uint32_t L, uint32_t logN, uint32_t s_log, const uint32_t *twi,
                       const uint32_t *twish, const LimbConsts &lc, hipStream_t st, const LaunchEv *ev) {
    if constexpr (valid_variant(LOGM, LOGR)) {
        constexpr int T = 1 << (LOGM - LOGR);
        constexpr int TPW = T < 256 ? 256 : T;
        uint32_t RW = TPW / T;
        if (RW > g_o) RW = g_o;
        const uint32_t grid = B * K_out * L * (g_o / RW);
        const size_t lds = (size_t)(TPW / T) * ((1u << LOGM) + (1u << LOGM >> 5)) * sizeof(uint32_t);
        HE_LAUNCH(ev, (k_tail_rows<LOGM, LOGR>), dim3(grid), dim3(TPW), lds, st, h, out, sh_next, c_o, g_o, K_out,
                  L, logN, s_log, RW, twi, twish, lc);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

}  // namespace

#define HE_SWITCH_LOGR(LN, LR, CALL)          \
    switch (LR) {                              \
        case 2: return CALL(LN, 2);            \
        case 3: return CALL(LN, 3);            \
        case 4: return CALL(LN, 4);            \
        case 5: return CALL(LN, 5);            \
        default: return hipErrorInvalidValue;  \
    }

hipError_t launch_ntt_fwd2(int logn, int logr, const FwdJobs &jobs, uint32_t rows, const uint32_t *tw,
                           const uint32_t *twsh, const LimbConsts &lc, hipStream_t st, const LaunchEv *ev) {
    if (rows == 0) return hipSuccess;
    if (logr == 0 || !valid_variant(logn, logr)) logr = default_logr(logn, rows);
#define HE_FWD(LN, LR) fwd_launch<LN, LR>(jobs, rows, tw, twsh, lc, st, ev)
    switch (logn) {
        case 8: HE_SWITCH_LOGR(8, logr, HE_FWD)
        case 9: HE_SWITCH_LOGR(9, logr, HE_FWD)
        case 10: HE_SWITCH_LOGR(10, logr, HE_FWD)
        case 11: HE_SWITCH_LOGR(11, logr, HE_FWD)
        case 12: HE_SWITCH_LOGR(12, logr, HE_FWD)
        case 13: HE_SWITCH_LOGR(13, logr, HE_FWD)
        case 14: HE_SWITCH_LOGR(14, logr, HE_FWD)
        default: return hipErrorInvalidValue;
    }
#undef HE_FWD
}

hipError_t launch_ntt_fwd(int logn, const uint32_t *src, uint32_t *dst, const RowMap &map, uint32_t rows,
                          const uint32_t *tw, const uint32_t *twsh, const LimbConsts &lc, hipStream_t st,
                          const LaunchEv *ev, int logr) {
    FwdJobs jobs;
    jobs.src[0] = jobs.src[1] = src;
    jobs.dst[0] = jobs.dst[1] = dst;
    jobs.map[0] = jobs.map[1] = map;
    jobs.rows0 = rows;
    return launch_ntt_fwd2(logn, logr, jobs, rows, tw, twsh, lc, st, ev);
}

hipError_t launch_ntt_inv(int logn, const uint32_t *src, uint32_t *dst, const RowMap &map, uint32_t rows,
                          const uint32_t *twi, const uint32_t *twish, const LimbConsts &lc, int epi,
                          const EpiParams &ep, hipStream_t st, const LaunchEv *ev, int logr) {
    if (rows == 0) return hipSuccess;
    if (logr == 0 || !valid_variant(logn, logr)) logr = default_logr(logn, rows);
#define HE_INV(LN, LR) inv_launch<LN, LR>(src, dst, map, rows, twi, twish, lc, epi, ep, st, ev)
    switch (logn) {
        case 8: HE_SWITCH_LOGR(8, logr, HE_INV)
        case 9: HE_SWITCH_LOGR(9, logr, HE_INV)
        case 10: HE_SWITCH_LOGR(10, logr, HE_INV)
        case 11: HE_SWITCH_LOGR(11, logr, HE_INV)
        case 12: HE_SWITCH_LOGR(12, logr, HE_INV)
        case 13: HE_SWITCH_LOGR(13, logr, HE_INV)
        case 14: HE_SWITCH_LOGR(14, logr, HE_INV)
        default: return hipErrorInvalidValue;
    }
#undef HE_INV
}

hipError_t launch_tail_rows(const uint32_t *h, uint32_t *out, const uint32_t *sh_next, uint32_t B, uint32_t c_o,
                            uint32_t g_o, uint32_t K_out, uint32_t L, uint32_t N, uint32_t s, const uint32_t *twi,
                            const uint32_t *twish, const LimbConsts &lc, hipStream_t st, const LaunchEv *ev,
                            int logr) {
    if (B == 0) return hipSuccess;
    uint32_t logN = 0, s_log = 0;
    while ((1u << logN) < N) ++logN;
    while ((1u << s_log) < s) ++s_log;
    const int logm = (int)(logN - s_log);
    if (logr != 0 && !valid_variant(logm, logr)) logr = 0;
    if (logr == 0) {
        const uint32_t rows = B * K_out * g_o * L;
        logr = rows >= 1024 ? (logm <= 12 ? 4 : 5) : (logm - 8 > 2 ? logm - 8 : 2);   // few rows: 256 threads/row
        if (logr > logm) logr = logm;
    }
#define HE_TAIL(LM, LR) tail_launch<LM, LR>(h, out, sh_next, B, c_o, g_o, K_out, L, logN, s_log, twi, twish, lc, st, ev)
    switch (logm) {
        case 4: HE_SWITCH_LOGR(4, logr, HE_TAIL)
        case 5: HE_SWITCH_LOGR(5, logr, HE_TAIL)
        case 6: HE_SWITCH_LOGR(6, logr, HE_TAIL)
        case 7: HE_SWITCH_LOGR(7, logr, HE_TAIL)
        case 8: HE_SWITCH_LOGR(8, logr, HE_TAIL)
        case 9: HE_SWITCH_LOGR(9, logr, HE_TAIL)
        case 10: HE_SWITCH_LOGR(10, logr, HE_TAIL)
        case 11: HE_SWITCH_LOGR(11, logr, HE_TAIL)
        case 12: HE_SWITCH_LOGR(12, logr, HE_TAIL)
        case 13: HE_SWITCH_LOGR(13, logr, HE_TAIL)
        case 14: HE_SWITCH_LOGR(14, logr, HE_TAIL)
        default: return hipErrorInvalidValue;
    }
#undef HE_TAIL
}
