// Coefficient-wise multiply-accumulate, residue-class inverse tail, and
// pack-time operand kernels for gfx950.
//
// MAC (the c0 rho - Delta sh fhat products of Alg. 1 / Alg. 2 carried out as
// coefficient-wise products in the NTT domain, Sec. IV-A-1): each thread owns
// four consecutive NTT slots (one 16-byte load per operand row), accumulates
// 32x32->64-bit products over the input polynomials J, and folds the 64-bit
// sums back below q often enough that they never overflow.
//
// Residue-class form: the inverse transform's first log2(s) stages over each
// block of s slots are linear in the block, so the row of that block transform
// that yields residue class c_n is folded into the resident operands at pack
// time (factor N^-1 x_k^-c_n with x_k the k-th evaluation point).  The MAC then
// also sums over the s slots of a block (in-thread, then across s/4 lanes with
// wave shuffles), leaving N/s values per channel for an (N/s)-point tail.

#include "he_kernels.h"
#include "mac_device.h"

namespace {

constexpr int MAC_THREADS = 256;

__global__ void __launch_bounds__(MAC_THREADS)
k_mac_full(const uint32_t *__restrict__ X, const uint32_t *__restrict__ Op, uint32_t *__restrict__ out, uint32_t B,
           uint32_t Jtot, uint32_t Juse, uint32_t c_o, uint32_t L, uint32_t N, LimbConsts lc) {
    const uint32_t k4 = (blockIdx.x * MAC_THREADS + threadIdx.x) * 4u;
    if (k4 >= N) return;
    const uint32_t l = blockIdx.y % L;
    const uint32_t n = blockIdx.y / L;
    const LimbConst c = lc.l[l];
    const uint32_t *op = Op + (size_t)(n * L + l) * Jtot * N + k4;
    for (uint32_t b = 0; b < B; ++b) {
        const uint32_t *x = X + ((size_t)b * Jtot * L + l) * N + k4;
        uint32_t r[4];
        mac4(x, (size_t)L * N, op, N, Juse, c, r);
        *reinterpret_cast<uint4 *>(out + ((size_t)(b * c_o + n) * L + l) * N + k4) = make_uint4(r[0], r[1], r[2], r[3]);
    }
}

__global__ void __launch_bounds__(MAC_THREADS)
k_mac_class(const uint32_t *__restrict__ X, const uint32_t *__restrict__ Op, uint32_t *__restrict__ h, uint32_t B,
            uint32_t Jtot, uint32_t Juse, uint32_t c_o, uint32_t L, uint32_t N, uint32_t s_log, LimbConsts lc) {
    // every lane stays alive to the shuffles; out-of-range lanes contribute zero
    const uint32_t k4 = (blockIdx.x * MAC_THREADS + threadIdx.x) * 4u;
    const bool live = k4 < N;
    const uint32_t l = blockIdx.y % L;
    const uint32_t n = blockIdx.y / L;
    const LimbConst c = lc.l[l];
    const uint32_t s = 1u << s_log;
    const uint32_t M = N >> s_log;
    const uint32_t *op = Op + (size_t)(n * L + l) * Jtot * N + k4;
    for (uint32_t b = 0; b < B; ++b) {
        uint32_t r[4] = {0, 0, 0, 0};
        if (live) {
            const uint32_t *x = X + ((size_t)b * Jtot * L + l) * N + k4;
            mac4(x, (size_t)L * N, op, N, Juse, c, r);
        }
        uint32_t *hb = h + ((size_t)(b * c_o + n) * L + l) * M;
        if (s == 1) {
            if (live) *reinterpret_cast<uint4 *>(hb + k4) = make_uint4(r[0], r[1], r[2], r[3]);
        } else if (s == 2) {
            if (live) {
                hb[k4 >> 1] = addmod(r[0], r[1], c.q);
                hb[(k4 >> 1) + 1] = addmod(r[2], r[3], c.q);
            }
        } else {
            uint32_t v = r[0] + r[1] + r[2] + r[3];     // [0, 4q)
            v = csub(csub(v, c.q2), c.q);
            const uint32_t lanes = s >> 2;               // lanes per block, <= 64
            for (uint32_t w = 1; w < lanes; w <<= 1) v = addmod(v, (uint32_t)__shfl_xor((int)v, (int)w), c.q);
            if (live && ((threadIdx.x & (lanes - 1)) == 0)) hb[k4 >> s_log] = v;
        }
    }
}

// ------------------------------------------------------------------ batched MAC
// Register-blocked over images and channels: one thread owns two consecutive
// slots for a tile of IB images x NB channels (IB*NB*2 64-bit accumulators),
// so each loaded input word feeds NB products and each operand word IB.  A
// workgroup covers 512 slots of one limb; the IB x NB tiles of one (limb,
// 512-slot) slice all run on the same XCD (workgroup ids are dealt to the 8
// XCDs round robin), so that slice of inputs and operands is read from HBM
// about once and then served by that XCD's L2.
constexpr int TB_IB = 4, TB_NB = 4, TB_THREADS = 256, TB_SLOTS = 2 * TB_THREADS;

template <bool CLASS>
__global__ void __launch_bounds__(TB_THREADS)
k_mac_tiled(const uint32_t *__restrict__ X, const uint32_t *__restrict__ Op, uint32_t *__restrict__ out, uint32_t B,
            uint32_t Jtot, uint32_t Juse, uint32_t c_o, uint32_t L, uint32_t N, uint32_t s_log, uint32_t n_super,
            uint32_t tiles_b, uint32_t tiles_n, LimbConsts lc) {
    // In the residue-class form with s >= 2 the thread's two slots lie in one block
    // and are summed into one accumulator (two products per input row J, folded
    // every 7 rows); otherwise each slot keeps its own accumulator (folded every 15).
    constexpr int NS = CLASS ? 1 : 2;
    const uint32_t w = blockIdx.x;
    const uint32_t xcd = w & 7u;
    const uint32_t r = w >> 3;
    const uint32_t per = tiles_b * tiles_n;
    const uint32_t t = r % per;
    const uint32_t S = (r / per) * 8u + xcd;          // (limb, slot chunk) slice
    if (S >= n_super) return;                          // whole workgroup: no shuffles skipped
    const uint32_t chunks = (N + TB_SLOTS - 1) / TB_SLOTS;
    const uint32_t l = S / chunks;
    const uint32_t k2 = (S % chunks) * TB_SLOTS + threadIdx.x * 2u;
    const bool live = k2 < N;
    // image tiles fastest: the workgroups resident on an XCD at one time share a few
    // operand tiles (each read from HBM once) and the slice's inputs, which fit its L2
    const uint32_t b0 = (t % tiles_b) * TB_IB;
    const uint32_t n0 = (t / tiles_b) * TB_NB;
    const LimbConst c = lc.l[l];
    uint64_t acc[TB_IB][TB_NB][NS];
#pragma unroll
    for (int i = 0; i < TB_IB; ++i)
#pragma unroll
        for (int j = 0; j < TB_NB; ++j)
#pragma unroll
            for (int u = 0; u < NS; ++u) acc[i][j][u] = 0;
    if (live) {
        const uint32_t *xp[TB_IB];
        const uint32_t *op[TB_NB];
#pragma unroll
        for (int i = 0; i < TB_IB; ++i) {
            const uint32_t b = min(b0 + i, B - 1);
            xp[i] = X + ((size_t)b * Jtot * L + l) * N + k2;
        }
#pragma unroll
        for (int j = 0; j < TB_NB; ++j) {
            const uint32_t n = min(n0 + j, c_o - 1);
            op[j] = Op + (size_t)(n * L + l) * Jtot * N + k2;
        }
        const size_t xs = (size_t)L * N;
        const uint32_t fold = CLASS ? 7u : 15u;
        uint32_t cnt = 0;
        for (uint32_t J = 0; J < Juse; ++J) {
            uint2 xv[TB_IB], ov[TB_NB];
#pragma unroll
            for (int i = 0; i < TB_IB; ++i) xv[i] = *reinterpret_cast<const uint2 *>(xp[i] + J * xs);
#pragma unroll
            for (int j = 0; j < TB_NB; ++j) ov[j] = *reinterpret_cast<const uint2 *>(op[j] + (size_t)J * N);
#pragma unroll
            for (int i = 0; i < TB_IB; ++i)
#pragma unroll
                for (int j = 0; j < TB_NB; ++j) {
                    if (CLASS) {
                        acc[i][j][0] += (uint64_t)xv[i].x * ov[j].x;
                        acc[i][j][0] += (uint64_t)xv[i].y * ov[j].y;
                    } else {
                        acc[i][j][0] += (uint64_t)xv[i].x * ov[j].x;
                        acc[i][j][NS - 1] += (uint64_t)xv[i].y * ov[j].y;
                    }
                }
            if (++cnt == fold) {
#pragma unroll
                for (int i = 0; i < TB_IB; ++i)
#pragma unroll
                    for (int j = 0; j < TB_NB; ++j)
#pragma unroll
                        for (int u = 0; u < NS; ++u) acc[i][j][u] = reduce64(acc[i][j][u], c);
                cnt = 0;
            }
        }
    }
    const uint32_t M = CLASS ? (N >> s_log) : N;
#pragma unroll
    for (int i = 0; i < TB_IB; ++i)
#pragma unroll
        for (int j = 0; j < TB_NB; ++j) {
            const uint32_t b = b0 + i, n = n0 + j;
            const bool mine = live && b < B && n < c_o;
            uint32_t *dst = out + ((size_t)(b * c_o + n) * L + l) * M;
            if (!CLASS) {
                if (mine)
                    *reinterpret_cast<uint2 *>(dst + k2) =
                        make_uint2(reduce64(acc[i][j][0], c), reduce64(acc[i][j][NS - 1], c));
            } else {
                uint32_t v = reduce64(acc[i][j][0], c);
                const uint32_t lanes = (1u << s_log) >> 1;   // lanes per block (<= 64)
                for (uint32_t m = 1; m < lanes; m <<= 1) v = addmod(v, (uint32_t)__shfl_xor((int)v, (int)m), c.q);
                if (mine && (threadIdx.x & (lanes - 1)) == 0) dst[k2 >> s_log] = v;
            }
        }
}

// ------------------------------------------------------------------ batched MAC, LDS-staged
// (mac_device.h holds the tile body.)
template <int GS>
__global__ void __launch_bounds__(ML_THREADS)
k_mac_lds(const uint32_t *__restrict__ X, const uint32_t *__restrict__ Op, uint32_t *__restrict__ h, uint32_t B,
          uint32_t Jtot, uint32_t Juse, uint32_t c_o, uint32_t L, uint32_t N, uint32_t s_log, MacLdsGeom gm,
          uint32_t xcd_order, LimbConsts lc) {
    extern __shared__ uint32_t lds[];
    // xcd_order: consecutive tiles and slot ranges on one XCD (see xcd_logical); otherwise the
    // round-robin dealing of workgroup ids spreads them over the XCDs
    uint32_t w = blockIdx.x;
    if (xcd_order && !xcd_logical(blockIdx.x, L * gm.ranges * gm.tiles_b * gm.tiles_n, w)) return;
    mac_lds_tile<GS, false>(X, Op, h, B, Jtot, Juse, c_o, L, N, s_log, gm, w, lds, lc);
}

// (mac_device.h holds the tile body.)
template <int GS>
__global__ void __launch_bounds__(ML_THREADS)
k_mac_dma(const uint32_t *__restrict__ X, const uint32_t *__restrict__ Op, uint32_t *__restrict__ h, uint32_t B,
          uint32_t Jtot, uint32_t Juse, uint32_t c_o, uint32_t L, uint32_t N, uint32_t s_log, MacLdsGeom gm,
          uint32_t xcd_order, LimbConsts lc) {
    extern __shared__ uint32_t lds[];
    uint32_t w = blockIdx.x;
    if (xcd_order && !xcd_logical(blockIdx.x, L * gm.ranges * gm.tiles_b * gm.tiles_n, w)) return;
    mac_dma_tile<GS, false>(X, Op, h, B, Jtot, Juse, c_o, L, N, s_log, gm, w, lds, lc);
}

__device__ __forceinline__ uint32_t mul_delta(uint32_t m, const LimbConst &c) {
    return csub(shoup_lazy(m, c.delta, c.delta_sh, c.q), c.q);
}

constexpr int TAIL_THREADS = 256;

__global__ void __launch_bounds__(TAIL_THREADS)
k_tail_class(const uint32_t *__restrict__ h, uint32_t *__restrict__ out, const uint32_t *__restrict__ sh_next,
             uint32_t c_o, uint32_t g_o, uint32_t K_out, uint32_t L, uint32_t logN, uint32_t s_log,
             const uint32_t *__restrict__ twi, const uint32_t *__restrict__ twish, LimbConsts lc) {
    extern __shared__ uint32_t lds[];
    const uint32_t tid = threadIdx.x;
    const uint32_t r = blockIdx.x;
    const uint32_t l = r % L;
    const uint32_t g = (r / L) % K_out;
    const uint32_t b = r / (L * K_out);
    const LimbConst c = lc.l[l];
    const uint32_t N = 1u << logN;
    const uint32_t logM = logN - s_log;
    const uint32_t M = 1u << logM;
    const uint32_t tot = g_o * M;
    for (uint32_t i = tid; i < tot; i += TAIL_THREADS) {
        const uint32_t np = i >> logM, m = i & (M - 1);
        const uint32_t n = g * g_o + np;
        lds[i] = (n < c_o) ? h[((size_t)(b * c_o + n) * L + l) * M + m] : 0u;
    }
    __syncthreads();
    const uint32_t *W = twi + (size_t)l * N;
    const uint32_t *Wsh = twish + (size_t)l * N;
    const uint32_t nb = tot >> 1;
    for (uint32_t k = 0; k < logM; ++k) {
        const uint32_t t = 1u << k;
        for (uint32_t bi = tid; bi < nb; bi += TAIL_THREADS) {
            const uint32_t np = bi >> (logM - 1);
            const uint32_t i = bi & ((M >> 1) - 1);
            const uint32_t j = ((i >> k) << (k + 1)) | (i & (t - 1));
            const uint32_t top = np * M + j;
            const uint32_t ti = (M >> (k + 1)) + (j >> (k + 1));
            uint32_t x = lds[top], y = lds[top + t];
            gs_bfly(x, y, W[ti], Wsh[ti], c.q, c.q2);
            lds[top] = x;
            lds[top + t] = y;
        }
        __syncthreads();
    }
    const uint32_t s = 1u << s_log;
    const uint32_t cls_w = s / g_o;
    uint32_t *o = out + ((size_t)(b * K_out + g) * L + l) * N;
    const uint32_t *sh = sh_next ? sh_next + (size_t)(b * K_out + g) * N : nullptr;
    for (uint32_t idx = tid; idx < N; idx += TAIL_THREADS) {
        const uint32_t cc = idx & (s - 1);
        const uint32_t m = idx >> s_log;
        uint32_t val = 0;
        if ((cc & (cls_w - 1)) == 0) {
            const uint32_t np = cc / cls_w;
            if (g * g_o + np < c_o) val = csub(lds[np * M + m], c.q);
        }
        if (sh) val = addmod(val, mul_delta(sh[idx], c), c.q);
        o[idx] = val;
    }
}

// ------------------------------------------------------------------ pack-time kernels
__device__ __forceinline__ uint32_t mulmod_c(uint32_t a, uint32_t b, const LimbConst &c) {
    return reduce64((uint64_t)a * b, c);
}

__global__ void k_expand(const uint32_t *__restrict__ rho, const int16_t *__restrict__ fhat, uint32_t *__restrict__ Op,
                         uint32_t K_in, uint32_t c_o, uint32_t L, uint32_t N, LimbConsts lc) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const uint32_t row = blockIdx.y;          // (n, l, J)
    const uint32_t Jtot = 2 * K_in;
    const uint32_t J = row % Jtot;
    const uint32_t l = (row / Jtot) % L;
    const uint32_t n = row / (Jtot * L);
    const LimbConst c = lc.l[l];
    uint32_t v;
    if (J < K_in) {
        v = rho[((size_t)J * c_o + n) * N + k];
    } else {
        const int32_t f = fhat[((size_t)(J - K_in) * c_o + n) * N + k];
        const uint32_t a = mulmod_c((uint32_t)(f < 0 ? -f : f), c.delta, c);
        // -Delta f mod q
        v = (f > 0) ? (a == 0 ? 0u : c.q - a) : a;
    }
    Op[(size_t)row * N + k] = v;
}

__global__ void k_scale(uint32_t *__restrict__ Op, const uint32_t *__restrict__ xinv, const uint32_t *__restrict__ cls,
                        uint32_t Jtot, uint32_t L, uint32_t N, LimbConsts lc) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const uint32_t row = blockIdx.y;          // (n, l, J)
    const uint32_t l = (row / Jtot) % L;
    const uint32_t n = row / (Jtot * L);
    const LimbConst c = lc.l[l];
    uint32_t fac = c.ninv;
    if (cls) {
        uint32_t e = cls[n];
        uint32_t base = xinv[(size_t)l * N + k];
        uint32_t p = 1;
        while (e) {
            if (e & 1) p = mulmod_c(p, base, c);
            base = mulmod_c(base, base, c);
            e >>= 1;
        }
        fac = mulmod_c(fac, p, c);
    }
    Op[(size_t)row * N + k] = mulmod_c(Op[(size_t)row * N + k], fac, c);
}

__global__ void k_pointwise(const uint32_t *__restrict__ a, const uint32_t *__restrict__ b, uint32_t *__restrict__ cc,
                            uint32_t L, uint32_t N, LimbConsts lc) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const uint32_t row = blockIdx.y;          // (r, l)
    const uint32_t l = row % L;
    const size_t i = (size_t)row * N + k;
    cc[i] = reduce64((uint64_t)a[i] * b[i], lc.l[l]);
}

}  // namespace

hipError_t launch_mac_full(const uint32_t *X, const uint32_t *Op, uint32_t *out, uint32_t B, uint32_t Jtot,
                           uint32_t Juse, uint32_t c_o, uint32_t L, uint32_t N, const LimbConsts &lc,
                           hipStream_t st, const LaunchEv *ev) {
    if (B == 0) return hipSuccess;
    dim3 grid((N / 4 + MAC_THREADS - 1) / MAC_THREADS, c_o * L);
    HE_LAUNCH(ev, k_mac_full, grid, dim3(MAC_THREADS), 0, st, X, Op, out, B, Jtot, Juse, c_o, L, N, lc);
    return hipGetLastError();
}

hipError_t launch_mac_class(const uint32_t *X, const uint32_t *Op, uint32_t *h, uint32_t B, uint32_t Jtot,
                            uint32_t Juse, uint32_t c_o, uint32_t L, uint32_t N, uint32_t s, const LimbConsts &lc,
                            hipStream_t st, const LaunchEv *ev) {
    if (B == 0) return hipSuccess;
    uint32_t s_log = 0;
    while ((1u << s_log) < s) ++s_log;
    if (s > 256) return hipErrorInvalidValue;   // s/4 lanes must fit one wave
    dim3 grid((N / 4 + MAC_THREADS - 1) / MAC_THREADS, c_o * L);
    HE_LAUNCH(ev, k_mac_class, grid, dim3(MAC_THREADS), 0, st, X, Op, h, B, Jtot, Juse, c_o, L, N, s_log, lc);
    return hipGetLastError();
}

hipError_t launch_tail_class(const uint32_t *h, uint32_t *out, const uint32_t *sh_next, uint32_t B, uint32_t c_o,
                             uint32_t g_o, uint32_t K_out, uint32_t L, uint32_t N, uint32_t s, const uint32_t *twi,
                             const uint32_t *twish, const LimbConsts &lc, hipStream_t st, const LaunchEv *ev) {
    if (B == 0) return hipSuccess;
    uint32_t logN = 0, s_log = 0;
    while ((1u << logN) < N) ++logN;
    while ((1u << s_log) < s) ++s_log;
    const size_t lds = (size_t)g_o * (N >> s_log) * sizeof(uint32_t);
    HE_LAUNCH(ev, k_tail_class, dim3(B * K_out * L), dim3(TAIL_THREADS), lds, st, h, out, sh_next, c_o, g_o,
              K_out, L, logN, s_log, twi, twish, lc);
    return hipGetLastError();
}

hipError_t launch_expand_operands(const uint32_t *rho, const int16_t *fhat, uint32_t *Op, uint32_t K_in, uint32_t c_o,
                                  uint32_t L, uint32_t N, const LimbConsts &lc, hipStream_t st) {
    dim3 grid((N + 255) / 256, c_o * L * 2 * K_in);
    hipLaunchKernelGGL(k_expand, grid, dim3(256), 0, st, rho, fhat, Op, K_in, c_o, L, N, lc);
    return hipGetLastError();
}

hipError_t launch_scale_operands(uint32_t *Op, const uint32_t *xinv, const uint32_t *cls, uint32_t Jtot, uint32_t c_o,
                                 uint32_t L, uint32_t N, const LimbConsts &lc, hipStream_t st) {
    dim3 grid((N + 255) / 256, c_o * L * Jtot);
    hipLaunchKernelGGL(k_scale, grid, dim3(256), 0, st, Op, xinv, cls, Jtot, L, N, lc);
    return hipGetLastError();
}

hipError_t launch_pointwise_mul(const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t rows, uint32_t L,
                                uint32_t N, const LimbConsts &lc, hipStream_t st) {
    dim3 grid((N + 255) / 256, rows * L);
    hipLaunchKernelGGL(k_pointwise, grid, dim3(256), 0, st, a, b, c, L, N, lc);
    return hipGetLastError();
}

hipError_t launch_mac_tiled(const uint32_t *X, const uint32_t *Op, uint32_t *out, uint32_t B, uint32_t Jtot,
                            uint32_t Juse, uint32_t c_o, uint32_t L, uint32_t N, uint32_t s, bool class_form,
                            const LimbConsts &lc, hipStream_t st, const LaunchEv *ev) {
    if (B == 0) return hipSuccess;
    uint32_t s_log = 0;
    while ((1u << s_log) < s) ++s_log;
    if (class_form && (s < 2 || s > 2 * 64)) return hipErrorInvalidValue;   // one block spans 1..64 lanes
    const uint32_t chunks = (N + TB_SLOTS - 1) / TB_SLOTS;
    const uint32_t n_super = chunks * L;
    const uint32_t tiles_b = (B + TB_IB - 1) / TB_IB;
    const uint32_t tiles_n = (c_o + TB_NB - 1) / TB_NB;
    const uint32_t grid = ((n_super + 7) / 8) * 8 * tiles_b * tiles_n;
    if (class_form)
        HE_LAUNCH(ev, k_mac_tiled<true>, dim3(grid), dim3(TB_THREADS), 0, st, X, Op, out, B, Jtot, Juse, c_o, L, N,
                  s_log, n_super, tiles_b, tiles_n, lc);
    else
        HE_LAUNCH(ev, k_mac_tiled<false>, dim3(grid), dim3(TB_THREADS), 0, st, X, Op, out, B, Jtot, Juse, c_o, L, N,
                  s_log, n_super, tiles_b, tiles_n, lc);
    return hipGetLastError();
}

bool mac_lds_geometry(uint32_t B, uint32_t c_o, uint32_t N, uint32_t s, MacLdsGeom *gm, size_t *lds_bytes,
                      uint32_t short_stage) {
    if (B == 0 || c_o == 0 || s < 2 || s > N || N < 256) return false;
    auto pow2_at_least = [](uint32_t x) {
        uint32_t p = 1;
        while (p < x) p <<= 1;
        return p;
    };
    uint32_t TBq = pow2_at_least((B + 3) / 4), TNq = pow2_at_least((c_o + 3) / 4);
    if (TBq > 16) TBq = 16;
    if (TNq > 16) TNq = 16;
    const uint32_t GS = s < 16 ? s : 16;
    // R staged slots per stage, at most 32 (ML_UNITS loads per thread), at least 4 (16-byte loads)
    while ((ML_THREADS / (TBq * TNq)) * GS > 32) {
        if (TBq <= TNq && TBq < 16) TBq <<= 1;
        else if (TNq < 16) TNq <<= 1;
        else break;   // 16 x 16: one group, R = GS <= 16
    }
    while ((ML_THREADS / (TBq * TNq)) * GS < 4) {
        if (TNq >= TBq && TNq > 1) TNq >>= 1;
        else TBq >>= 1;
    }
    // blocks shorter than 16 slots: stage short_stage slots (rows of 128 or 256 contiguous
    // bytes), trading image x channel reuse for full-line loads and more products per stage
    while (GS < 16 && (ML_THREADS / (TBq * TNq)) * GS < short_stage && TBq * TNq > 1) {
        if (TBq >= TNq) TBq >>= 1;
        else TNq >>= 1;
    }
    const uint32_t G = ML_THREADS / (TBq * TNq);
    const uint32_t R = G * GS;
    const uint32_t spans = s / GS;            // thread spans per block
    gm->TBq = TBq;
    gm->TNq = TNq;
    gm->GS = GS;
    gm->R = R;
    if (spans <= G) {
        gm->cpb = 1;
        gm->gpb = spans;
    } else {
        gm->cpb = spans / G;
        gm->gpb = G;
    }
    gm->ranges = N / (R * gm->cpb);
    gm->tiles_b = (B + 4 * TBq - 1) / (4 * TBq);
    gm->tiles_n = (c_o + 4 * TNq - 1) / (4 * TNq);
    const size_t stage = (size_t)2 * 4 * (TBq + TNq) * (R + 2);
    const size_t red = (size_t)ML_THREADS * ML_RED_STRIDE;
    *lds_bytes = (stage > red ? stage : red) * sizeof(uint32_t);
    return true;
}

hipError_t launch_mac_lds(const uint32_t *X, const uint32_t *Op, uint32_t *h, uint32_t B, uint32_t Jtot,
                          uint32_t Juse, uint32_t c_o, uint32_t L, uint32_t N, uint32_t s, bool xcd_order,
                          const LimbConsts &lc, hipStream_t st, const LaunchEv *ev) {
    if (B == 0) return hipSuccess;
    MacLdsGeom gm;
    size_t lds = 0;
    if (Juse == 0 || !mac_lds_geometry(B, c_o, N, s, &gm, &lds, 32)) return hipErrorInvalidValue;
    uint32_t s_log = 0;
    while ((1u << s_log) < s) ++s_log;
    const uint32_t tiles = L * gm.ranges * gm.tiles_b * gm.tiles_n;
    const uint32_t grid = xcd_order ? xcd_grid(tiles) : tiles;
    const uint32_t xo = xcd_order ? 1u : 0u;
    switch (gm.GS) {
        case 2: HE_LAUNCH(ev, k_mac_lds<2>, dim3(grid), dim3(ML_THREADS), lds, st, X, Op, h, B, Jtot, Juse, c_o, L, N, s_log, gm, xo, lc); break;
        case 4: HE_LAUNCH(ev, k_mac_lds<4>, dim3(grid), dim3(ML_THREADS), lds, st, X, Op, h, B, Jtot, Juse, c_o, L, N, s_log, gm, xo, lc); break;
        case 8: HE_LAUNCH(ev, k_mac_lds<8>, dim3(grid), dim3(ML_THREADS), lds, st, X, Op, h, B, Jtot, Juse, c_o, L, N, s_log, gm, xo, lc); break;
        case 16: HE_LAUNCH(ev, k_mac_lds<16>, dim3(grid), dim3(ML_THREADS), lds, st, X, Op, h, B, Jtot, Juse, c_o, L, N, s_log, gm, xo, lc); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

size_t mac_dma_lds_bytes(const MacLdsGeom &gm) {
    // 16-byte chunks: R a power of two in [4, 64]; every slot of a stage within ML_UNITS loads per thread
    if (gm.R < 4 || gm.R > 64 || (gm.R & (gm.R - 1)) || (4 * (gm.TBq + gm.TNq)) * (gm.R / 4) > ML_UNITS * ML_THREADS)
        return SIZE_MAX;
    const size_t stage = (size_t)MD_BUFS * 4 * (gm.TBq + gm.TNq) * gm.R;
    const size_t red = (size_t)ML_THREADS * ML_RED_STRIDE;
    return (stage > red ? stage : red) * sizeof(uint32_t);
}

hipError_t launch_mac_dma(const uint32_t *X, const uint32_t *Op, uint32_t *h, uint32_t B, uint32_t Jtot,
                          uint32_t Juse, uint32_t c_o, uint32_t L, uint32_t N, uint32_t s, bool xcd_order,
                          const LimbConsts &lc, hipStream_t st, const LaunchEv *ev) {
    if (B == 0) return hipSuccess;
    MacLdsGeom gm;
    size_t lds_pad = 0;
    // without register staging, blocks shorter than 16 slots take 64-slot stages (x4 MAC 10.3 -> 9.4 ms)
    if (Juse == 0 || !mac_lds_geometry(B, c_o, N, s, &gm, &lds_pad, 64)) return hipErrorInvalidValue;
    const size_t lds = mac_dma_lds_bytes(gm);
    if (lds == SIZE_MAX) return hipErrorInvalidValue;
    uint32_t s_log = 0;
    while ((1u << s_log) < s) ++s_log;
    const uint32_t tiles = L * gm.ranges * gm.tiles_b * gm.tiles_n;
    const uint32_t grid = xcd_order ? xcd_grid(tiles) : tiles;
    const uint32_t xo = xcd_order ? 1u : 0u;
    switch (gm.GS) {
        case 2: HE_LAUNCH(ev, k_mac_dma<2>, dim3(grid), dim3(ML_THREADS), lds, st, X, Op, h, B, Jtot, Juse, c_o, L, N, s_log, gm, xo, lc); break;
        case 4: HE_LAUNCH(ev, k_mac_dma<4>, dim3(grid), dim3(ML_THREADS), lds, st, X, Op, h, B, Jtot, Juse, c_o, L, N, s_log, gm, xo, lc); break;
        case 8: HE_LAUNCH(ev, k_mac_dma<8>, dim3(grid), dim3(ML_THREADS), lds, st, X, Op, h, B, Jtot, Juse, c_o, L, N, s_log, gm, xo, lc); break;
        case 16: HE_LAUNCH(ev, k_mac_dma<16>, dim3(grid), dim3(ML_THREADS), lds, st, X, Op, h, B, Jtot, Juse, c_o, L, N, s_log, gm, xo, lc); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
