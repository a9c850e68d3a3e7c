// The LDS-staged batched MAC of one tile, as a device function: the body of the batched MAC
// kernel, and a work item of the grouped layer launch.
#pragma once

#include "he_kernels.h"

namespace {

// ------------------------------------------------------------------ batched MAC, LDS-staged
// Residue-class form only.  Per NTT slot the MAC is a small product of an
// (images x J) and a (J x channels) matrix, summed over the s slots of each
// block.  A workgroup takes a tile of TB images x TN channels of one limb and a
// range of slots; per stage (one input row J, R slots) it stages the TB + TN
// rows of R words in LDS (double-buffered, loads of the next stage in flight
// during the products), and each thread accumulates a 4 x 4 sub-tile (images
// bi + TBq u, channels ni + TNq v) over GS consecutive slots of one block, so a
// staged word feeds 4 products from LDS and a global word TB or TN.  Threads are
// split into G groups by slot span; when a block spans several groups their
// sums are added through LDS at the end.  The 64-bit sums are kept below 2^64 by
// replacing hi 2^32 + lo with hi (2^32 mod q) + lo (one multiply-add) every 10
// products, and reduced mod q once at the end.
constexpr int ML_THREADS = 256;
constexpr int ML_UNITS = 4;          // 16-byte staging loads per thread and stage (R <= 32)
constexpr int ML_RED_STRIDE = 17;    // words per thread in the cross-group sum (16 + pad)

// Tile w of the launch geometry gm: w = ((l ranges + range) tiles_n + tn) tiles_b + tb.  The
// workgroup's threads all call it (it meets barriers); some return before the block-sum stores.
// DEV: the block sums are stored with device scope (read by workgroups on other XCDs within the
// same launch).  lds holds max(2 (TB + TN)(R + 2), ML_THREADS ML_RED_STRIDE) words.
template <int GS, bool DEV>
__device__ __forceinline__ void mac_lds_tile(const uint32_t *__restrict__ X, const uint32_t *__restrict__ Op,
                                             uint32_t *__restrict__ h, uint32_t B, uint32_t Jtot, uint32_t Juse,
                                             uint32_t c_o, uint32_t L, uint32_t N, uint32_t s_log,
                                             const MacLdsGeom &gm, uint32_t w, uint32_t *lds, const LimbConsts &lc) {
    // rows padded by two words: 8-byte aligned pairs, and 16 rows of a wave on distinct banks
    const uint32_t TBq = gm.TBq, TNq = gm.TNq, TB = 4 * TBq, TN = 4 * TNq, RP = gm.R + 2, R4 = gm.R >> 2;
    const uint32_t buf_words = (TB + TN) * RP;   // one stage: one input row J, R slots
    const uint32_t tb = w % gm.tiles_b;
    w /= gm.tiles_b;
    const uint32_t tn = w % gm.tiles_n;
    w /= gm.tiles_n;
    const uint32_t range = w % gm.ranges;
    const uint32_t l = w / gm.ranges;
    const uint32_t b0 = tb * TB, n0 = tn * TN;
    const uint32_t tid = threadIdx.x;
    const uint32_t sub = tid % (TBq * TNq);
    const uint32_t g = tid / (TBq * TNq);
    const uint32_t bi = sub / TNq, ni = sub % TNq;
    const LimbConst c = lc.l[l];
    const uint32_t base = range * gm.R * gm.cpb;
    const uint32_t stages = Juse * gm.cpb;
    const uint32_t units = (TB + TN) * R4;

    // staging unit u of stage st: input row J = st / cpb, row u / R4 of the tile (x rows first,
    // then operand rows), 4 words at column 4 (u % R4)
    auto load_stage = [&](uint32_t st, uint4 (&pre)[ML_UNITS]) {
        const uint32_t J = st / gm.cpb, k_st = base + (st % gm.cpb) * gm.R;
#pragma unroll
        for (int i = 0; i < ML_UNITS; ++i) {
            const uint32_t u = tid + i * ML_THREADS;
            if (u < units) {
                const uint32_t row = u / R4, k = k_st + (u % R4) * 4;
                const uint32_t *src;
                if (row < TB) {
                    const uint32_t b = min(b0 + row, B - 1);
                    src = X + (((size_t)b * Jtot + J) * L + l) * N + k;
                } else {
                    const uint32_t n = min(n0 + row - TB, c_o - 1);
                    src = Op + (((size_t)n * L + l) * Jtot + J) * N + k;
                }
                pre[i] = *reinterpret_cast<const uint4 *>(src);
            }
        }
    };
    auto store_stage = [&](uint32_t buf, const uint4 (&pre)[ML_UNITS]) {
        uint32_t *dst = lds + buf * buf_words;
#pragma unroll
        for (int i = 0; i < ML_UNITS; ++i) {
            const uint32_t u = tid + i * ML_THREADS;
            if (u < units) {
                uint2 *d = reinterpret_cast<uint2 *>(dst + (u / R4) * RP + (u % R4) * 4);
                d[0] = make_uint2(pre[i].x, pre[i].y);
                d[1] = make_uint2(pre[i].z, pre[i].w);
            }
        }
    };

    uint64_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0;
    uint32_t pc = 0;   // products in acc since the last fold (uniform)
    uint4 pre[ML_UNITS];
    load_stage(0, pre);
    store_stage(0, pre);
    __syncthreads();
    const uint32_t off = g * GS;   // even: 8-byte aligned pairs
    for (uint32_t st = 0; st < stages; ++st) {
        const uint32_t buf = st & 1u;
        if (st + 1 < stages) load_stage(st + 1, pre);
        const uint32_t *xs = lds + buf * buf_words + off;
        const uint32_t *os = xs + TB * RP;
        const uint2 *xr[4], *orow[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            xr[u] = reinterpret_cast<const uint2 *>(xs + (bi + TBq * u) * RP);
            orow[u] = reinterpret_cast<const uint2 *>(os + (ni + TNq * u) * RP);
        }
#pragma unroll
        for (int k2 = 0; k2 < GS / 2; ++k2) {   // two slots per 8-byte read
            uint2 xv[4], ov[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                xv[u] = xr[u][k2];
                ov[u] = orow[u][k2];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    acc[i][j] += (uint64_t)xv[i].x * ov[j].x;
                    acc[i][j] += (uint64_t)xv[i].y * ov[j].y;
                }
            pc += 2;
            if (pc >= 10) {
                // hi 2^32 + lo == hi (2^32 mod q) + lo: below 2^62 + 2^32, and ten more
                // products keep the sum below 2^64
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[i][j] = (uint64_t)(uint32_t)(acc[i][j] >> 32) * c.r32 + (acc[i][j] & 0xffffffffull);
                pc = 0;
            }
        }
        if (st + 1 < stages) store_stage(buf ^ 1u, pre);
        __syncthreads();
    }
    uint32_t v[16];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) v[i * 4 + j] = reduce64(acc[i][j], c);
    if (gm.gpb > 1) {
        // the gpb groups that share a block are consecutive; the first adds the others' sums
        uint32_t *red = lds;
#pragma unroll
        for (int u = 0; u < 16; ++u) red[tid * ML_RED_STRIDE + u] = v[u];
        __syncthreads();
        if (g % gm.gpb == 0) {
            for (uint32_t p = 1; p < gm.gpb; ++p) {
                const uint32_t *o = red + (tid + p * TBq * TNq) * ML_RED_STRIDE;
#pragma unroll
                for (int u = 0; u < 16; ++u) v[u] = addmod(v[u], o[u], c.q);
            }
        }
    }
    if (g % gm.gpb != 0) return;
    const uint32_t M = N >> s_log;
    const uint32_t m = (base + off) >> s_log;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t b = b0 + bi + TBq * i, n = n0 + ni + TNq * j;
            if (b < B && n < c_o) {
                uint32_t *dst = h + ((size_t)(b * c_o + n) * L + l) * M + m;
                if constexpr (DEV)
                    __hip_atomic_store(dst, v[i * 4 + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                else
                    *dst = v[i * 4 + j];
            }
        }
}



// ------------------------------------------------------------------ batched MAC, staged by LDS DMA
// The products of k_mac_lds with the stages brought in by global_load_lds_dwordx4: a lane's 16
// bytes go straight from memory to LDS (at the wave's base + 16 lane), so a stage takes no
// registers and no store pass, and three stage buffers keep two stages in flight during the
// products.  Rows are not padded (a wave's lanes fill contiguous LDS); instead the 16-byte chunks
// of a row are permuted by an XOR with bits of the row index, so that the rows a wave reads at
// one column fall in different banks.  A wave waits for its own loads of the stage with a
// load-count wait and then meets the others at a plain barrier, which leaves the newer stage's
// loads in flight.
__device__ __forceinline__ void wait_loads_at_most(uint32_t n) {
    // s_waitcnt with vmcnt = n and the other counters at their maxima
    switch (n) {
        case 0: __builtin_amdgcn_s_waitcnt(0x0F70); break;
        case 1: __builtin_amdgcn_s_waitcnt(0x0F71); break;
        case 2: __builtin_amdgcn_s_waitcnt(0x0F72); break;
        case 3: __builtin_amdgcn_s_waitcnt(0x0F73); break;
        default: __builtin_amdgcn_s_waitcnt(0x0F74); break;
    }
}

constexpr int MD_BUFS = 3;

// Tile w of the launch geometry gm (decoded as in mac_lds_tile), staged by DMA; the workgroup's
// threads all call it, with no vector loads of their own outstanding.  DEV: device-scope block-sum
// stores.  lds holds max(MD_BUFS (TB + TN) R, ML_THREADS ML_RED_STRIDE) words.
template <int GS, bool DEV>
__device__ __forceinline__ void mac_dma_tile(const uint32_t *__restrict__ X, const uint32_t *__restrict__ Op,
                                             uint32_t *__restrict__ h, uint32_t B, uint32_t Jtot, uint32_t Juse,
                                             uint32_t c_o, uint32_t L, uint32_t N, uint32_t s_log,
                                             const MacLdsGeom &gm, uint32_t w, uint32_t *lds, const LimbConsts &lc) {
    const uint32_t TBq = gm.TBq, TNq = gm.TNq, TB = 4 * TBq, TN = 4 * TNq, R = gm.R;
    const uint32_t R4 = R >> 2, r4_log = 31u - __clz(R4);
    // rows whose starts share a bank (R words apart, 32 banks) get distinct chunk permutations;
    // at R >= 32 every row starts on bank 0 and the low row bits spread 8 rows over the banks
    const uint32_t sw_shift = R >= 32 ? 0u : 5u - (31u - __clz(R));
    const uint32_t buf_words = (TB + TN) * R;
    const uint32_t tb = w % gm.tiles_b;
    w /= gm.tiles_b;
    const uint32_t tn = w % gm.tiles_n;
    w /= gm.tiles_n;
    const uint32_t range = w % gm.ranges;
    const uint32_t l = w / gm.ranges;
    const uint32_t b0 = tb * TB, n0 = tn * TN;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint32_t sub = tid % (TBq * TNq);
    const uint32_t g = tid / (TBq * TNq);
    const uint32_t bi = sub / TNq, ni = sub % TNq;
    const LimbConst c = lc.l[l];
    const uint32_t cpb = gm.cpb, gpb = gm.gpb;   // (locals: the lambdas below capture by reference)
    const uint32_t base = range * R * cpb;
    const uint32_t stages = Juse * cpb;
    const uint32_t units = (TB + TN) * R4;
    // load instructions this wave issues per stage (the same for every stage)
    uint32_t nld = 0;
#pragma unroll
    for (int i = 0; i < ML_UNITS; ++i) nld += (i * ML_THREADS + 64u * wave < units) ? 1u : 0u;

    // slot u of a stage buffer holds chunk (u mod R4) ^ swz(row) of row u / R4 (x rows first,
    // then operand rows) of input row J = st / cpb
    auto issue = [&](uint32_t st, uint32_t buf) {
        const uint32_t J = st / cpb, k_st = base + (st % cpb) * R;
        uint32_t *dst = lds + buf * buf_words;
#pragma unroll
        for (int i = 0; i < ML_UNITS; ++i) {
            const uint32_t u0 = i * ML_THREADS + 64u * wave;   // first slot of this wave's lanes
            if (u0 < units) {
                const uint32_t u = u0 + lane;
                const uint32_t uc = u < units ? u : units - 1u;
                const uint32_t row = uc >> r4_log;
                const uint32_t chunk = (uc & (R4 - 1u)) ^ ((row >> sw_shift) & (R4 - 1u));
                const uint32_t k = k_st + chunk * 4u;
                // both candidate addresses as integers, then one select (a per-lane choice between
                // the two base pointers would otherwise go through a stack array)
                const uint32_t b = min(b0 + row, B - 1);
                const uint32_t n = min(n0 + (row < TB ? 0u : row - TB), c_o - 1);
                const uintptr_t xa = reinterpret_cast<uintptr_t>(X + ((((size_t)b * Jtot + J) * L + l) * N + k));
                const uintptr_t oa = reinterpret_cast<uintptr_t>(Op + ((((size_t)n * L + l) * Jtot + J) * N + k));
                const uint32_t *src = reinterpret_cast<const uint32_t *>(row < TB ? xa : oa);
                if (u < units) __builtin_amdgcn_global_load_lds(src, dst + u0 * 4u, 16, 0, 0);
            }
        }
    };

    uint64_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0;
    uint32_t pc = 0;   // products in acc since the last fold (uniform)
    const uint32_t off = g * GS;
    // row r's word at column 4 ch + wd sits at r R + ((ch ^ sw(r)) << 2) + wd; with R a power of two
    // and (ch ^ sw) << 2 below R this is (r R | sw(r) << 2) ^ (ch << 2), plus wd: one register per row
    uint32_t xb[4], ob[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const uint32_t rx = bi + TBq * u, ro = TB + ni + TNq * u;
        xb[u] = rx * R | (((rx >> sw_shift) & (R4 - 1u)) << 2);
        ob[u] = ro * R | (((ro >> sw_shift) & (R4 - 1u)) << 2);
    }
    issue(0, 0);
    if (stages > 1) issue(1, 1);
    for (uint32_t st = 0; st < stages; ++st) {
        // this stage has landed once at most the next one's loads remain in flight
        wait_loads_at_most(st + 1 < stages ? nld : 0u);
        __builtin_amdgcn_s_barrier();
        if (st + 2 < stages) issue(st + 2, (st + 2) % MD_BUFS);
        const uint32_t *sb = lds + (st % MD_BUFS) * buf_words;
        // unrolled by two, not fully: 102 registers instead of 146-162, one more wave per SIMD
#pragma unroll 2
        for (int k2 = 0; k2 < GS / 2; ++k2) {   // two slots per 8-byte read
            const uint32_t k = off + 2u * k2;
            const uint32_t ch = k >> 2, wd = k & 3u;
            uint2 xv[4], ov[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                xv[u] = *reinterpret_cast<const uint2 *>(sb + (xb[u] ^ (ch << 2)) + wd);
                ov[u] = *reinterpret_cast<const uint2 *>(sb + (ob[u] ^ (ch << 2)) + wd);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    acc[i][j] += (uint64_t)xv[i].x * ov[j].x;
                    acc[i][j] += (uint64_t)xv[i].y * ov[j].y;
                }
            pc += 2;
            if (pc >= 10) {
                // hi 2^32 + lo == hi (2^32 mod q) + lo: below 2^62 + 2^32, and ten more
                // products keep the sum below 2^64
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[i][j] = (uint64_t)(uint32_t)(acc[i][j] >> 32) * c.r32 + (acc[i][j] & 0xffffffffull);
                pc = 0;
            }
        }
    }
    uint32_t v[16];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) v[i * 4 + j] = reduce64(acc[i][j], c);
    if (gpb > 1) {
        // the gpb groups that share a block are consecutive; the first adds the others' sums
        __syncthreads();   // every wave is done with the stage buffers
        uint32_t *red = lds;
#pragma unroll
        for (int u = 0; u < 16; ++u) red[tid * ML_RED_STRIDE + u] = v[u];
        __syncthreads();
        if (g % gpb == 0) {
            for (uint32_t p = 1; p < gpb; ++p) {
                const uint32_t *o = red + (tid + p * TBq * TNq) * ML_RED_STRIDE;
#pragma unroll
                for (int u = 0; u < 16; ++u) v[u] = addmod(v[u], o[u], c.q);
            }
        }
    }
    if (g % gpb != 0) return;
    const uint32_t M = N >> s_log;
    const uint32_t m = (base + off) >> s_log;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t b = b0 + bi + TBq * i, n = n0 + ni + TNq * j;
            if (b < B && n < c_o) {
                uint32_t *dst = h + ((size_t)(b * c_o + n) * L + l) * M + m;
                if constexpr (DEV)
                    __hip_atomic_store(dst, v[i * 4 + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                else
                    *dst = v[i * 4 + j];
            }
        }
}

}  // namespace
