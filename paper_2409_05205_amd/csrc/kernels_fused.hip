// One launch per layer call: forward NTT, coefficient-wise MAC and the inverse with extraction
// (Alg. 1 / Alg. 2 server evaluation; the NTT-domain products of Sec. IV-A-1).
//
// The launch is a list of work items, one per workgroup, in workgroup-id order.  Items come in
// three phases, in this order:
//
//   NTT   sub-block `sub` (of 4) of the forward transform of one input row (b, j, l): the two
//         leading stages are formed on load from the whole row, the remaining N/4-point
//         transform runs alone (the split of the multi-workgroup forward transform).
//   MAC   image b, limb l, a chunk of 1024 slots and a group of output channels: the products
//         summed over the input rows, folded over the s slots of each residue block (conv) into
//         the block sums h, or (FC) multiplied out to this chunk's share of the first n_o'
//         inverse-transform coefficients.
//   TAIL  (conv) the (N/s)-point inverse of RW channel vectors of one output group and limb,
//         scattered to their residue classes plus Delta sh' (as the residue-class tail kernel).
//
// An item waits only for items of lower ids, through counters in a small zeroed "sync block": a
// MAC item for the NTT sub-block it reads, a tail item for every MAC item of its image and limb.
// Each XCD starts the workgroups dealt to it in id order, so the lowest-id item that has not
// finished either runs or waits for a slot held by lower ids of its XCD, and the items it waits
// for have lower ids still: every wait ends.  Before waiting, a MAC item issues the loads of
// its first channel's resident operands, so that the operand stream overlaps the forward
// transforms.  A wait that does not end within FZ_SPIN_LIMIT polls sets an error word and gives
// up (the words are then undefined), so a launch always drains.  Each counter is returned to
// zero by the last item that uses it (found by the value an atomic add returns), so the sync
// block is zero again for the next launch that uses it.
//
// Visibility across the XCDs' separate L2 caches without writing back or invalidating whole
// caches: every word one item hands to another (NTT outputs, block sums, FC shares) is stored
// with device scope (written through to the device's point of coherence), each thread waits
// for its stores to complete, the workgroup meets at a barrier, and only then does thread 0
// add to the counter.  A consumer polls the counter with device-scope loads; it reads block
// sums and shares with device-scope loads, and NTT outputs with plain loads: every line of an
// NTT output is written whole by one item, no workgroup reads it before its counter says it is
// written, and the caches hold nothing of it from before the launch (they are invalidated when
// a launch starts), so no cache can return a stale copy.  Counters sit one per 128-byte line
// when the sync block has room (ctr_stride), so that polls of different counters do not queue
// behind each other.
//
// FC: the first n_o' coefficients of an N-point inverse are c[m] = sum_k A[k] x_k^-m (N^-1 is
// folded into the operands), so each MAC item adds its chunk's share of them for m in a range
// of up to 16, reduced over the workgroup; the last item of a block (by a counter) sums the
// chunk shares and adds Delta (d + sh').  No full-length inverse is run.

#include "he_kernels.h"
#include "mac_device.h"
#include "ntt_device.h"

namespace {

constexpr int FZ_THREADS = 256;
constexpr uint32_t FZ_CHUNK = 4 * FZ_THREADS;      // slots per MAC item
constexpr uint32_t FZ_SPIN_LIMIT = 1u << 24;       // polls (s_sleep 2 each, about 2^24 x 0.1 us) before a wait gives up
constexpr int FZ_LDS = 4096 + 128;                 // words: an N/4-point sub-block or a tail of <= 4096 points
constexpr int FZ_MR = 16;                          // FC output coefficients per item
constexpr int FZ_JB = 4;                           // input rows per MAC register block

// Device-scope load and store of one word (the handed-over data and the counters).
__device__ __forceinline__ uint32_t ld_dev(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// This thread's stores have completed (and the compiler keeps every memory access on its side).
__device__ __forceinline__ void stores_done() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Every thread's device-scope stores of this item have completed; then thread 0 adds v.
__device__ __forceinline__ void fz_signal(uint32_t *ctr, uint32_t v) {
    stores_done();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(ctr, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// As fz_signal with v = 1; true in every thread of the item whose add completes the count
// `total` (every other user of the counter has then added).
__device__ __forceinline__ bool fz_signal_last(uint32_t *ctr, uint32_t total) {
    __shared__ uint32_t s_last;
    stores_done();
    __syncthreads();
    if (threadIdx.x == 0)
        s_last = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == total - 1u;
    __syncthreads();
    return s_last != 0;
}

// Two counters at once (thread 0 adds to a, thread 64 to b): *last_a / *last_b as fz_signal_last.
__device__ __forceinline__ void fz_signal_last2(uint32_t *a, uint32_t total_a, uint32_t *b, uint32_t total_b,
                                                bool *last_a, bool *last_b) {
    __shared__ uint32_t s_last2[2];
    stores_done();
    __syncthreads();
    if (threadIdx.x == 0)
        s_last2[0] = __hip_atomic_fetch_add(a, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == total_a - 1u;
    if (threadIdx.x == 64)
        s_last2[1] = __hip_atomic_fetch_add(b, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == total_b - 1u;
    __syncthreads();
    *last_a = s_last2[0] != 0;
    *last_b = s_last2[1] != 0;
}

// Thread 0 polls until *ctr >= target (or the poll limit); the workgroup then goes on together.
__device__ __forceinline__ void fz_wait(const uint32_t *ctr, uint32_t target, uint32_t *err) {
    if (threadIdx.x == 0 && target > 0) {
        uint32_t n = 0;
        while (ld_dev(ctr) < target) {
            if (++n > FZ_SPIN_LIMIT) {
                __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    __syncthreads();
}

__device__ __forceinline__ uint32_t mulmod(uint32_t a, uint32_t b, const LimbConst &c) {
    return reduce64((uint64_t)a * b, c);
}

// Images of counter tile bt (tiles of 2^tile_log images; the last may be short).
__device__ __forceinline__ uint32_t fz_tile_imgs(const FusedLayer &jb, uint32_t bt) {
    const uint32_t first = bt << jb.tile_log, n = 1u << jb.tile_log;
    return jb.B - first < n ? jb.B - first : n;
}

// ------------------------------------------------------------------ NTT items
// TWB: the workgroup size the twiddle prefetch is sized for (PassTw); a larger value keeps fewer
// twiddles in registers.  K: the row is transformed as 2^K sub-blocks of N / 2^K points, one per
// item (K = 0: the whole row); an item counts itself done for each quarter of the row it covers.
template <int LOGN, int TWB = FZ_THREADS, int K = 2>
__device__ __forceinline__ void fz_ntt_item(const FusedLayer &jb, uint32_t it, uint32_t *lds, const uint32_t *__restrict__ tw,
                            const uint32_t *__restrict__ twsh, const LimbConsts &lc, uint32_t *ctr) {
    static_assert(K >= 0 && K <= 2, "whole rows, halves or quarters");
    constexpr int LS = LOGN - K;
    constexpr int NS = 1 << LS;
    constexpr int LOGR = LS - 8;                     // 256 threads per sub-block
    constexpr int T = 1 << (LS - LOGR);
    static_assert(T == FZ_THREADS, "one sub-block per workgroup");
    const uint32_t tid = threadIdx.x;
    const uint32_t sub = it & ((1u << K) - 1u);
    uint32_t r = it >> K;
    const uint32_t L = jb.L;
    const uint32_t l = r % L;
    r /= L;
    const uint32_t R = jb.ntt_c0 + jb.ntt_sh;
    const uint32_t jj = r % R;
    const uint32_t b = r / R;
    const uint32_t N = 1u << LOGN;
    const uint32_t *in;
    uint32_t jrow;
    if (jj < jb.ntt_c0) {
        jrow = jj;
        in = jb.c0 + ((size_t)(b * jb.K_in + jj) * L + l) * N;
    } else {
        jrow = jb.K_in + (jj - jb.ntt_c0);
        in = jb.sh + (size_t)(b * jb.K_in + (jj - jb.ntt_c0)) * N;   // shares carry no limb axis
    }
    uint32_t *out = jb.x + ((size_t)(b * jb.Jtot + jrow) * L + l) * N + (size_t)sub * NS;
    const uint32_t q = lc.l[l].q, q2 = lc.l[l].q2;
    const uint32_t *W = tw + (size_t)l * N;
    const uint32_t *Wsh = twsh + (size_t)l * N;
    const uint32_t tb = (1u << K) + sub;
    // twiddles of the leading passes in registers: loads under the operand stream are slow
    PassTw<LS, LOGR, TWB> ptw;
    fwd_tw_load<LS, LOGR, TWB, 0>(ptw, tid, W, Wsh, tb);
    uint32_t v[1 << LOGR];
    fwd_pass<LS, LOGR, TWB, 0, K>(v, ptw, lds, tid, in, W, Wsh, q, q2, tb, sub);
#pragma unroll
    for (int i = 0; i < (1 << LOGR); ++i) {
        const uint32_t idx = tid + i * T;
        uint32_t y = lds[lpad(idx)];
        y = csub(y, q2);
        st_dev(out + idx, csub(y, q));
    }
    stores_done();
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t *c4 = ctr + ((b >> jb.tile_log) * L + l) * 4u * jb.ctr_stride;
#pragma unroll
        for (int qq = 0; qq < (4 >> K); ++qq)
            __hip_atomic_fetch_add(c4 + ((sub << (2 - K)) + qq) * jb.ctr_stride, 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Sub-blocks per row of the grouped launch's NTT items: whole rows up to 8192 points (the group's
// LDS holds one), halves of a 16384-point row.
constexpr int fz_group_ntt_k(int logn) { return logn > 13 ? logn - 13 : 0; }

// ------------------------------------------------------------------ MAC items (conv)
// The per-image MAC items below run with one image per counter tile (tile_log = 0).
// Image b, limb l, slots [c 1024, (c + 1) 1024) (4 per thread), channels [n0, n1).
__device__ __forceinline__ void fz_mac_conv_item(const FusedLayer &jb, uint32_t it, const LimbConsts &lc, uint32_t *ctr,
                                 uint32_t *err) {
    const uint32_t tid = threadIdx.x;
    const uint32_t N = 1u << jb.logN, L = jb.L, Juse = jb.Juse, Jtot = jb.Jtot;
    const uint32_t chunks = N / FZ_CHUNK;
    const uint32_t ngroups = (jb.rows + jb.ng - 1) / jb.ng;
    const uint32_t grp = it % ngroups;
    it /= ngroups;
    const uint32_t cidx = it % chunks;
    it /= chunks;
    const uint32_t l = it % L;
    const uint32_t b = it / L;
    const uint32_t n0 = grp * jb.ng;
    const uint32_t n1 = n0 + jb.ng < jb.rows ? n0 + jb.ng : jb.rows;
    const LimbConst c = lc.l[l];
    const uint32_t k0 = cidx * FZ_CHUNK + 4u * tid;
    const size_t xs = (size_t)L * N;                       // between input rows of one image and limb
    const size_t ocs = (size_t)L * Jtot * N;               // between channels of the operands
    const uint32_t *xb = jb.x + ((size_t)b * Jtot * L + l) * N + k0;
    const uint32_t *ob = jb.op + (size_t)l * Jtot * N + k0;
    // operand blocks of FZ_JB rows in order over (channel, block); two blocks stay in flight:
    // the first two are loaded before the wait, each later one as soon as a buffer frees
    const uint32_t nb = (Juse + FZ_JB - 1) / FZ_JB;
    const uint32_t steps = (n1 - n0) * nb;
    auto load_block = [&](uint32_t idx, uint4 (&o)[FZ_JB]) {
        if (idx >= steps) return;
        const uint32_t n = n0 + idx / nb, j0 = (idx % nb) * FZ_JB;
        const uint32_t *p = ob + n * ocs + (size_t)j0 * N;
#pragma unroll
        for (int u = 0; u < FZ_JB; ++u)
            if (j0 + u < Juse) o[u] = *reinterpret_cast<const uint4 *>(p + (size_t)u * N);
    };
    uint4 o0[FZ_JB], o1[FZ_JB];
    load_block(0, o0);
    load_block(1, o1);
    const uint32_t sub = (cidx * FZ_CHUNK) >> (jb.logN - 2);
    fz_wait(ctr + ((b * L + l) * 4u + sub) * jb.ctr_stride, jb.ntt_c0 + jb.ntt_sh, err);
    const uint32_t s_log = jb.s_log;
    const uint32_t M = N >> s_log;
    uint64_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    auto step = [&](uint32_t idx, const uint4 (&o)[FZ_JB]) {
        const uint32_t n = n0 + idx / nb, blk = idx % nb, j0 = blk * FZ_JB;
        uint4 xv[FZ_JB];
#pragma unroll
        for (int u = 0; u < FZ_JB; ++u)
            if (j0 + u < Juse) xv[u] = *reinterpret_cast<const uint4 *>(xb + (size_t)(j0 + u) * xs);
#pragma unroll
        for (int u = 0; u < FZ_JB; ++u) {
            if (j0 + u < Juse) {
                a0 += (uint64_t)xv[u].x * o[u].x;
                a1 += (uint64_t)xv[u].y * o[u].y;
                a2 += (uint64_t)xv[u].z * o[u].z;
                a3 += (uint64_t)xv[u].w * o[u].w;
            }
        }
        // FZ_JB products of two residues plus a carried residue stay below 2^64
        a0 = reduce64(a0, c);
        a1 = reduce64(a1, c);
        a2 = reduce64(a2, c);
        a3 = reduce64(a3, c);
        if (blk + 1 < nb) return;
        uint32_t *hrow = jb.h + ((size_t)(b * jb.rows + n) * L + l) * M;
        if (s_log == 1) {
            st_dev(hrow + (k0 >> 1), addmod((uint32_t)a0, (uint32_t)a1, c.q));
            st_dev(hrow + (k0 >> 1) + 1, addmod((uint32_t)a2, (uint32_t)a3, c.q));
        } else {
            // the s slots of a block are held by s/4 consecutive lanes of one wave
            uint32_t v = (uint32_t)a0 + (uint32_t)a1 + (uint32_t)a2 + (uint32_t)a3;   // [0, 4q)
            v = csub(csub(v, c.q2), c.q);
            const uint32_t lanes = 1u << (s_log - 2);
            for (uint32_t m = 1; m < lanes; m <<= 1) v = addmod(v, (uint32_t)__shfl_xor((int)v, (int)m), c.q);
            if ((tid & (lanes - 1)) == 0) st_dev(hrow + (k0 >> s_log), v);
        }
        a0 = a1 = a2 = a3 = 0;
    };
    for (uint32_t idx = 0; idx < steps; idx += 2) {
        step(idx, o0);
        load_block(idx + 2, o0);
        if (idx + 1 < steps) {
            step(idx + 1, o1);
            load_block(idx + 3, o1);
        }
    }
    // the last MAC item of (b, l) returns the NTT counters it waited on to zero
    const uint32_t per_bl = chunks * ngroups;
    if (fz_signal_last(ctr + (jb.n_tiles * L * 4u + b * L + l) * jb.ctr_stride, per_bl) && threadIdx.x < 4)
        st_dev(ctr + ((b * L + l) * 4u + threadIdx.x) * jb.ctr_stride, 0u);
}

// ------------------------------------------------------------------ MAC items, all channels (conv)
// Image b, limb l, slots [c 128, (c + 1) 128) for every output channel: a group of 32 lanes
// covers the 128 slots (4 per lane) and the 8 groups take channels n = g, g + 8, ...  The
// NTT-domain input rows of the chunk are read once, into registers, and reused for every
// channel.  A lane's operand words go in rounds of FZ_WROUND 16-byte loads ((channel, row) in
// order); the first round is loaded before the wait, so that for the plain-20 shapes (at most
// 16 (channel, row) pairs per lane) the whole operand stream overlaps the forward transforms.
// JU = Juse (1, 2, 4 or 8); s <= 128 (a residue block within one group of lanes).
constexpr uint32_t FZ_WCHUNK = 128;
constexpr int FZ_WROUND = 16;

template <int JU>
__device__ __forceinline__ void fz_mac_wide_item(const FusedLayer &jb, uint32_t it, const LimbConsts &lc,
                                                 uint32_t *ctr, uint32_t *err) {
    constexpr int CH = FZ_WROUND / JU;             // channels per round
    const uint32_t tid = threadIdx.x, lane = tid & 31u, grp = tid >> 5;
    const uint32_t N = 1u << jb.logN, L = jb.L, Jtot = jb.Jtot, c_o = jb.rows;
    const uint32_t chunks = N / FZ_WCHUNK;
    const uint32_t cidx = it % chunks;
    it /= chunks;
    const uint32_t l = it % L;
    const uint32_t b = it / L;
    const LimbConst c = lc.l[l];
    const uint32_t k0 = cidx * FZ_WCHUNK + 4u * lane;
    const size_t xs = (size_t)L * N;
    const size_t ocs = (size_t)L * Jtot * N;
    const uint32_t *xb = jb.x + ((size_t)b * Jtot * L + l) * N + k0;
    const uint32_t *ob = jb.op + (size_t)l * Jtot * N + k0;
    const uint32_t nch = grp < c_o ? (c_o - grp + 7u) / 8u : 0u;   // channels of this group
    const uint32_t rounds = (nch + CH - 1) / CH;
    uint4 o[FZ_WROUND];
    auto load_round = [&](uint32_t r) {
#pragma unroll
        for (int f = 0; f < FZ_WROUND; ++f) {
            const uint32_t m = r * CH + f / JU;
            if (m < nch) o[f] = *reinterpret_cast<const uint4 *>(ob + (grp + 8u * m) * ocs + (size_t)(f % JU) * N);
        }
    };
    if (rounds) load_round(0);
    const uint32_t sub = (cidx * FZ_WCHUNK) >> (jb.logN - 2);
    fz_wait(ctr + ((b * L + l) * 4u + sub) * jb.ctr_stride, jb.ntt_c0 + jb.ntt_sh, err);
    uint4 xv[JU];
#pragma unroll
    for (int j = 0; j < JU; ++j) xv[j] = *reinterpret_cast<const uint4 *>(xb + (size_t)j * xs);
    const uint32_t s_log = jb.s_log;
    const uint32_t M = N >> s_log;
    for (uint32_t r = 0; r < rounds; ++r) {
#pragma unroll
        for (int mm = 0; mm < CH; ++mm) {
            const uint32_t m = r * CH + mm;
            if (m >= nch) break;                   // uniform over the group
            uint64_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
            for (int j = 0; j < JU; ++j) {
                const uint4 w = o[mm * JU + j];
                a0 += (uint64_t)xv[j].x * w.x;
                a1 += (uint64_t)xv[j].y * w.y;
                a2 += (uint64_t)xv[j].z * w.z;
                a3 += (uint64_t)xv[j].w * w.w;
            }
            // at most 8 products of two residues: below 2^64
            const uint32_t r0 = reduce64(a0, c), r1 = reduce64(a1, c), r2 = reduce64(a2, c), r3 = reduce64(a3, c);
            const uint32_t n = grp + 8u * m;
            uint32_t *hrow = jb.h + ((size_t)(b * c_o + n) * L + l) * M;
            if (s_log == 1) {
                st_dev(hrow + (k0 >> 1), addmod(r0, r1, c.q));
                st_dev(hrow + (k0 >> 1) + 1, addmod(r2, r3, c.q));
            } else {
                // the s slots of a block are held by s/4 consecutive lanes of one group
                uint32_t v = r0 + r1 + r2 + r3;   // [0, 4q)
                v = csub(csub(v, c.q2), c.q);
                const uint32_t lanes = 1u << (s_log - 2);
                for (uint32_t mk = 1; mk < lanes; mk <<= 1) v = addmod(v, (uint32_t)__shfl_xor((int)v, (int)mk), c.q);
                if ((lane & (lanes - 1)) == 0) st_dev(hrow + (k0 >> s_log), v);
            }
        }
        if (r + 1 < rounds) load_round(r + 1);
    }
    // the count only: the NTT counters of (b, l) are returned to zero by its last tail item
    fz_signal(ctr + (jb.n_tiles * L * 4u + b * L + l) * jb.ctr_stride, 1u);
}

__device__ __forceinline__ void fz_mac_wide_switch(const FusedLayer &jb, uint32_t it, const LimbConsts &lc,
                                                   uint32_t *ctr, uint32_t *err) {
    switch (jb.Juse) {
        case 1: fz_mac_wide_item<1>(jb, it, lc, ctr, err); break;
        case 2: fz_mac_wide_item<2>(jb, it, lc, ctr, err); break;
        case 4: fz_mac_wide_item<4>(jb, it, lc, ctr, err); break;
        default: fz_mac_wide_item<8>(jb, it, lc, ctr, err); break;
    }
}

// ------------------------------------------------------------------ MAC items, image tiles (conv)
// Grouped launch at larger batches: one tile of the batched MAC staged in LDS by DMA (images x
// channels of one limb over a range of slots, mac_device.h) per item, so that a resident operand
// word is read once per tile of images instead of once per image.  It waits for the NTT sub-block holding its
// slot range for every image of its tile (one counter per tile), stores its block sums with
// device scope and counts itself done for the tile.
template <int GS>
__device__ __forceinline__ void fz_mac_tile_item(const FusedLayer &jb, uint32_t it, uint32_t *lds,
                                                 const LimbConsts &lc, uint32_t *ctr, uint32_t *err) {
    const MacLdsGeom &gm = jb.gm;
    const uint32_t L = jb.L;
    uint32_t w = it;
    const uint32_t bt = w % gm.tiles_b;
    w /= gm.tiles_b;
    w /= gm.tiles_n;
    const uint32_t range = w % gm.ranges;
    const uint32_t l = w / gm.ranges;
    const uint32_t sub = (range * gm.R * gm.cpb) >> (jb.logN - 2);
    fz_wait(ctr + ((bt * L + l) * 4u + sub) * jb.ctr_stride, fz_tile_imgs(jb, bt) * (jb.ntt_c0 + jb.ntt_sh), err);
    mac_dma_tile<GS, true>(jb.x, jb.op, jb.h, jb.B, jb.Jtot, jb.Juse, jb.rows, L, 1u << jb.logN, jb.s_log, gm, it,
                           lds, lc);
    fz_signal(ctr + (jb.n_tiles * L * 4u + bt * L + l) * jb.ctr_stride, 1u);
}

__device__ __forceinline__ void fz_mac_tile_switch(const FusedLayer &jb, uint32_t it, uint32_t *lds,
                                                   const LimbConsts &lc, uint32_t *ctr, uint32_t *err) {
    switch (jb.gm.GS) {
        case 2: fz_mac_tile_item<2>(jb, it, lds, lc, ctr, err); break;
        case 4: fz_mac_tile_item<4>(jb, it, lds, lc, ctr, err); break;
        case 8: fz_mac_tile_item<8>(jb, it, lds, lc, ctr, err); break;
        default: fz_mac_tile_item<16>(jb, it, lds, lc, ctr, err); break;
    }
}

// ------------------------------------------------------------------ tail items (conv)
// The residue-class tail of one output group and limb for RW channel vectors of M = N/s points
// (the steps of the residue-class tail kernel in kernels_ntt.hip, in a 256-thread item).  LOGR
// words per thread (T = M / 2^LOGR threads per vector); TWB sizes the twiddle prefetch (PassTw).
template <int LOGM, int LOGR = (LOGM - 8 > 2 ? LOGM - 8 : 2), int TWB = FZ_THREADS>
__device__ __forceinline__ void fz_tail_item(const FusedLayer &jb, uint32_t it, uint32_t *lds, const uint32_t *__restrict__ twi,
                             const uint32_t *__restrict__ twish, const LimbConsts &lc, uint32_t *ctr, uint32_t *err) {
    constexpr int M = 1 << LOGM;
    constexpr int T = 1 << (LOGM - LOGR);
    constexpr int MP = M + (M >> 5);
    static_assert(T <= FZ_THREADS, "one channel vector fits a workgroup");
    const uint32_t tid = threadIdx.x;
    const uint32_t row = tid / T;
    const uint32_t t = tid % T;
    const uint32_t L = jb.L, g_o = jb.g_o, K_out = jb.K_out, c_o = jb.rows, RW = jb.tail_rw;
    const uint32_t chunks = g_o / RW;
    uint32_t w = it;
    const uint32_t chunk = w % chunks;
    w /= chunks;
    const uint32_t l = w % L;
    w /= L;
    const uint32_t g = w % K_out;
    const uint32_t b = w / K_out;
    const LimbConst c = lc.l[l];
    const uint32_t logN = jb.logN, s_log = jb.s_log;
    const uint32_t N = 1u << logN;
    const uint32_t np0 = chunk * RW;
    uint32_t *my = lds + row * MP;
    const bool active = row < RW;
    const uint32_t n = g * g_o + np0 + row;
    const bool exists = active && n < c_o;
    const uint32_t *W = twi + (size_t)l * N;
    const uint32_t *Wsh = twish + (size_t)l * N;
    PassTw<LOGM, LOGR, TWB> ptw;
    inv_tw_load<LOGM, LOGR, TWB, 0>(ptw, t, W, Wsh);
    const uint32_t cw_log = s_log - (31u - __clz(g_o));
    const uint32_t span_log = (31u - __clz(RW)) + cw_log;
    const uint32_t c_lo = np0 << cw_log;
    const uint32_t *sh = jb.sh_next ? jb.sh_next + (size_t)(b * K_out + g) * N : nullptr;
    const uint32_t total = (uint32_t)M << span_log;
    // the sh' words of the first write rounds are fetched before the wait
    constexpr int TPF = 8;
    uint32_t shv[TPF];
#pragma unroll
    for (int i = 0; i < TPF; ++i) {
        const uint32_t e = tid + i * FZ_THREADS;
        shv[i] = (sh && e < total) ? sh[((e >> span_log) << s_log) + c_lo + (e & ((1u << span_log) - 1u))] : 0u;
    }
    const uint32_t bt = b >> jb.tile_log;
    fz_wait(ctr + (jb.n_tiles * L * 4u + bt * L + l) * jb.ctr_stride, jb.mac_per_bl, err);
    if (active) {
        const uint32_t *src = jb.h + ((size_t)(b * c_o + (exists ? n : 0)) * L + l) * M;
#pragma unroll
        for (int i = 0; i < (1 << LOGR); ++i) {
            const uint32_t idx = t + i * T;
            my[lpad(idx)] = exists ? ld_dev(src + idx) : 0u;
        }
    }
    __syncthreads();
    uint32_t v[1 << LOGR];
    inv_pass<LOGM, LOGR, TWB, 0>(v, ptw, my, t, W, Wsh, c.q, c.q2, active);
    __syncthreads();
    if (active) {
#pragma unroll
        for (int i = 0; i < (1 << LOGR); ++i) my[lpad(inv_final_idx<LOGM, LOGR>(t, i))] = csub(v[i], c.q);
    }
    __syncthreads();
    uint32_t *o = jb.out + ((size_t)(b * K_out + g) * L + l) * N;
    auto put = [&](uint32_t e, uint32_t shw) {
        const uint32_t m = e >> span_log;
        const uint32_t off = e & ((1u << span_log) - 1u);
        const uint32_t rr = off >> cw_log;
        uint32_t val = 0;
        if ((off & ((1u << cw_log) - 1u)) == 0 && g * g_o + np0 + rr < c_o) val = lds[rr * MP + lpad(m)];
        if (sh) val = csub(val + mul_delta_msg(shw, c), c.q);
        o[(m << s_log) + c_lo + off] = val;
    };
#pragma unroll
    for (int i = 0; i < TPF; ++i) {
        const uint32_t e = tid + i * FZ_THREADS;
        if (e < total) put(e, shv[i]);
    }
    for (uint32_t e = tid + TPF * FZ_THREADS; e < total; e += FZ_THREADS) {
        const uint32_t m = e >> span_log, off = e & ((1u << span_log) - 1u);
        put(e, sh ? sh[(m << s_log) + c_lo + off] : 0u);
    }
    // the last tail item of the tile and limb returns its counters to zero (every tail of them has
    // waited); the NTT counters too, unless the MAC items do that (ng > 0)
    uint32_t *mac_done = ctr + (jb.n_tiles * L * 4u + bt * L + l) * jb.ctr_stride;
    uint32_t *tail_done = ctr + (jb.n_tiles * L * 5u + bt * L + l) * jb.ctr_stride;
    if (fz_signal_last(tail_done, K_out * chunks * fz_tile_imgs(jb, bt))) {
        if (threadIdx.x == 0) {
            st_dev(mac_done, 0u);
            st_dev(tail_done, 0u);
        }
        if (jb.ng == 0 && threadIdx.x < 4) st_dev(ctr + ((bt * L + l) * 4u + threadIdx.x) * jb.ctr_stride, 0u);
    }
}

__device__ __forceinline__ void fz_tail_switch(const FusedLayer &jb, uint32_t it, uint32_t *lds, const uint32_t *twi,
                               const uint32_t *twish, const LimbConsts &lc, uint32_t *ctr, uint32_t *err) {
    switch (jb.logN - jb.s_log) {
        case 4: fz_tail_item<4>(jb, it, lds, twi, twish, lc, ctr, err); break;
        case 5: fz_tail_item<5>(jb, it, lds, twi, twish, lc, ctr, err); break;
        case 6: fz_tail_item<6>(jb, it, lds, twi, twish, lc, ctr, err); break;
        case 7: fz_tail_item<7>(jb, it, lds, twi, twish, lc, ctr, err); break;
        case 8: fz_tail_item<8>(jb, it, lds, twi, twish, lc, ctr, err); break;
        case 9: fz_tail_item<9>(jb, it, lds, twi, twish, lc, ctr, err); break;
        case 10: fz_tail_item<10>(jb, it, lds, twi, twish, lc, ctr, err); break;
        case 11: fz_tail_item<11>(jb, it, lds, twi, twish, lc, ctr, err); break;
        case 12: fz_tail_item<12>(jb, it, lds, twi, twish, lc, ctr, err); break;
        default: break;   // excluded by the host (fused_layer_ok)
    }
}

// Tails in the grouped launch: 64 threads per vector from 256 points up (four or more vectors per
// item; 128 threads at 4096 points), twiddles read per pass (registers go to occupancy).
constexpr int fz_group_tail_logr(int logm) { return logm >= 8 ? (logm - 6 < 5 ? logm - 6 : 5) : 2; }

__device__ __forceinline__ void fz_tail_switch_group(const FusedLayer &jb, uint32_t it, uint32_t *lds,
                                                     const uint32_t *twi, const uint32_t *twish, const LimbConsts &lc,
                                                     uint32_t *ctr, uint32_t *err) {
#define FZ_GT(LM) fz_tail_item<LM, fz_group_tail_logr(LM), TW_IN_PASS>(jb, it, lds, twi, twish, lc, ctr, err)
    switch (jb.logN - jb.s_log) {
        case 4: FZ_GT(4); break;
        case 5: FZ_GT(5); break;
        case 6: FZ_GT(6); break;
        case 7: FZ_GT(7); break;
        case 8: FZ_GT(8); break;
        case 9: FZ_GT(9); break;
        case 10: FZ_GT(10); break;
        case 11: FZ_GT(11); break;
        case 12: FZ_GT(12); break;
        default: break;   // excluded by the host (fused_layer_ok)
    }
#undef FZ_GT
}

// ------------------------------------------------------------------ FC items
// Image b, block blk, limb l, slots [c 1024, (c + 1) 1024), output coefficients [m0, m0 + MR):
// A[k] = sum_j X_j[k] Op_j[k] for this thread's 4 slots, then sum_k A[k] x_k^-m per m, summed
// over the workgroup into this chunk's share.  The last item of (b, blk, l) adds the shares of
// every chunk and writes c[m] + Delta ((d + sh') mod t) for all m < n_o'.
__device__ __forceinline__ void fz_fc_item(const FusedLayer &jb, uint32_t it, uint32_t *lds, const uint32_t *__restrict__ xinv,
                           const LimbConsts &lc, uint32_t *ctr, uint32_t *err) {
    const uint32_t tid = threadIdx.x;
    const uint32_t N = 1u << jb.logN, L = jb.L, Juse = jb.Juse, Jtot = jb.Jtot, n_o_p = jb.n_o_p;
    const uint32_t chunks = N / FZ_CHUNK;
    const uint32_t MR = n_o_p < (uint32_t)FZ_MR ? n_o_p : (uint32_t)FZ_MR;
    const uint32_t mgroups = n_o_p / MR;
    const uint32_t mg = it % mgroups;
    it /= mgroups;
    const uint32_t cidx = it % chunks;
    it /= chunks;
    const uint32_t l = it % L;
    it /= L;
    const uint32_t blk = it % jb.rows;
    const uint32_t b = it / jb.rows;
    const LimbConst c = lc.l[l];
    const uint32_t k0 = cidx * FZ_CHUNK + 4u * tid;
    const uint32_t *xb = jb.x + ((size_t)b * Jtot * L + l) * N + k0;
    const uint32_t *ob = jb.op + ((size_t)blk * L + l) * Jtot * N + k0;
    uint4 ov[2];
    ov[0] = *reinterpret_cast<const uint4 *>(ob);
    if (Juse > 1) ov[1] = *reinterpret_cast<const uint4 *>(ob + N);
    const uint4 xi4 = *reinterpret_cast<const uint4 *>(xinv + (size_t)l * N + k0);
    const uint32_t sub = (cidx * FZ_CHUNK) >> (jb.logN - 2);
    fz_wait(ctr + ((b * L + l) * 4u + sub) * jb.ctr_stride, jb.ntt_c0 + jb.ntt_sh, err);
    uint64_t a[4];
    {
        const uint4 xv = *reinterpret_cast<const uint4 *>(xb);
        a[0] = (uint64_t)xv.x * ov[0].x;
        a[1] = (uint64_t)xv.y * ov[0].y;
        a[2] = (uint64_t)xv.z * ov[0].z;
        a[3] = (uint64_t)xv.w * ov[0].w;
    }
    if (Juse > 1) {
        const uint4 xv = *reinterpret_cast<const uint4 *>(xb + (size_t)L * N);
        a[0] += (uint64_t)xv.x * ov[1].x;
        a[1] += (uint64_t)xv.y * ov[1].y;
        a[2] += (uint64_t)xv.z * ov[1].z;
        a[3] += (uint64_t)xv.w * ov[1].w;
    }
    const uint32_t xi[4] = {xi4.x, xi4.y, xi4.z, xi4.w};
    uint32_t cur[4];
    const uint32_t m0 = mg * MR;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        cur[i] = reduce64(a[i], c);
        if (m0) {
            // x^-m0 by squaring (m0 is a multiple of MR)
            uint32_t p = xi[i], e = m0, acc = 1;
            while (e) {
                if (e & 1u) acc = mulmod(acc, p, c);
                p = mulmod(p, p, c);
                e >>= 1;
            }
            cur[i] = mulmod(cur[i], acc, c);
        }
    }
    // one coefficient at a time: this thread's 4 terms, summed over the wave by shuffles; lane 0
    // of each wave keeps the wave's sum in LDS
    const uint32_t wave = tid >> 6;
    for (uint32_t m = 0; m < MR; ++m) {
        uint32_t p = addmod(addmod(cur[0], cur[1], c.q), addmod(cur[2], cur[3], c.q), c.q);
#pragma unroll
        for (int i = 0; i < 4; ++i) cur[i] = mulmod(cur[i], xi[i], c);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) p = addmod(p, (uint32_t)__shfl_xor((int)p, off), c.q);
        if ((tid & 63u) == 0) lds[wave * FZ_MR + m] = p;
    }
    __syncthreads();
    const size_t part = (((size_t)b * jb.rows + blk) * L + l) * chunks * n_o_p;   // shares of (b, blk, l)
    if (tid < MR) {
        uint32_t sm = 0;
        for (uint32_t w = 0; w < FZ_THREADS / 64; ++w) sm = addmod(sm, lds[w * FZ_MR + tid], c.q);
        st_dev(jb.h + part + (size_t)cidx * n_o_p + m0 + tid, sm);
    }
    // the last item of (b, l) over every block returns the NTT counters of (b, l) to zero; the
    // last of this (b, blk, l)'s items finishes the block and returns its own counter to zero
    uint32_t *bl_done = ctr + (jb.n_tiles * L * 4u + b * L + l) * jb.ctr_stride;
    uint32_t *blk_done = ctr + (jb.n_tiles * L * 5u + (b * jb.rows + blk) * L + l) * jb.ctr_stride;
    bool last_bl, last_blk;
    fz_signal_last2(bl_done, jb.rows * chunks * mgroups, blk_done, chunks * mgroups, &last_bl, &last_blk);
    if (last_bl) {
        if (tid < 4) st_dev(ctr + ((b * L + l) * 4u + tid) * jb.ctr_stride, 0u);
        if (tid == 0) st_dev(bl_done, 0u);
    }
    if (!last_blk) return;
    if (tid == 0) st_dev(blk_done, 0u);
    const uint32_t *shp = jb.sh_next ? jb.sh_next + (size_t)(b * jb.rows + blk) * n_o_p : nullptr;
    const int32_t *biasp = jb.bias + (size_t)blk * n_o_p;
    uint32_t *outp = jb.out + ((size_t)(b * jb.rows + blk) * L + l) * n_o_p;
    for (uint32_t m = tid; m < n_o_p; m += FZ_THREADS) {
        // the chunk shares (N / 1024 <= 16 of them), all loads issued before the sum
        uint32_t pv[16];
#pragma unroll
        for (uint32_t ci = 0; ci < 16; ++ci) pv[ci] = ci < chunks ? ld_dev(jb.h + part + (size_t)ci * n_o_p + m) : 0u;
        uint32_t v = 0;
#pragma unroll
        for (uint32_t ci = 0; ci < 16; ++ci) v = addmod(v, pv[ci], c.q);
        const int64_t t = (int64_t)c.t_mod;
        int64_t mm = (int64_t)biasp[m] + (shp ? (int64_t)shp[m] : 0);
        mm %= t;
        if (mm < 0) mm += t;
        outp[m] = csub(v + mul_delta_msg((uint32_t)mm, c), c.q);
    }
}

// ------------------------------------------------------------------ row form (1024-thread items)
// A second item layout for conv layers: whole-row NTT items, then one item per output row
// (b, g, n', l) that forms the row's MAC over all N slots, folds the residue blocks into LDS,
// inverts them there and writes its span of residue classes plus Delta sh' (the steps of the
// fused MAC + tail kernel).  The block sums never leave the workgroup; the only hand-off is the
// NTT output.  Before its wait a row item loads up to FZ_RPF of its operand words (16 bytes
// each) per thread, its sh' words and the tail's twiddles.
constexpr int FZ_RT = 1024;
constexpr int FZ_RPF = 8;
constexpr int FZ_RPF_SH = 8;

template <int LOGN>
__device__ __forceinline__ void fz_row_ntt_item(const FusedLayer &jb, uint32_t it, uint32_t *lds,
                                                const uint32_t *__restrict__ tw, const uint32_t *__restrict__ twsh,
                                                const LimbConsts &lc, uint32_t *ctr) {
    constexpr int LOGR = LOGN - 10;
    constexpr int T = 1 << (LOGN - LOGR);
    static_assert(T == FZ_RT, "one row per workgroup");
    const uint32_t tid = threadIdx.x;
    const uint32_t L = jb.L;
    const uint32_t l = it % L;
    uint32_t r = it / L;
    const uint32_t R = jb.ntt_c0 + jb.ntt_sh;
    const uint32_t jj = r % R;
    const uint32_t b = r / R;
    const uint32_t N = 1u << LOGN;
    const uint32_t *in;
    uint32_t jrow;
    if (jj < jb.ntt_c0) {
        jrow = jj;
        in = jb.c0 + ((size_t)(b * jb.K_in + jj) * L + l) * N;
    } else {
        jrow = jb.K_in + (jj - jb.ntt_c0);
        in = jb.sh + (size_t)(b * jb.K_in + (jj - jb.ntt_c0)) * N;
    }
    uint32_t *out = jb.x + ((size_t)(b * jb.Jtot + jrow) * L + l) * N;
    const uint32_t q = lc.l[l].q, q2 = lc.l[l].q2;
    const uint32_t *W = tw + (size_t)l * N;
    const uint32_t *Wsh = twsh + (size_t)l * N;
    PassTw<LOGN, LOGR, FZ_RT> ptw;
    fwd_tw_load<LOGN, LOGR, FZ_RT, 0>(ptw, tid, W, Wsh);
    uint32_t v[1 << LOGR];
    fwd_pass<LOGN, LOGR, FZ_RT, 0>(v, ptw, lds, tid, in, W, Wsh, q, q2);
#pragma unroll
    for (int i = 0; i < (1 << LOGR); ++i) {
        const uint32_t idx = tid + i * T;
        uint32_t y = lds[lpad(idx)];
        y = csub(y, q2);
        st_dev(out + idx, csub(y, q));
    }
    fz_signal(ctr + (b * L + l) * jb.ctr_stride, 1u);
}

template <int LOGM, int JU>
__device__ __forceinline__ void fz_row_mac_tail_item(const FusedLayer &jb, uint32_t w, uint32_t *lds,
                                                     const uint32_t *__restrict__ twi,
                                                     const uint32_t *__restrict__ twish, const LimbConsts &lc,
                                                     uint32_t *ctr, uint32_t *err) {
    constexpr int LOGR = LOGM - 10 > 2 ? LOGM - 10 : 2;
    constexpr int M = 1 << LOGM;
    constexpr int T = 1 << (LOGM - LOGR);
    const uint32_t tid = threadIdx.x;
    const uint32_t L = jb.L, g_o = jb.g_o, K_out = jb.K_out, c_o = jb.rows, Juse = jb.Juse, Jtot = jb.Jtot;
    const uint32_t l = w % L;
    w /= L;
    const uint32_t np = w % g_o;
    w /= g_o;
    const uint32_t g = w % K_out;
    const uint32_t b = w / K_out;
    const uint32_t n = g * g_o + np;
    const bool exists = n < c_o;
    const LimbConst c = lc.l[l];
    const uint32_t logN = jb.logN, s_log = jb.s_log;
    const uint32_t N = 1u << logN;
    const uint32_t cw_log = s_log - (31u - __clz(g_o));
    const uint32_t cw_mask = (1u << cw_log) - 1u;
    const uint32_t c_lo = np << cw_log;
    const uint32_t total = (uint32_t)M << cw_log;
    uint32_t *o = jb.out + ((size_t)(b * K_out + g) * L + l) * N;
    const uint32_t *sh = jb.sh_next ? jb.sh_next + (size_t)(b * K_out + g) * N : nullptr;
    uint32_t shv[FZ_RPF_SH];
#pragma unroll
    for (int i = 0; i < FZ_RPF_SH; ++i) {
        const uint32_t e = tid + i * FZ_RT;
        shv[i] = (sh && e < total) ? sh[((e >> cw_log) << s_log) + c_lo + (e & cw_mask)] : 0u;
    }
    // operand words of this thread, (slot group i, row j) in order; the first FZ_RPF before the wait
    const uint32_t groups = N / (4u * FZ_RT);
    const uint32_t *op = jb.op + (size_t)(exists ? n : 0) * L * Jtot * N + (size_t)l * Jtot * N + 4u * tid;
    const uint32_t *x = jb.x + ((size_t)b * Jtot * L + l) * N + 4u * tid;
    uint4 pf[FZ_RPF];
    if (exists) {
#pragma unroll
        for (int f = 0; f < FZ_RPF; ++f) {
            const uint32_t i = f / JU, j = f % JU;
            if (i < groups && j < Juse) pf[f] = *reinterpret_cast<const uint4 *>(op + (size_t)j * N + i * 4u * FZ_RT);
        }
    }
    const uint32_t *W = twi + (size_t)l * N;
    const uint32_t *Wsh = twish + (size_t)l * N;
    const bool act = tid < (uint32_t)T;
    PassTw<LOGM, LOGR, TW_IN_PASS> ptw;
    inv_tw_load<LOGM, LOGR, TW_IN_PASS, 0>(ptw, act ? tid : 0u, W, Wsh);
    fz_wait(ctr + (b * L + l) * jb.ctr_stride, jb.ntt_c0 + jb.ntt_sh, err);
    if (exists) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if ((uint32_t)i >= groups) break;
            const uint32_t k4 = 4u * tid + i * 4u * FZ_RT;
            uint64_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
            for (int j = 0; j < JU; ++j) {
                if ((uint32_t)j >= Juse) break;
                const uint4 xv = *reinterpret_cast<const uint4 *>(x + (size_t)j * L * N + i * 4u * FZ_RT);
                const int f = i * JU + j;
                // a prefetched word, else a load now
                const uint4 ov = f < FZ_RPF ? pf[f < FZ_RPF ? f : 0]
                                            : *reinterpret_cast<const uint4 *>(op + (size_t)j * N + i * 4u * FZ_RT);
                a0 += (uint64_t)xv.x * ov.x;
                a1 += (uint64_t)xv.y * ov.y;
                a2 += (uint64_t)xv.z * ov.z;
                a3 += (uint64_t)xv.w * ov.w;
                if ((j & 7) == 7) {
                    a0 = reduce64(a0, c);
                    a1 = reduce64(a1, c);
                    a2 = reduce64(a2, c);
                    a3 = reduce64(a3, c);
                }
            }
            const uint32_t r0 = reduce64(a0, c), r1 = reduce64(a1, c), r2 = reduce64(a2, c), r3 = reduce64(a3, c);
            if (s_log == 1) {
                lds[lpad(k4 >> 1)] = addmod(r0, r1, c.q);
                lds[lpad((k4 >> 1) + 1)] = addmod(r2, r3, c.q);
            } else {
                uint32_t v = r0 + r1 + r2 + r3;   // [0, 4q)
                v = csub(csub(v, c.q2), c.q);
                const uint32_t lanes = 1u << (s_log - 2);
                for (uint32_t m = 1; m < lanes; m <<= 1) v = addmod(v, (uint32_t)__shfl_xor((int)v, (int)m), c.q);
                if ((tid & (lanes - 1)) == 0) lds[lpad(k4 >> s_log)] = v;
            }
        }
        __syncthreads();
        uint32_t v[1 << LOGR];
        inv_pass<LOGM, LOGR, TW_IN_PASS, 0>(v, ptw, lds, act ? tid : 0u, W, Wsh, c.q, c.q2, act);
        __syncthreads();
        if (act) {
#pragma unroll
            for (int i = 0; i < (1 << LOGR); ++i) lds[lpad(inv_final_idx<LOGM, LOGR>(tid, i))] = csub(v[i], c.q);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < FZ_RPF_SH; ++i) {
        const uint32_t e = tid + i * FZ_RT;
        if (e < total) {
            const uint32_t m = e >> cw_log, off = e & cw_mask;
            uint32_t val = (exists && off == 0) ? lds[lpad(m)] : 0u;
            if (sh) val = csub(val + mul_delta_msg(shv[i], c), c.q);
            o[(m << s_log) + c_lo + off] = val;
        }
    }
    for (uint32_t e = tid + FZ_RPF_SH * FZ_RT; e < total; e += FZ_RT) {
        const uint32_t m = e >> cw_log, off = e & cw_mask;
        const uint32_t k = (m << s_log) + c_lo + off;
        uint32_t val = (exists && off == 0) ? lds[lpad(m)] : 0u;
        if (sh) val = csub(val + mul_delta_msg(sh[k], c), c.q);
        o[k] = val;
    }
    // the last row item of (b, l) returns the counters of (b, l) to zero
    uint32_t *done = ctr + (jb.B * L + b * L + l) * jb.ctr_stride;
    if (fz_signal_last(done, K_out * g_o) && threadIdx.x == 0) {
        st_dev(ctr + (b * L + l) * jb.ctr_stride, 0u);
        st_dev(done, 0u);
    }
}

template <int LOGM>
__device__ __forceinline__ void fz_row_ju_switch(const FusedLayer &jb, uint32_t w, uint32_t *lds, const uint32_t *twi,
                                                 const uint32_t *twish, const LimbConsts &lc, uint32_t *ctr,
                                                 uint32_t *err) {
    if (jb.Juse <= 1) fz_row_mac_tail_item<LOGM, 1>(jb, w, lds, twi, twish, lc, ctr, err);
    else if (jb.Juse <= 2) fz_row_mac_tail_item<LOGM, 2>(jb, w, lds, twi, twish, lc, ctr, err);
    else if (jb.Juse <= 4) fz_row_mac_tail_item<LOGM, 4>(jb, w, lds, twi, twish, lc, ctr, err);
    else fz_row_mac_tail_item<LOGM, 8>(jb, w, lds, twi, twish, lc, ctr, err);
}

template <int LOGN>
__global__ void __launch_bounds__(FZ_RT, 1)
k_fused_rows(FusedLayer jb, const uint32_t *__restrict__ tw, const uint32_t *__restrict__ twsh,
             const uint32_t *__restrict__ twi, const uint32_t *__restrict__ twish, LimbConsts lc,
             uint32_t *__restrict__ sync) {
    __shared__ uint32_t lds[(1 << LOGN) + (1 << LOGN >> 5)];
    uint32_t *err = sync + FZ_SB_ERR;
    uint32_t *ctr = sync + FZ_SB_HDR;
    const uint32_t t = blockIdx.x;
    if (t < jb.n_ntt) {
        fz_row_ntt_item<LOGN>(jb, t, lds, tw, twsh, lc, ctr);
        return;
    }
    const uint32_t w = t - jb.n_ntt;
    switch (jb.logN - jb.s_log) {
        case 4: fz_row_ju_switch<4>(jb, w, lds, twi, twish, lc, ctr, err); break;
        case 5: fz_row_ju_switch<5>(jb, w, lds, twi, twish, lc, ctr, err); break;
        case 6: fz_row_ju_switch<6>(jb, w, lds, twi, twish, lc, ctr, err); break;
        case 7: fz_row_ju_switch<7>(jb, w, lds, twi, twish, lc, ctr, err); break;
        case 8: fz_row_ju_switch<8>(jb, w, lds, twi, twish, lc, ctr, err); break;
        case 9: fz_row_ju_switch<9>(jb, w, lds, twi, twish, lc, ctr, err); break;
        case 10: fz_row_ju_switch<10>(jb, w, lds, twi, twish, lc, ctr, err); break;
        case 11: fz_row_ju_switch<11>(jb, w, lds, twi, twish, lc, ctr, err); break;
        case 12: fz_row_ju_switch<12>(jb, w, lds, twi, twish, lc, ctr, err); break;
        default: break;   // excluded by the host
    }
}

// ------------------------------------------------------------------ the launch
template <int LOGN>
// two workgroups per CU (at most 256 VGPRs): the items of a batch-one plain-20 layer at N = 8192
// are all resident
__global__ void __launch_bounds__(FZ_THREADS, 2)
k_fused_layer(FusedLayer jb, const uint32_t *__restrict__ tw, const uint32_t *__restrict__ twsh,
              const uint32_t *__restrict__ twi, const uint32_t *__restrict__ twish, const uint32_t *__restrict__ xinv,
              LimbConsts lc, uint32_t *__restrict__ sync) {
    __shared__ uint32_t lds[FZ_LDS];
    uint32_t *err = sync + FZ_SB_ERR;
    uint32_t *ctr = sync + FZ_SB_HDR;
    const uint32_t t = blockIdx.x;
    if (t < jb.n_ntt) {
        fz_ntt_item<LOGN>(jb, t, lds, tw, twsh, lc, ctr);
    } else if (t < jb.n_ntt + jb.n_mac) {
        if (jb.kind == FZ_KIND_CONV && jb.ng == 0)
            fz_mac_wide_switch(jb, t - jb.n_ntt, lc, ctr, err);
        else if (jb.kind == FZ_KIND_CONV)
            fz_mac_conv_item(jb, t - jb.n_ntt, lc, ctr, err);
        else
            fz_fc_item(jb, t - jb.n_ntt, lds, xinv, lc, ctr, err);
    } else if (t < jb.n_ntt + jb.n_mac + jb.n_inv) {
        fz_tail_switch(jb, t - jb.n_ntt - jb.n_mac, lds, twi, twish, lc, ctr, err);
    }
}

// ------------------------------------------------------------------ the grouped launch
// The items of every job, phase by phase: all NTT items, then all MAC items, then all tail
// items, so that an item waits only for items of earlier phases, which have lower workgroup ids
// (the argument at the top of the file).  Phase p takes 8 per_p workgroups from a multiple of 8;
// within a phase the items go to the XCDs in chunks of 2^chunk_log consecutive items, round
// robin, so that neighbouring items of one job (the sub-blocks of one row, the slot ranges of one
// tile) share an XCD and its L2 while the jobs, which differ widely in cost, spread over every
// XCD (the chunk is a tuning knob of the group); workgroups past the phase's item count return
// at once.  The job of an item is found by a binary search over the jobs' first items of that
// phase.
// Four workgroups per CU (at most 128 VGPRs; the LDS of four fits a CU): the MAC and inverse items
// of batched calls need the occupancy, so the NTT items keep fewer twiddles in registers than in
// the one-layer launch, the tiled MAC item is the DMA-staged one (no staging registers), and a
// per-image MAC takes the channel-group item (the all-channel item holds too many operand words
// in registers).  A few bytes per lane spill at this cap; three workgroups per CU without the
// spill ran the three batched stacks 8 % slower.
// words: the three DMA stage buffers of the largest tile geometry (3 x 96 rows x 32 words), more
// than an 8192-point row
constexpr int FG_LDS = 9216;
constexpr int FG_TWB = 1024;
// Workgroups per XCD of a phase of `count` items (whole chunks of 2^chunk_log).
__host__ __device__ constexpr uint32_t fg_per_xcd(uint32_t count, uint32_t chunk_log) {
    return ((count + (8u << chunk_log) - 1u) >> (chunk_log + 3u)) << chunk_log;
}
static_assert(FG_LDS >= FZ_LDS && FG_LDS >= 8192 + 256, "the group's LDS holds every item's");

__global__ void __launch_bounds__(FZ_THREADS, 4)
k_fused_group(const FusedJob *__restrict__ jobs, uint32_t n_jobs, uint32_t c0, uint32_t c1, uint32_t c2,
              uint32_t chunk_log, uint32_t *__restrict__ sync) {
    __shared__ __align__(16) uint32_t lds[FG_LDS];   // 16-byte aligned: the tiled MAC reads 8-byte pairs
    const uint32_t p0 = fg_per_xcd(c0, chunk_log), p1 = fg_per_xcd(c1, chunk_log);
    uint32_t t = blockIdx.x, phase, count;
    if (t < 8u * p0) {
        phase = 0;
        count = c0;
    } else if ((t -= 8u * p0) < 8u * p1) {
        phase = 1;
        count = c1;
    } else {
        t -= 8u * p1;
        phase = 2;
        count = c2;
    }
    // XCD x's k-th workgroup of the phase takes item k mod 2^chunk_log of chunk (k >> chunk_log) 8 + x
    const uint32_t k = t >> 3;
    const uint32_t item = ((((k >> chunk_log) << 3) + (t & 7u)) << chunk_log) + (k & ((1u << chunk_log) - 1u));
    if (item >= count) return;
    uint32_t lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (jobs[mid].first[phase] <= item) lo = mid;
        else hi = mid - 1;
    }
    const FusedJob &J = jobs[lo];
    const FusedLayer &jb = J.jb;
    const LimbConsts &lc = *J.lc;
    const uint32_t it = item - J.first[phase];
    uint32_t *err = sync + FZ_SB_ERR;
    uint32_t *ctr = sync + FZ_SB_HDR + J.ctr_off;
    if (phase == 0) {
        switch (jb.logN) {
            case 12: fz_ntt_item<12, FG_TWB, fz_group_ntt_k(12)>(jb, it, lds, J.tw, J.twsh, lc, ctr); break;
            case 13: fz_ntt_item<13, FG_TWB, fz_group_ntt_k(13)>(jb, it, lds, J.tw, J.twsh, lc, ctr); break;
            default: fz_ntt_item<14, FG_TWB, fz_group_ntt_k(14)>(jb, it, lds, J.tw, J.twsh, lc, ctr); break;
        }
    } else if (phase == 1) {
        if (jb.kind != FZ_KIND_CONV)
            fz_fc_item(jb, it, lds, J.xinv, lc, ctr, err);
        else if (jb.mac_tiled)
            fz_mac_tile_switch(jb, it, lds, lc, ctr, err);
        else
            fz_mac_conv_item(jb, it, lc, ctr, err);   // grouped: the plan gave ng >= 1
    } else {
        fz_tail_switch_group(jb, it, lds, J.twi, J.twish, lc, ctr, err);
    }
}

}  // namespace

bool fused_layer_ok(const FusedLayer &jb) {
    if (jb.logN < 12 || jb.logN > 14 || jb.B == 0 || jb.L == 0) return false;
    if (jb.Juse == 0 || jb.Jtot < jb.Juse) return false;
    if (jb.rows_form) {
        // conv only; a residue block within one wave (s <= 256); the tail fits the LDS row
        const uint32_t logm = jb.logN - jb.s_log;
        return jb.kind == FZ_KIND_CONV && jb.s_log >= 1 && jb.s_log <= 8 && logm >= 4 && logm <= 12 && jb.g_o &&
               jb.g_o <= (1u << jb.s_log) && !(jb.g_o & (jb.g_o - 1)) && jb.Juse <= 8;
    }
    if (jb.kind == FZ_KIND_CONV) {
        const uint32_t logm = jb.logN - jb.s_log;
        if (jb.s_log < 1 || jb.s_log > 8 || logm < 4 || logm > 12) return false;
        if (jb.g_o == 0 || jb.g_o > (1u << jb.s_log) || (jb.g_o & (jb.g_o - 1))) return false;
    } else if (jb.kind == FZ_KIND_FC) {
        if (jb.n_o_p == 0 || (jb.n_o_p & (jb.n_o_p - 1)) || jb.n_o_p > 1024 || jb.Juse > 2) return false;
    } else {
        return false;
    }
    return true;
}

uint32_t fused_layer_plan(FusedLayer &jb) {
    const uint32_t N = 1u << jb.logN;
    const uint32_t chunks = N / FZ_CHUNK;
    jb.tile_log = 0;
    jb.n_tiles = jb.B;
    if (jb.rows_form) {
        // whole-row NTT items, then one item per output row (b, g, n', l)
        jb.n_ntt = jb.B * (jb.ntt_c0 + jb.ntt_sh) * jb.L;
        jb.ng = 0;
        jb.tail_rw = 0;
        jb.mac_per_bl = jb.K_out * jb.g_o;
        jb.n_mac = jb.B * jb.K_out * jb.g_o * jb.L;
        jb.n_inv = 0;
        jb.n_ctr = 2u * jb.B * jb.L;          // NTT rows done, row items done, per (b, l)
        jb.ctr_stride = (FZ_SB_HDR + jb.n_ctr * 32u <= FZ_SYNC_WORDS) ? 32u : 1u;
        return jb.n_ctr * jb.ctr_stride;
    }
    jb.n_ntt = jb.B * (jb.ntt_c0 + jb.ntt_sh) * jb.L * (jb.grouped ? (1u << fz_group_ntt_k((int)jb.logN)) : 4u);
    if (jb.kind == FZ_KIND_CONV) {
        if (jb.mac_tiled) {
            // LDS-staged tiles of 4 TBq images (one counter tile each) x 4 TNq channels
            jb.ng = 0;
            jb.tile_log = 31u - __builtin_clz(4u * jb.gm.TBq);
            jb.n_tiles = jb.gm.tiles_b;
            jb.mac_per_bl = jb.gm.ranges * jb.gm.tiles_n;
            jb.n_mac = jb.L * jb.gm.ranges * jb.gm.tiles_b * jb.gm.tiles_n;
        } else if (!jb.grouped && (jb.Juse == 1 || jb.Juse == 2 || jb.Juse == 4 || jb.Juse == 8) && jb.s_log <= 7) {
            // every channel of a 128-slot chunk per item (ng = 0 marks this form)
            jb.ng = 0;
            jb.mac_per_bl = N / FZ_WCHUNK;
            jb.n_mac = jb.B * jb.L * jb.mac_per_bl;
        } else {
            // channels per MAC item: about a thousand items, up to 4 channels each; in a grouped
            // launch (many calls' items at once) 8 channels, fewer and longer items
            const uint64_t base = (uint64_t)jb.B * jb.L * chunks * jb.rows;
            uint32_t ng = 1;
            if (jb.grouped)
                ng = jb.rows < 8 ? jb.rows : 8;
            else
                while (ng < 4 && base / (2 * ng) >= 1024) ng <<= 1;
            jb.ng = ng;
            jb.mac_per_bl = chunks * ((jb.rows + ng - 1) / ng);
            jb.n_mac = jb.B * jb.L * jb.mac_per_bl;
        }
        const uint32_t logm = jb.logN - jb.s_log;
        const uint32_t logr = jb.grouped ? (uint32_t)fz_group_tail_logr((int)logm) : (logm > 10 ? logm - 8 : 2);
        const uint32_t T = 1u << (logm - logr);
        uint32_t rw = FZ_THREADS / T;
        if (rw > jb.g_o) rw = jb.g_o;
        jb.tail_rw = rw;
        jb.n_inv = jb.B * jb.K_out * jb.L * (jb.g_o / rw);
        jb.n_ctr = jb.n_tiles * jb.L * 6u;       // per tile and limb: NTT sub-blocks (4), MAC done, tails done
    } else {
        const uint32_t mr = jb.n_o_p < (uint32_t)FZ_MR ? jb.n_o_p : (uint32_t)FZ_MR;
        jb.ng = 1;
        jb.tail_rw = 0;
        jb.n_mac = jb.B * jb.rows * jb.L * chunks * (jb.n_o_p / mr);
        jb.n_inv = 0;
        jb.n_ctr = jb.B * jb.L * 5u + jb.B * jb.rows * jb.L;  // NTT sub-blocks, items of (b, l), of (b, blk, l)
    }
    // one counter per 128-byte line when they fit
    jb.ctr_stride = (FZ_SB_HDR + jb.n_ctr * 32u <= FZ_SYNC_WORDS) ? 32u : 1u;
    return jb.n_ctr * jb.ctr_stride;
}

hipError_t launch_fused_layer(const FusedLayer &jb, const uint32_t *tw, const uint32_t *twsh, const uint32_t *twi,
                              const uint32_t *twish, const uint32_t *xinv, const LimbConsts &lc, uint32_t *sync,
                              hipStream_t st, const LaunchEv *ev) {
    const uint32_t grid = jb.n_ntt + jb.n_mac + jb.n_inv;
    if (grid == 0) return hipSuccess;
    if (FZ_SB_HDR + jb.n_ctr * jb.ctr_stride > FZ_SYNC_WORDS) return hipErrorInvalidValue;
    if (jb.rows_form) {
        switch (jb.logN) {
            case 12:
                HE_LAUNCH(ev, k_fused_rows<12>, dim3(grid), dim3(FZ_RT), 0, st, jb, tw, twsh, twi, twish, lc, sync);
                break;
            case 13:
                HE_LAUNCH(ev, k_fused_rows<13>, dim3(grid), dim3(FZ_RT), 0, st, jb, tw, twsh, twi, twish, lc, sync);
                break;
            case 14:
                HE_LAUNCH(ev, k_fused_rows<14>, dim3(grid), dim3(FZ_RT), 0, st, jb, tw, twsh, twi, twish, lc, sync);
                break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (jb.logN) {
        case 12:
            HE_LAUNCH(ev, k_fused_layer<12>, dim3(grid), dim3(FZ_THREADS), 0, st, jb, tw, twsh, twi, twish, xinv, lc,
                      sync);
            break;
        case 13:
            HE_LAUNCH(ev, k_fused_layer<13>, dim3(grid), dim3(FZ_THREADS), 0, st, jb, tw, twsh, twi, twish, xinv, lc,
                      sync);
            break;
        case 14:
            HE_LAUNCH(ev, k_fused_layer<14>, dim3(grid), dim3(FZ_THREADS), 0, st, jb, tw, twsh, twi, twish, xinv, lc,
                      sync);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

uint32_t fused_group_lds_bytes() { return (uint32_t)FG_LDS * 4u; }

hipError_t launch_fused_group(const FusedJob *jobs, uint32_t n_jobs, const uint32_t count[3], uint32_t chunk_log,
                              uint32_t *sync, hipStream_t st, const LaunchEv *ev) {
    if (n_jobs == 0) return hipSuccess;
    if (chunk_log > 10) return hipErrorInvalidValue;
    const uint64_t grid = 8ull * ((uint64_t)fg_per_xcd(count[0], chunk_log) + fg_per_xcd(count[1], chunk_log) +
                                  fg_per_xcd(count[2], chunk_log));
    if (grid == 0) return hipSuccess;
    if (grid > 0x7fffffffull) return hipErrorInvalidValue;
    HE_LAUNCH(ev, k_fused_group, dim3((uint32_t)grid), dim3(FZ_THREADS), 0, st, jobs, n_jobs, count[0], count[1],
              count[2], chunk_log, sync);
    return hipGetLastError();
}
