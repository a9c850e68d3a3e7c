// Batched residue-class MAC on the matrix cores (a2 of Alg. 1 over a batch of images).
//
// For a layer at batch B the block sums the residue-class tail reads are, for every limb l and
// block m (the s consecutive NTT slots [m s, m s + s)),
//     H(b, n, l, m) = sum over input rows j < Juse and slots k of block m of
//                     X[b][j][l][k] * Op[n][l][j][k]  mod q_l,
// a product of a B x K matrix (images by (row, slot) pairs, K = Juse s) with a K x c_o one
// (operands by output channel): a dense contraction, which this kernel runs on the integer matrix
// cores (v_mfma_i32_16x16x64_i8).  The sums are stored in groups of 8 channels,
// h[l][b][n / 8][m][n % 8] (the tail reads that order with its by_block option): a block's tile
// then goes out as 32-byte pieces, where the order of the other MAC forms, h[b][n][l][m], would
// scatter it into 4-byte writes that no L2 holds until the neighbouring blocks fill them.
//
// Exactness.  Every residue x < q < 2^30 is written in signed base-256 digits,
//     x = d0 + d1 2^8 + d2 2^16 + d3 2^24,  d0, d1, d2 in [-128, 128), d3 in [0, 64],
// read off the bytes of (x + 0x00808080) ^ 0x00808080.  The 16 digit-plane products are
// accumulated exactly in 32-bit integers, one accumulator per shift a + b (7 of them):
// |C_s| <= K 3 2^14 < 2^31 for K <= 32768.  Each output word is then
//     (C0 + C1 2^8 + C2 2^16 + C3 2^24) + (C4 + C5 2^8 + C6 2^16) 2^32   mod q,
// two signed 64-bit sums below 2^56 in magnitude, each made positive by a multiple of q and
// reduced.  The words are the same as every other MAC form's.
//
// Tiling.  A workgroup of 256 threads (4 waves) owns 64 images x TN channels (TN = 64, 32 or 16)
// of one limb and 2^mb_log consecutive blocks (one, at the shapes measured).  Per chunk of 64 K
// elements, each thread loads 16 words of one image row and the first 4 TN threads 16 of one
// channel row (4 x 16 bytes each, a row's slots being contiguous for s >= 4), converts them to
// digit planes and stores those to LDS (rows padded to 80 bytes, so that the 16-byte operand
// reads of 8 consecutive rows fall in distinct banks).  At TN = 64 each wave then computes a
// 32 x 32 corner of the tile: 2 x 2 MFMA tiles x 16 digit pairs = 64 MFMAs per chunk.  The next
// chunk's global loads are issued before the products, so their latency overlaps them.

#include "he_kernels.h"

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int MM_THREADS = 256;
constexpr int MM_T = 64;                     // images per workgroup tile
constexpr int MM_KC = 64;                    // K elements per chunk
constexpr int MM_ROWB = 80;                  // bytes per staged row (64 digit bytes + 16 pad)
constexpr int MM_XPL = MM_T * MM_ROWB;       // bytes per digit plane of the image rows
constexpr uint32_t MM_KMAX = 32768;          // longest exact contraction

// Channel tile TN = 64, 32 or 16 (layers of fewer channels take the narrower tiles, which hold
// fewer accumulators and so run more workgroups per CU).  The 4 waves split the 64 x TN tile
// WR (images) by WC (channels); each wave owns RT x CT MFMA tiles of 16 x 16.
template <int TN>
struct MMShape {
    static constexpr int WC = TN >= 32 ? 2 : 1;
    static constexpr int WR = 4 / WC;
    static constexpr int CT = TN / (16 * WC);
    static constexpr int RT = MM_T / (16 * WR);
    static constexpr int OPL = TN * MM_ROWB;                 // bytes per digit plane of the channel rows
    static constexpr int LDS = 4 * MM_XPL + 4 * OPL;
    static constexpr int WG_PER_CU = TN == 64 ? 2 : (TN == 32 ? 3 : 4);
};

// signed base-256 digits of x < 2^30, one per byte
__device__ __forceinline__ uint32_t sdigits(uint32_t x) { return (x + 0x00808080u) ^ 0x00808080u; }

// byte transpose: p[a] holds digit a of w0, w1, w2, w3 (in that byte order)
__device__ __forceinline__ void planes4(uint4 w, uint32_t (&p)[4]) {
    const uint32_t w0 = sdigits(w.x), w1 = sdigits(w.y), w2 = sdigits(w.z), w3 = sdigits(w.w);
    const uint32_t t0 = (w0 & 0x00FF00FFu) | ((w1 & 0x00FF00FFu) << 8);   // w0.0 w1.0 w0.2 w1.2
    const uint32_t t1 = ((w0 >> 8) & 0x00FF00FFu) | (w1 & 0xFF00FF00u);   // w0.1 w1.1 w0.3 w1.3
    const uint32_t t2 = (w2 & 0x00FF00FFu) | ((w3 & 0x00FF00FFu) << 8);
    const uint32_t t3 = ((w2 >> 8) & 0x00FF00FFu) | (w3 & 0xFF00FF00u);
    p[0] = (t0 & 0xFFFFu) | (t2 << 16);
    p[1] = (t1 & 0xFFFFu) | (t3 << 16);
    p[2] = (t0 >> 16) | (t2 & 0xFFFF0000u);
    p[3] = (t1 >> 16) | (t3 & 0xFFFF0000u);
}

// the residue of a signed sum |v| < 2^56: v plus a multiple of q in [2^56, 2^57), reduced
__device__ __forceinline__ uint32_t reduce_signed56(int64_t v, uint64_t off, const LimbConst &c) {
    return reduce64((uint64_t)(v + (int64_t)off), c);
}

template <int TN>
__global__ void __launch_bounds__(MM_THREADS, MMShape<TN>::WG_PER_CU)
k_mac_mfma(const uint32_t *__restrict__ X, const uint32_t *__restrict__ Op, uint32_t *__restrict__ h, uint32_t B,
           uint32_t Jtot, uint32_t Juse, uint32_t c_o, uint32_t L, uint32_t N, uint32_t s_log, uint32_t mb_log,
           uint32_t tiles_b, uint32_t tiles_n, LimbConsts lc) {
    using S = MMShape<TN>;
    constexpr int RT = S::RT, CT = S::CT;
    __shared__ __align__(16) uint8_t lds[S::LDS];
    const uint32_t M = N >> s_log;
    const uint32_t ranges = M >> mb_log;
    uint32_t w;
    if (!xcd_logical(blockIdx.x, L * ranges * tiles_b * tiles_n, w)) return;
    const uint32_t tn = w % tiles_n;
    w /= tiles_n;
    const uint32_t tb = w % tiles_b;
    w /= tiles_b;
    const uint32_t mr = w % ranges;
    const uint32_t l = w / ranges;
    const LimbConst c = lc.l[l];
    const uint32_t b0 = tb * MM_T, n0 = tn * TN;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;

    // staging role: image row tid / 4 and, for the first 4 TN threads, channel row tid / 4; K
    // quarter tid % 4 (16 elements)
    const uint32_t srow = tid >> 2, sq = tid & 3u;
    const bool ostage = srow < (uint32_t)TN;
    const bool xv = b0 + srow < B, ov = ostage && n0 + srow < c_o;
    const uint32_t *xrow = X + ((size_t)(xv ? b0 + srow : 0) * Jtot * L + l) * N;    // + (j L) N + slot
    const uint32_t *orow = Op + ((size_t)(ov ? n0 + srow : 0) * L + l) * Jtot * N;   // + j N + slot
    const uint32_t K = Juse << s_log;
    const uint32_t nch = (K + MM_KC - 1) / MM_KC;
    const uint32_t total = nch << mb_log;
    const uint32_t s_mask = (1u << s_log) - 1u;

    uint4 px[4], po[4];
    auto load = [&](uint32_t qi) {
        const uint32_t m = (mr << mb_log) + qi / nch;
        const uint32_t k0 = (qi % nch) * MM_KC + sq * 16u;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t kk = k0 + 4u * u;   // 4 elements of one row j (s >= 4)
            const uint32_t j = kk >> s_log, slot = (m << s_log) + (kk & s_mask);
            const bool in = kk < K;
            px[u] = (in && xv) ? *reinterpret_cast<const uint4 *>(xrow + (size_t)j * L * N + slot) : make_uint4(0, 0, 0, 0);
            po[u] = (in && ov) ? *reinterpret_cast<const uint4 *>(orow + (size_t)j * N + slot) : make_uint4(0, 0, 0, 0);
        }
    };
    auto stage = [&](const uint4 (&pv)[4], uint8_t *base, int plane_bytes) {
        uint32_t pl[4][4];   // [plane][u]
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            uint32_t p[4];
            planes4(pv[u], p);
#pragma unroll
            for (int a = 0; a < 4; ++a) pl[a][u] = p[a];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
            *reinterpret_cast<uint4 *>(base + a * plane_bytes) = make_uint4(pl[a][0], pl[a][1], pl[a][2], pl[a][3]);
    };

    // product role: the wave's RT x CT tiles; lane row / column li, K group lg
    const uint32_t li = lane & 15u, lg = lane >> 4;
    const uint32_t rb = 16u * RT * (wave % S::WR), cb = 16u * CT * (wave / S::WR);
    v4i acc[RT][CT][7];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < CT; ++j)
#pragma unroll
            for (int s = 0; s < 7; ++s) acc[i][j][s] = v4i{0, 0, 0, 0};
    const uint64_t off = (uint64_t)c.q << (25 + __clz(c.q));   // a multiple of q in [2^56, 2^57)
    uint8_t *const lx = lds, *const lo_ = lds + 4 * MM_XPL;

    load(0);
    for (uint32_t qi = 0; qi < total; ++qi) {
        __syncthreads();   // every wave is done reading the previous chunk's planes
        stage(px, lx + srow * MM_ROWB + sq * 16u, MM_XPL);
        if (ostage) stage(po, lo_ + srow * MM_ROWB + sq * 16u, S::OPL);
        __syncthreads();   // the planes of this chunk are in LDS
        if (qi + 1 < total) load(qi + 1);

        v4i A[RT][4], Bm[CT][4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
#pragma unroll
            for (int r = 0; r < RT; ++r)
                A[r][a] = *reinterpret_cast<const v4i *>(lx + a * MM_XPL + (rb + 16u * r + li) * MM_ROWB + 16u * lg);
#pragma unroll
            for (int cc = 0; cc < CT; ++cc)
                Bm[cc][a] = *reinterpret_cast<const v4i *>(lo_ + a * S::OPL + (cb + 16u * cc + li) * MM_ROWB + 16u * lg);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int bd = 0; bd < 4; ++bd)
#pragma unroll
                for (int r = 0; r < RT; ++r)
#pragma unroll
                    for (int cc = 0; cc < CT; ++cc)
                        acc[r][cc][a + bd] =
                            __builtin_amdgcn_mfma_i32_16x16x64_i8(A[r][a], Bm[cc][bd], acc[r][cc][a + bd], 0, 0, 0);

        if (qi % nch == nch - 1) {
            // block m done: lane holds images rb + 16 r + 4 lg + e, channel cb + 16 cc + li
            const uint32_t m = (mr << mb_log) + qi / nch;
#pragma unroll
            for (int r = 0; r < RT; ++r)
#pragma unroll
                for (int cc = 0; cc < CT; ++cc) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int64_t lo = (int64_t)acc[r][cc][0][e] + (int64_t)acc[r][cc][1][e] * 256 +
                                           (int64_t)acc[r][cc][2][e] * 65536 + (int64_t)acc[r][cc][3][e] * 16777216;
                        const int64_t hi = (int64_t)acc[r][cc][4][e] + (int64_t)acc[r][cc][5][e] * 256 +
                                           (int64_t)acc[r][cc][6][e] * 65536;
                        const uint32_t rl = reduce_signed56(lo, off, c);
                        const uint32_t rh = reduce_signed56(hi, off, c);
                        const uint32_t v = csub(rl + csub(shoup_lazy(rh, c.r32, c.r32_sh, c.q), c.q), c.q);
                        const uint32_t b = b0 + rb + 16u * r + 4u * lg + e, n = n0 + cb + 16u * cc + li;
                        if (b < B && n < c_o) h[(((size_t)(l * B + b) * c_o + (n & ~7u)) * M + m * 8u) + (n & 7u)] = v;
                    }
#pragma unroll
                    for (int s = 0; s < 7; ++s) acc[r][cc][s] = v4i{0, 0, 0, 0};
                }
        }
    }
}

}  // namespace

bool mac_mfma_ok(uint32_t B, uint32_t c_o, uint32_t Juse, uint32_t N, uint32_t s) {
    return B >= 1 && c_o >= 8 && c_o % 8 == 0 && Juse >= 1 && s >= 4 && (s & (s - 1)) == 0 && 16 * s <= N && N >= 256 && (N & (N - 1)) == 0 &&
           (uint64_t)Juse * s <= MM_KMAX;
}

hipError_t launch_mac_mfma(const uint32_t *X, const uint32_t *Op, uint32_t *h, uint32_t B, uint32_t Jtot,
                           uint32_t Juse, uint32_t c_o, uint32_t L, uint32_t N, uint32_t s, const LimbConsts &lc,
                           hipStream_t st, const LaunchEv *ev) {
    if (B == 0) return hipSuccess;
    if (Juse == 0 || Juse > Jtot || !mac_mfma_ok(B, c_o, Juse, N, s)) return hipErrorInvalidValue;
    uint32_t s_log = 0;
    while ((1u << s_log) < s) ++s_log;
    const uint32_t M = N >> s_log;
    const uint32_t tn_w = c_o <= 16 ? 16u : (c_o <= 32 ? 32u : 64u);   // channel tile
    const uint32_t tiles_b = (B + MM_T - 1) / MM_T, tiles_n = (c_o + tn_w - 1) / tn_w;
    // blocks per workgroup: one unless the grid would exceed 16384 workgroups.  On the x4 stack
    // (L = 6, 2048 blocks) one block per workgroup ran the s = 8 layers in 445 us against 590 us
    // with four and 583 us with sixteen: the shorter workgroups fill the CUs more evenly
    uint32_t mb_log = 0;
    while (mb_log < 4 && (M >> (mb_log + 1)) >= 1 && (uint64_t)L * (M >> (mb_log + 1)) * tiles_b * tiles_n >= 16384)
        ++mb_log;
    const uint32_t tiles = L * (M >> mb_log) * tiles_b * tiles_n;
#define HE_MM(T)                                                                                              \
    HE_LAUNCH(ev, k_mac_mfma<T>, dim3(xcd_grid(tiles)), dim3(MM_THREADS), 0, st, X, Op, h, B, Jtot, Juse, c_o, L, \
              N, s_log, mb_log, tiles_b, tiles_n, lc)
    if (tn_w == 16) HE_MM(16);
    else if (tn_w == 32) HE_MM(32);
    else HE_MM(64);
#undef HE_MM
    return hipGetLastError();
}
