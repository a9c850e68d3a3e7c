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
#include "ntt_device.h"

namespace {

// PF: twiddles of the first passes prefetched into registers (a launch of a few rows, where
// their latency would otherwise stand alone) or read per pass (many rows: occupancy instead).
template <int LOGN, int LOGR, bool PF>
__global__ void __launch_bounds__(1 << (LOGN - LOGR))
k_ntt_fwd(FwdJobs jobs, const uint32_t *__restrict__ tw, const uint32_t *__restrict__ twsh, LimbConsts lc) {
    constexpr int N = 1 << LOGN;
    constexpr int T = 1 << (LOGN - LOGR);
    constexpr int TWB = PF ? T : TW_IN_PASS;
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
    const uint32_t *W = tw + (size_t)l * N;
    const uint32_t *Wsh = twsh + (size_t)l * N;
    PassTw<LOGN, LOGR, TWB> ptw;
    fwd_tw_load<LOGN, LOGR, TWB, 0>(ptw, tid, W, Wsh);
    uint32_t v[1 << LOGR];
    fwd_pass<LOGN, LOGR, TWB, 0>(v, ptw, lds, tid, in, W, Wsh, q, q2);
#pragma unroll
    for (int i = 0; i < (1 << LOGR); ++i) {
        const uint32_t idx = tid + i * T;
        uint32_t x = lds[lpad(idx)];
        x = csub(x, q2);
        out[idx] = csub(x, q);
    }
}

// A launch of few rows leaves most CUs idle while each row's transform is ALU time on one CU.
// Here 2^K workgroups share a row: after the first K stages the row splits into 2^K independent
// sub-transforms of N / 2^K points, so workgroup `sub` reads the whole row, forms the K leading
// stages of its own sub-block on load (fwd_lead) and runs the rest alone; no workgroup waits for
// another.  The output words and their positions are those of k_ntt_fwd.
template <int LOGN, int LOGR, int K>
__global__ void __launch_bounds__(1 << (LOGN - K - LOGR))
k_ntt_fwd_split(FwdJobs jobs, const uint32_t *__restrict__ tw, const uint32_t *__restrict__ twsh, LimbConsts lc) {
    constexpr int LS = LOGN - K;
    constexpr int NS = 1 << LS;
    constexpr int T = 1 << (LS - LOGR);
    __shared__ uint32_t lds[NS + (NS >> 5)];
    const uint32_t tid = threadIdx.x;
    const uint32_t sub = blockIdx.x & ((1u << K) - 1u);
    uint32_t r = blockIdx.x >> K;
    const int js = r < jobs.rows0 ? 0 : 1;       // rows of job 0 first, then job 1
    if (js) r -= jobs.rows0;
    const RowMap &map = jobs.map[js];
    const uint32_t l = r % map.L;
    const uint32_t jb = r / map.L;
    const uint32_t j = jb % map.J;
    const uint32_t b = jb / map.J;
    const uint32_t *in = jobs.src[js] + b * map.src_b + j * map.src_j + l * map.src_l;
    uint32_t *out = jobs.dst[js] + b * map.dst_b + j * map.dst_j + l * map.dst_l + (size_t)sub * NS;
    const uint32_t q = lc.l[l].q, q2 = lc.l[l].q2;
    const uint32_t *W = tw + (size_t)l * (NS << K);
    const uint32_t *Wsh = twsh + (size_t)l * (NS << K);
    const uint32_t tb = (1u << K) + sub;
    PassTw<LS, LOGR, T> ptw;
    fwd_tw_load<LS, LOGR, T, 0>(ptw, tid, W, Wsh, tb);
    uint32_t v[1 << LOGR];
    fwd_pass<LS, LOGR, T, 0, K>(v, ptw, lds, tid, in, W, Wsh, q, q2, tb, sub);
#pragma unroll
    for (int i = 0; i < (1 << LOGR); ++i) {
        const uint32_t idx = tid + i * T;
        uint32_t x = lds[lpad(idx)];
        x = csub(x, q2);
        out[idx] = csub(x, q);
    }
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

    const uint32_t *W = twi + (size_t)l * N;
    const uint32_t *Wsh = twish + (size_t)l * N;
    PassTw<LOGN, LOGR, T> ptw;
    inv_tw_load<LOGN, LOGR, T, 0>(ptw, tid, W, Wsh);
    // coalesced load into LDS
#pragma unroll
    for (int i = 0; i < (1 << LOGR); ++i) {
        const uint32_t idx = tid + i * T;
        lds[lpad(idx)] = in[idx];
    }
    __syncthreads();
    uint32_t v[1 << LOGR];
    inv_pass<LOGN, LOGR, T, 0>(v, ptw, lds, tid, W, Wsh, q, q2);

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

// Rows shared by 2^K workgroups when a launch has at most 64 (K = 2) or 128 (K = 1) rows of
// N >= 4096; 0 otherwise.  A shared row is read whole by each of its 2^K workgroups while each
// writes only its own sub-block, so a launch that transforms any row in place (destination
// overlapping the source) keeps whole rows: one workgroup per row reads all of it before its
// first store.
inline bool fwd_job_in_place(const FwdJobs &jobs, uint32_t rows, uint32_t n) {
    uintptr_t lo[2][2], hi[2][2];   // [job][source, destination] byte ranges
    int nj = 0;
    for (int i = 0; i < 2; ++i) {
        const uint32_t jr = i == 0 ? (rows < jobs.rows0 ? rows : jobs.rows0) : (rows > jobs.rows0 ? rows - jobs.rows0 : 0);
        if (jr == 0) continue;
        const RowMap &m = jobs.map[i];
        const uint64_t nb = (jr + m.J * m.L - 1) / (m.J * m.L);   // images of the job
        const uint64_t se = (nb - 1) * m.src_b + (m.J - 1) * m.src_j + (m.L - 1) * m.src_l + n;
        const uint64_t de = (nb - 1) * m.dst_b + (m.J - 1) * m.dst_j + (m.L - 1) * m.dst_l + n;
        lo[nj][0] = (uintptr_t)jobs.src[i];
        hi[nj][0] = lo[nj][0] + se * 4;
        lo[nj][1] = (uintptr_t)jobs.dst[i];
        hi[nj][1] = lo[nj][1] + de * 4;
        ++nj;
    }
    for (int a = 0; a < nj; ++a)
        for (int b = 0; b < nj; ++b)
            if (lo[a][0] < hi[b][1] && lo[b][1] < hi[a][0]) return true;
    return false;
}

inline int fwd_split_k(int logn, uint32_t rows, bool in_place) {
    if (logn < 12 || in_place) return 0;
    return rows <= 64 ? 2 : (rows <= 128 ? 1 : 0);
}

template <int LOGN, int LOGR>
hipError_t fwd_launch(const FwdJobs &jobs, uint32_t rows, const uint32_t *tw, const uint32_t *twsh,
                      const LimbConsts &lc, hipStream_t st, const LaunchEv *ev) {
    if constexpr (LOGN >= 12) {
        // the radix applies to the sub-transforms; one the split cannot take keeps whole rows
        const int k = fwd_split_k(LOGN, rows, fwd_job_in_place(jobs, rows, 1u << LOGN));
        if (k == 2 && valid_variant(LOGN - 2, LOGR)) {
            if constexpr (valid_variant(LOGN - 2, LOGR)) {
                HE_LAUNCH(ev, (k_ntt_fwd_split<LOGN, LOGR, 2>), dim3(rows << 2), dim3(1 << (LOGN - 2 - LOGR)), 0, st,
                          jobs, tw, twsh, lc);
                return hipGetLastError();
            }
        }
        if (k == 1 && valid_variant(LOGN - 1, LOGR)) {
            if constexpr (valid_variant(LOGN - 1, LOGR)) {
                HE_LAUNCH(ev, (k_ntt_fwd_split<LOGN, LOGR, 1>), dim3(rows << 1), dim3(1 << (LOGN - 1 - LOGR)), 0, st,
                          jobs, tw, twsh, lc);
                return hipGetLastError();
            }
        }
    }
    if constexpr (valid_variant(LOGN, LOGR)) {
        // a launch of up to one row per CU keeps the twiddle prefetch; larger ones read per pass
        if (rows <= 256)
            HE_LAUNCH(ev, (k_ntt_fwd<LOGN, LOGR, true>), dim3(rows), dim3(1 << (LOGN - LOGR)), 0, st, jobs, tw, twsh, lc);
        else
            HE_LAUNCH(ev, (k_ntt_fwd<LOGN, LOGR, false>), dim3(rows), dim3(1 << (LOGN - LOGR)), 0, st, jobs, tw, twsh, lc);
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
// A launch has thousands of workgroups, so registers go to occupancy rather than to
// prefetched twiddles (each pass reads its own from cache), and the sh' words of the
// write are fetched with the channel rows, so that their latency overlaps the inverse.

template <int LOGM, int LOGR>
constexpr int tail_tpw() { return (1 << (LOGM - LOGR)) < 256 ? 256 : (1 << (LOGM - LOGR)); }

template <int LOGM, int LOGR>
__global__ void __launch_bounds__((tail_tpw<LOGM, LOGR>()))
k_tail_rows(const uint32_t *__restrict__ h, uint32_t *__restrict__ out, const uint32_t *__restrict__ sh_next,
            uint32_t B, uint32_t c_o, uint32_t g_o, uint32_t K_out, uint32_t L, uint32_t logN, uint32_t s_log, uint32_t RW,
            const uint32_t *__restrict__ twi, const uint32_t *__restrict__ twish, LimbConsts lc, uint32_t by_block) {
    constexpr int M = 1 << LOGM;
    constexpr int T = 1 << (LOGM - LOGR);
    constexpr int MP = M + (M >> 5);
    extern __shared__ uint32_t lds[];
    const uint32_t tid = threadIdx.x;
    const uint32_t row = tid / T;               // row within the workgroup
    const uint32_t t = tid % T;
    const uint32_t chunks = g_o / RW;
    uint32_t w;
    if (!xcd_logical(blockIdx.x, B * K_out * L * chunks, w)) return;
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
    const uint32_t *W = twi + (size_t)l * N;
    const uint32_t *Wsh = twish + (size_t)l * N;
    PassTw<LOGM, LOGR, TW_IN_PASS> ptw;
    inv_tw_load<LOGM, LOGR, TW_IN_PASS, 0>(ptw, t, W, Wsh);
    // g_o, RW and s are powers of two: class width, span and indices by shifts
    const uint32_t cw_log = s_log - (31u - __clz(g_o));
    const uint32_t span_log = (31u - __clz(RW)) + cw_log;
    const uint32_t c_lo = np0 << cw_log;
    const uint32_t *sh = sh_next ? sh_next + (size_t)(b * K_out + g) * N : nullptr;
    const uint32_t total = (uint32_t)M << span_log;
    if (!by_block) {
        if (active) {
            const uint32_t *src = h + ((size_t)(b * c_o + (exists ? n : 0)) * L + l) * M;
#pragma unroll
            for (int i = 0; i < (1 << LOGR); ++i) {
                const uint32_t idx = t + i * T;
                my[lpad(idx)] = exists ? src[idx] : 0u;
            }
        }
    } else {
        // sums in groups of 8 channels, h[l][b][n / 8][m][n % 8] (c_o a multiple of 8): a block's
        // words of 8 channels are adjacent, so the workgroups of neighbouring channels, which run
        // together, read whole 32-byte pieces between them
        const uint32_t rw_log = 31u - __clz(RW);
        const uint32_t nb = g * g_o + np0;
        const uint32_t *src = h + (size_t)(l * B + b) * c_o * M;
        for (uint32_t e = tid; e < ((uint32_t)M << rw_log); e += blockDim.x) {
            const uint32_t r = e & (RW - 1u), idx = e >> rw_log, n = nb + r;
            lds[r * MP + lpad(idx)] = n < c_o ? src[((size_t)(n >> 3) * M + idx) * 8u + (n & 7u)] : 0u;
        }
    }
    // the sh' words of the first 16 write rounds, fetched now so that they arrive during the inverse
    constexpr int TPF = 16;
    uint32_t shv[TPF];
#pragma unroll
    for (int i = 0; i < TPF; ++i) {
        const uint32_t e = tid + i * blockDim.x;
        shv[i] = (sh && e < total) ? sh[((e >> span_log) << s_log) + c_lo + (e & ((1u << span_log) - 1u))] : 0u;
    }
    __syncthreads();
    uint32_t v[1 << LOGR];
    inv_pass<LOGM, LOGR, TW_IN_PASS, 0>(v, ptw, my, t, W, Wsh, c.q, c.q2);
    __syncthreads();
    if (active) {
#pragma unroll
        for (int i = 0; i < (1 << LOGR); ++i) my[lpad(inv_final_idx<LOGM, LOGR>(t, i))] = csub(v[i], c.q);
    }
    __syncthreads();
    uint32_t *o = out + ((size_t)(b * K_out + g) * L + l) * N;
    auto put = [&](uint32_t e, uint32_t shw) {
        const uint32_t m = e >> span_log;
        const uint32_t off = e & ((1u << span_log) - 1u);
        const uint32_t r = off >> cw_log;
        uint32_t val = 0;
        if ((off & ((1u << cw_log) - 1u)) == 0 && g * g_o + np0 + r < c_o) val = lds[r * MP + lpad(m)];
        if (sh) val = csub(val + mul_delta_msg(shw, c), c.q);
        o[(m << s_log) + c_lo + off] = val;
    };
#pragma unroll
    for (int i = 0; i < TPF; ++i) {
        const uint32_t e = tid + i * blockDim.x;
        if (e < total) put(e, shv[i]);
    }
    for (uint32_t e = tid + TPF * blockDim.x; e < total; e += blockDim.x) {
        const uint32_t m = e >> span_log, off = e & ((1u << span_log) - 1u);
        put(e, sh ? sh[(m << s_log) + c_lo + off] : 0u);
    }
}

template <int LOGM, int LOGR>
hipError_t tail_launch(const uint32_t *h, uint32_t *out, const uint32_t *sh_next, uint32_t B, uint32_t c_o,
                       uint32_t g_o, uint32_t K_out, uint32_t L, uint32_t logN, uint32_t s_log, const uint32_t *twi,
                       const uint32_t *twish, const LimbConsts &lc, hipStream_t st, const LaunchEv *ev,
                       uint32_t by_block) {
    if constexpr (valid_variant(LOGM, LOGR)) {
        constexpr int T = 1 << (LOGM - LOGR);
        constexpr int TPW = tail_tpw<LOGM, LOGR>();
        uint32_t RW = TPW / T;
        if (RW > g_o) RW = g_o;
        const uint32_t grid = xcd_grid(B * K_out * L * (g_o / RW));
        const size_t lds = (size_t)(TPW / T) * ((1u << LOGM) + (1u << LOGM >> 5)) * sizeof(uint32_t);
        HE_LAUNCH(ev, (k_tail_rows<LOGM, LOGR>), dim3(grid), dim3(TPW), lds, st, h, out, sh_next, B, c_o, g_o,
                  K_out, L, logN, s_log, RW, twi, twish, lc, by_block);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------ fused MAC + residue-class tail
// One workgroup per output row (b, g, n', l).  It accumulates the
// coefficient-wise products of its channel over all N slots and sums the s
// slots of each block (as the class-form MAC does), keeps the M = N/s block
// sums in LDS, inverts them there (the M-point Gentleman-Sande of k_tail_rows)
// and writes its span of residue classes plus Delta sh'.  Against the MAC and
// tail launches it saves one launch and the round trip of the block sums
// through memory; the sh' words it adds are fetched at entry so that their
// latency overlaps the MAC.
constexpr int MT_THREADS = 1024;
constexpr int MT_PF = 8;   // sh' words per thread fetched at entry

template <int LOGM>
constexpr int mt_logr() { return LOGM - 10 > 2 ? LOGM - 10 : 2; }

// Workgroups go round-robin over the 8 XCDs.  When the limb count does not divide 8, a
// limb-fastest order would spread several limbs' input rows over every XCD's L2.
__host__ __device__ constexpr bool mt_xcd_order(uint32_t L) { return L != 0u && (8u % L) != 0u; }

template <int LOGM>
__global__ void __launch_bounds__(MT_THREADS)
k_mac_tail(const uint32_t *__restrict__ X, const uint32_t *__restrict__ Op, uint32_t *__restrict__ out,
           const uint32_t *__restrict__ sh_next, uint32_t Jtot, uint32_t Juse, uint32_t c_o, uint32_t g_o,
           uint32_t K_out, uint32_t L, uint32_t rows, uint32_t logN, uint32_t s_log, const uint32_t *__restrict__ twi,
           const uint32_t *__restrict__ twish, LimbConsts lc) {
    constexpr int LOGR = mt_logr<LOGM>();
    constexpr int M = 1 << LOGM;
    constexpr int T = 1 << (LOGM - LOGR);
    __shared__ uint32_t lds[M + (M >> 5)];
    const uint32_t tid = threadIdx.x;
    const uint32_t tpb = blockDim.x;             // N/4 or MT_THREADS: every thread has the same chunk count
    uint32_t w, l;
    if (mt_xcd_order(L)) {
        // limb slowest, each XCD a contiguous range: its workgroups cover one or two limbs, whose
        // input rows then stay in that XCD's L2 for all of its output rows
        if (!xcd_logical(blockIdx.x, rows, w)) return;
        const uint32_t per_limb = rows / L;
        l = w / per_limb;
        w %= per_limb;
    } else {
        // limb fastest: with L dividing 8, the round-robin dispatch already gives each XCD one limb
        w = blockIdx.x;
        l = w % L;
        w /= L;
    }
    const uint32_t np = w % g_o;
    w /= g_o;
    const uint32_t g = w % K_out;
    const uint32_t b = w / K_out;
    const uint32_t n = g * g_o + np;
    const bool exists = n < c_o;                 // uniform over the workgroup
    const LimbConst c = lc.l[l];
    const uint32_t N = 1u << logN;
    const uint32_t s = 1u << s_log;
    // this channel's output span: classes [c_lo, c_lo + cw) of every block, cw = s / g_o
    const uint32_t cw_log = s_log - (31u - __clz(g_o));
    const uint32_t cw_mask = (1u << cw_log) - 1u;
    const uint32_t c_lo = np << cw_log;
    const uint32_t total = (uint32_t)M << cw_log;
    uint32_t *o = out + ((size_t)(b * K_out + g) * L + l) * N;
    const uint32_t *sh = sh_next ? sh_next + (size_t)(b * K_out + g) * N : nullptr;
    uint32_t shv[MT_PF];
#pragma unroll
    for (int i = 0; i < MT_PF; ++i) {
        const uint32_t e = tid + i * tpb;
        shv[i] = (sh && e < total) ? sh[((e >> cw_log) << s_log) + c_lo + (e & cw_mask)] : 0u;
    }
    if (exists) {
        const uint32_t *W = twi + (size_t)l * N;
        const uint32_t *Wsh = twish + (size_t)l * N;
        const bool act = tid < (uint32_t)T;
        PassTw<LOGM, LOGR, MT_THREADS> ptw;
        inv_tw_load<LOGM, LOGR, MT_THREADS, 0>(ptw, act ? tid : 0u, W, Wsh);
        const uint32_t *x = X + ((size_t)b * Jtot * L + l) * N;
        const uint32_t *op = Op + (size_t)(n * L + l) * Jtot * N;
        for (uint32_t k4 = tid * 4u; k4 < N; k4 += tpb * 4u) {
            uint32_t r[4];
            mac4(x + k4, (size_t)L * N, op + k4, N, Juse, c, r);
            if (s == 1) {
#pragma unroll
                for (int i = 0; i < 4; ++i) lds[lpad(k4 + i)] = r[i];
            } else if (s == 2) {
                lds[lpad(k4 >> 1)] = addmod(r[0], r[1], c.q);
                lds[lpad((k4 >> 1) + 1)] = addmod(r[2], r[3], c.q);
            } else {
                // the s slots of a block are held by s/4 consecutive lanes
                uint32_t v = r[0] + r[1] + r[2] + r[3];   // [0, 4q)
                v = csub(csub(v, c.q2), c.q);
                const uint32_t lanes = s >> 2;
                for (uint32_t m = 1; m < lanes; m <<= 1) v = addmod(v, (uint32_t)__shfl_xor((int)v, (int)m), c.q);
                if ((tid & (lanes - 1)) == 0) lds[lpad(k4 >> s_log)] = v;
            }
        }
        __syncthreads();
        uint32_t v[1 << LOGR];
        inv_pass<LOGM, LOGR, MT_THREADS, 0>(v, ptw, lds, act ? tid : 0u, W, Wsh, c.q, c.q2, act);
        __syncthreads();
        if (act) {
#pragma unroll
            for (int i = 0; i < (1 << LOGR); ++i) lds[lpad(inv_final_idx<LOGM, LOGR>(tid, i))] = csub(v[i], c.q);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < MT_PF; ++i) {
        const uint32_t e = tid + i * tpb;
        if (e < total) {
            const uint32_t m = e >> cw_log, off = e & cw_mask;
            uint32_t val = (exists && off == 0) ? lds[lpad(m)] : 0u;
            if (sh) val = csub(val + mul_delta_msg(shv[i], c), c.q);
            o[(m << s_log) + c_lo + off] = val;
        }
    }
    for (uint32_t e = tid + MT_PF * tpb; e < total; e += tpb) {
        const uint32_t m = e >> cw_log, off = e & cw_mask;
        const uint32_t k = (m << s_log) + c_lo + off;
        uint32_t val = (exists && off == 0) ? lds[lpad(m)] : 0u;
        if (sh) val = csub(val + mul_delta_msg(sh[k], c), c.q);
        o[k] = val;
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
                            int logr, bool by_block) {
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
#define HE_TAIL(LM, LR) \
    tail_launch<LM, LR>(h, out, sh_next, B, c_o, g_o, K_out, L, logN, s_log, twi, twish, lc, st, ev, by_block ? 1u : 0u)
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

hipError_t launch_mac_tail(const uint32_t *X, const uint32_t *Op, uint32_t *out, const uint32_t *sh_next, uint32_t B,
                           uint32_t Jtot, uint32_t Juse, uint32_t c_o, uint32_t g_o, uint32_t K_out, uint32_t L,
                           uint32_t N, uint32_t s, const uint32_t *twi, const uint32_t *twish, const LimbConsts &lc,
                           hipStream_t st, const LaunchEv *ev) {
    if (B == 0) return hipSuccess;
    uint32_t logN = 0, s_log = 0;
    while ((1u << logN) < N) ++logN;
    while ((1u << s_log) < s) ++s_log;
    const int logm = (int)(logN - s_log);
    // s/4 lanes per block within one wave; every thread owns the same number of 4-slot chunks
    if (s > 256 || logm < 4 || logm > 14 || N < 256 || g_o == 0 || g_o > s || Juse == 0) return hipErrorInvalidValue;
    const uint32_t tpb = N / 4 < (uint32_t)MT_THREADS ? N / 4 : (uint32_t)MT_THREADS;
    const uint32_t rows = B * K_out * g_o * L;
    const uint32_t grid = mt_xcd_order(L) ? xcd_grid(rows) : rows;
#define HE_MT(LM)                                                                                                    \
    case LM:                                                                                                         \
        HE_LAUNCH(ev, k_mac_tail<LM>, dim3(grid), dim3(tpb), 0, st, X, Op, out, sh_next, Jtot, Juse, c_o, g_o, K_out, \
                  L, rows, logN, s_log, twi, twish, lc);                                                             \
        return hipGetLastError();
    switch (logm) {
        HE_MT(4)
        HE_MT(5)
        HE_MT(6)
        HE_MT(7)
        HE_MT(8)
        HE_MT(9)
        HE_MT(10)
        HE_MT(11)
        HE_MT(12)
        HE_MT(13)
        HE_MT(14)
        default: return hipErrorInvalidValue;
    }
#undef HE_MT
}
