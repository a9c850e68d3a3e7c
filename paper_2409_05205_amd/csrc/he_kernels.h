// Launch interfaces of the HIP kernels (host side).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "he_device.h"

// Optional timing events for one launch: recorded by the dispatch itself
// (hipExtLaunchKernelGGL), so they add no packets between kernels.
struct LaunchEv {
    hipEvent_t start = nullptr, stop = nullptr;
};

#define HE_LAUNCH(ev, kernel, grid, block, lds, st, ...)                                                  \
    do {                                                                                                  \
        if ((ev) && (ev)->start)                                                                          \
            hipExtLaunchKernelGGL(kernel, grid, block, lds, st, (ev)->start, (ev)->stop, 0, __VA_ARGS__); \
        else                                                                                              \
            hipLaunchKernelGGL(kernel, grid, block, lds, st, __VA_ARGS__);                                \
    } while (0)

// Maps a flat row id r to (b, j, l) with l = r % L, j = (r / L) % J, b = r / (L J)
// and gives element strides of the source and destination polynomials.
struct RowMap {
    uint32_t J, L;
    uint64_t src_b, src_j, src_l;
    uint64_t dst_b, dst_j, dst_l;
};

// One or two forward-transform jobs in a single launch (rows of job 0 first).
struct FwdJobs {
    const uint32_t *src[2];
    uint32_t *dst[2];
    RowMap map[2];
    uint32_t rows0;
};

// Epilogues of the inverse transform.
enum EpiKind {
    EPI_STORE = 0,        // dst row = result (optionally times N^-1)
    EPI_CONV_CLASS = 1,   // write residue-class range of channel n into its output poly
    EPI_FC_PREFIX = 2     // write first n_o' coefficients plus Delta (d + sh') mod t
};

struct EpiParams {
    // geometry
    uint32_t c_o, g_o, K_out, s_log, n_o_p, blocks;
    // conv: out [B][K_out][L][N]; sh_next [B][K_out][N] or null
    // fc:   out [B][blocks][L][n_o_p]; sh_next [B][blocks][n_o_p] or null; bias [blocks][n_o_p]
    uint32_t *out;
    const uint32_t *sh_next;
    const int32_t *bias;
    uint32_t scale;   // EPI_STORE: 1 = multiply by N^-1
};

// Forward negacyclic NTT (natural order in, bit-reversed order out), rows of N words.
// logr = register radix log2 (2..5, threads per row N / 2^logr <= 1024); 0 = default choice.
hipError_t launch_ntt_fwd(int logn, const uint32_t *src, uint32_t *dst, const RowMap &map, uint32_t rows,
                          const uint32_t *tw, const uint32_t *twsh, const LimbConsts &lc, hipStream_t st,
                          const LaunchEv *ev = nullptr, int logr = 0);
hipError_t launch_ntt_fwd2(int logn, int logr, const FwdJobs &jobs, uint32_t rows, const uint32_t *tw,
                           const uint32_t *twsh, const LimbConsts &lc, hipStream_t st, const LaunchEv *ev = nullptr);

// Inverse (bit-reversed in, natural out, unscaled unless EPI_STORE with scale).
// For EPI_CONV_CLASS rows are (b, g, n', l) with l fastest; src is [B][c_o][L][N].
// For EPI_FC_PREFIX rows are (b, blk, l); src is [B][blocks][L][N].
hipError_t launch_ntt_inv(int logn, const uint32_t *src, uint32_t *dst, const RowMap &map, uint32_t rows,
                          const uint32_t *twi, const uint32_t *twish, const LimbConsts &lc,
                          int epi, const EpiParams &ep, hipStream_t st, const LaunchEv *ev = nullptr, int logr = 0);

// Pointwise MAC, full length: out[b][n][l][k] = sum_{J<Juse} X[b][J][l][k] * Op[n][l][J][k].
hipError_t launch_mac_full(const uint32_t *X, const uint32_t *Op, uint32_t *out, uint32_t B, uint32_t Jtot,
                           uint32_t Juse, uint32_t c_o, uint32_t L, uint32_t N, const LimbConsts &lc,
                           hipStream_t st, const LaunchEv *ev = nullptr);

// Pointwise MAC folded over residue blocks of s slots:
// h[b][n][l][blk] = sum_{J<Juse} sum_{u<s} X[b][J][l][blk s + u] * Op[n][l][J][blk s + u].
hipError_t launch_mac_class(const uint32_t *X, const uint32_t *Op, uint32_t *h, uint32_t B, uint32_t Jtot,
                            uint32_t Juse, uint32_t c_o, uint32_t L, uint32_t N, uint32_t s,
                            const LimbConsts &lc, hipStream_t st, const LaunchEv *ev = nullptr);

// Batched MAC, register-blocked over 4 images x 4 channels per thread (either form).
hipError_t launch_mac_tiled(const uint32_t *X, const uint32_t *Op, uint32_t *out, uint32_t B, uint32_t Jtot,
                            uint32_t Juse, uint32_t c_o, uint32_t L, uint32_t N, uint32_t s, bool class_form,
                            const LimbConsts &lc, hipStream_t st, const LaunchEv *ev = nullptr);

// Inverse transform of size N/s of each channel's folded vector, scattered to its residue
// class of the output poly, plus Delta sh'.  One workgroup per (b, g, l).
hipError_t launch_tail_class(const uint32_t *h, uint32_t *out, const uint32_t *sh_next, uint32_t B,
                             uint32_t c_o, uint32_t g_o, uint32_t K_out, uint32_t L, uint32_t N, uint32_t s,
                             const uint32_t *twi, const uint32_t *twish, const LimbConsts &lc,
                             hipStream_t st, const LaunchEv *ev = nullptr);

// Residue-class tail on registers: one (N/s)-point inverse per channel vector, several
// channel vectors per workgroup, coalesced scatter into the output poly (N/s >= 16).  The
// block sums are h[b][n][l][m], or h[l][b][n / 8][m][n % 8] with by_block (the matrix-core
// MAC's output; c_o a multiple of 8).
hipError_t launch_tail_rows(const uint32_t *h, uint32_t *out, const uint32_t *sh_next, uint32_t B, uint32_t c_o,
                            uint32_t g_o, uint32_t K_out, uint32_t L, uint32_t N, uint32_t s, const uint32_t *twi,
                            const uint32_t *twish, const LimbConsts &lc, hipStream_t st,
                            const LaunchEv *ev = nullptr, int logr = 0, bool by_block = false);

// LDS-staged batched MAC, residue-class form (s >= 2): same output as launch_mac_class.
struct MacLdsGeom {
    uint32_t TBq, TNq;        // thread sub-tile grid: TB = 4 TBq images x TN = 4 TNq channels
    uint32_t GS, R;           // slots per thread span and per stage
    uint32_t cpb, gpb;        // stages per block and row (1 when a stage holds whole blocks); groups per block
    uint32_t ranges;          // slot ranges per limb
    uint32_t tiles_b, tiles_n;
};
// short_stage: slots per stage for blocks shorter than 16 slots (32 with register staging, 64 by DMA).
bool mac_lds_geometry(uint32_t B, uint32_t c_o, uint32_t N, uint32_t s, MacLdsGeom *gm, size_t *lds_bytes,
                      uint32_t short_stage);
hipError_t launch_mac_lds(const uint32_t *X, const uint32_t *Op, uint32_t *h, uint32_t B, uint32_t Jtot,
                          uint32_t Juse, uint32_t c_o, uint32_t L, uint32_t N, uint32_t s, bool xcd_order,
                          const LimbConsts &lc, hipStream_t st, const LaunchEv *ev = nullptr);
// LDS bytes of the DMA-staged form for geometry gm (from mac_lds_geometry with 64-slot short
// stages), or SIZE_MAX when the form cannot take it.
size_t mac_dma_lds_bytes(const MacLdsGeom &gm);
// Same products and output as launch_mac_lds, with the stages moved to LDS by global_load_lds
// (three stage buffers, no register staging).
hipError_t launch_mac_dma(const uint32_t *X, const uint32_t *Op, uint32_t *h, uint32_t B, uint32_t Jtot,
                          uint32_t Juse, uint32_t c_o, uint32_t L, uint32_t N, uint32_t s, bool xcd_order,
                          const LimbConsts &lc, hipStream_t st, const LaunchEv *ev = nullptr);

// The same block sums on the integer matrix cores (kernels_mac_mfma.hip): residues split into
// signed base-256 digits, digit-plane products accumulated exactly in i32, written in groups of 8
// channels (h[l][b][n / 8][m][n % 8], for launch_tail_rows with by_block).  Needs c_o a multiple
// of 8, s a power of two >= 4, N/s >= 16 and Juse s <= 32768 (mac_mfma_ok).
bool mac_mfma_ok(uint32_t B, uint32_t c_o, uint32_t Juse, uint32_t N, uint32_t s);
hipError_t launch_mac_mfma(const uint32_t *X, const uint32_t *Op, uint32_t *h, uint32_t B, uint32_t Jtot,
                           uint32_t Juse, uint32_t c_o, uint32_t L, uint32_t N, uint32_t s, const LimbConsts &lc,
                           hipStream_t st, const LaunchEv *ev = nullptr);

// Fused class-form MAC + residue-class tail: one workgroup per output row
// (b, g, n', l); same output as launch_mac_class followed by launch_tail_rows.
// Requires s <= 256, 16 <= N/s <= 16384, N >= 256.
hipError_t launch_mac_tail(const uint32_t *X, const uint32_t *Op, uint32_t *out, const uint32_t *sh_next, uint32_t B,
                           uint32_t Jtot, uint32_t Juse, uint32_t c_o, uint32_t g_o, uint32_t K_out, uint32_t L,
                           uint32_t N, uint32_t s, const uint32_t *twi, const uint32_t *twish, const LimbConsts &lc,
                           hipStream_t st, const LaunchEv *ev = nullptr);

// One launch per layer call (kernels_fused.hip): forward NTT of the input rows, coefficient-wise
// MAC and inverse with extraction, as work items in workgroup order that wait on counters in a
// zeroed sync block of FZ_SYNC_WORDS words (left zero again when the launch ends).
enum { FZ_KIND_CONV = 0, FZ_KIND_FC = 1 };
enum { FZ_SB_ERR = 2, FZ_SB_HDR = 64, FZ_SYNC_WORDS = 16384 };
struct FusedLayer {
    const uint32_t *c0;       // [B][K_in][L][N] coefficient form (ntt_c0 = K_in), else unused
    const uint32_t *sh;       // [B][K_in][N] shares (ntt_sh = K_in), else unused
    const uint32_t *sh_next;  // conv [B][K_out][N]; fc [B][blocks][n_o_p]; or null
    uint32_t *out;            // conv [B][K_out][L][N]; fc [B][blocks][L][n_o_p]
    const uint32_t *op;       // resident operands [rows][L][Jtot][N]
    const int32_t *bias;      // fc [blocks][n_o_p]
    uint32_t *x;              // NTT-domain inputs [B][Jtot][L][N] (written by the NTT items)
    uint32_t *h;              // conv block sums [B][c_o][L][N/s]; fc chunk shares [B][blocks][L][N/1024][n_o_p]
    uint32_t kind;            // FZ_KIND_CONV (residue-class form) or FZ_KIND_FC
    uint32_t B, K_in, Jtot, Juse;
    uint32_t rows;            // c_o (conv) or blocks (fc)
    uint32_t g_o, K_out, L, logN, s_log, n_o_p;
    uint32_t ntt_c0, ntt_sh;  // input rows per image transformed in this launch (K_in or 0 each)
    uint32_t rows_form;       // conv: 1 = whole-row NTT items and one MAC + tail item per output row
                              // (1024-thread workgroups); 0 = sub-block NTT, MAC chunk and tail items
    uint32_t mac_tiled;       // conv, grouped launch: MAC items are LDS-staged tiles of images x
                              // channels (geometry gm); 0 = one image per MAC item
    uint32_t grouped;         // planned for the grouped launch: per-image conv MAC items by channel
                              // groups only, tails of 128 threads per vector from 512 points up
    MacLdsGeom gm;
    // filled by fused_layer_plan.  Counters go per image tile of 2^tile_log images (n_tiles of
    // them; one image per tile unless the MAC is tiled)
    uint32_t ng, mac_per_bl, tail_rw, n_ntt, n_mac, n_inv, n_ctr, ctr_stride, tile_log, n_tiles;
};
// Whether the one-launch form handles this layer shape (N 4096..16384; conv 2 <= s <= 256 with
// N/s <= 4096; fc n_o' <= 1024).
bool fused_layer_ok(const FusedLayer &jb);
// Item counts, per-item geometry and counter spacing; returns the words the launch's counters
// span past FZ_SB_HDR.
uint32_t fused_layer_plan(FusedLayer &jb);
hipError_t launch_fused_layer(const FusedLayer &jb, const uint32_t *tw, const uint32_t *twsh, const uint32_t *twi,
                              const uint32_t *twish, const uint32_t *xinv, const LimbConsts &lc, uint32_t *sync,
                              hipStream_t st, const LaunchEv *ev = nullptr);

// Grouped launch: the work items of several independent layer calls (any contexts, shapes and
// batch sizes) in one launch, read from a device-side job list.  Each job is a planned
// FusedLayer (rows_form = 0) with its context's tables and its own counters.
struct FusedJob {
    FusedLayer jb;
    const uint32_t *tw, *twsh, *twi, *twish, *xinv;
    const LimbConsts *lc;     // device copy of the context's limb constants
    uint32_t ctr_off;         // the job's counters: words past FZ_SB_HDR of the group's sync block
    uint32_t first[3];        // first item of the job in each phase (NTT, MAC, tail)
};
// Largest LDS need (bytes) of a tiled MAC item the grouped launch accepts.
uint32_t fused_group_lds_bytes();
// jobs: device array of n_jobs entries; count[p]: items of phase p over all jobs; the items of a
// phase go to the XCDs in chunks of 2^chunk_log (0..10).
hipError_t launch_fused_group(const FusedJob *jobs, uint32_t n_jobs, const uint32_t count[3], uint32_t chunk_log,
                              uint32_t *sync, hipStream_t st, const LaunchEv *ev = nullptr);

// Client masks from the server's resident operands (kernels_client.hip): noise rows into the
// operand layout, then the combination with NTT(b) (in place on E).
hipError_t launch_mask_noise(const int32_t *e1, const int32_t *e2, uint32_t *E, uint32_t K_in, uint32_t n_rows,
                             uint32_t L, uint32_t N, const LimbConsts &lc, hipStream_t st);
hipError_t launch_mask_combine(const uint32_t *S, const uint32_t *bhat, uint32_t *E, uint32_t K_in, uint32_t n_rows,
                               uint32_t L, uint32_t N, const LimbConsts &lc, hipStream_t st);

// Client-side element-wise kernels (kernels_client.hip).
struct DecConsts {
    uint32_t t;
    uint32_t inv[HE_MAX_LIMBS];      // (Q / q_l)^-1 mod q_l
    uint32_t inv_sh[HE_MAX_LIMBS];   // Shoup companions
};
// out[r][l][k] = a[r][k] mod q_l for signed a
hipError_t launch_lift_signed(const int32_t *a, uint32_t *out, uint32_t rows, uint32_t L, uint32_t N,
                              const LimbConsts &lc, hipStream_t st);
// c[r][l][k] = a[r][l][k] * b[l][k] mod q_l
hipError_t launch_mul_bcast(const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t rows, uint32_t L, uint32_t N,
                            const LimbConsts &lc, hipStream_t st);
// out[r][l][k] = -(vb[r][l][k] + Delta_l msg[r][k] + e0[r][k]) mod q_l
hipError_t launch_encrypt_combine(const uint32_t *vb, const uint32_t *msg, const int32_t *e0, uint32_t *out,
                                  uint32_t rows, uint32_t L, uint32_t N, const LimbConsts &lc, hipStream_t st);
// msg[r][k] = round(t CRT(x0 + x1) / Q) mod t   (x1 may be null)
hipError_t launch_decrypt(const uint32_t *x0, const uint32_t *x1, uint32_t *msg, uint32_t rows, uint32_t L, uint32_t N,
                          const LimbConsts &lc, const DecConsts &dc, hipStream_t st);

// Pack-time helpers.
// Op[n][l][j][k]         = rho[j][n][k]                         for j < K_in
// Op[n][l][K_in + j][k]  = -Delta_l fhat[j][n][k] mod q_l         (fhat int16)
hipError_t launch_expand_operands(const uint32_t *rho, const int16_t *fhat, uint32_t *Op, uint32_t K_in,
                                  uint32_t c_o, uint32_t L, uint32_t N, const LimbConsts &lc, hipStream_t st);
// Op[n][l][J][k] *= N^-1 * xinv[l][k]^cls(n)   (cls = nullptr: factor N^-1 only)
hipError_t launch_scale_operands(uint32_t *Op, const uint32_t *xinv, const uint32_t *cls, uint32_t Jtot,
                                 uint32_t c_o, uint32_t L, uint32_t N, const LimbConsts &lc, hipStream_t st);
// c[r][l][k] = a[r][l][k] * b[r][l][k] mod q_l
hipError_t launch_pointwise_mul(const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t rows, uint32_t L,
                                uint32_t N, const LimbConsts &lc, hipStream_t st);

// Library-internal (he_api.hip): suppress kernel timing on the calling thread, e.g. while a
// graph is captured; returns the previous setting.
bool he_prof_suppress(bool on);
