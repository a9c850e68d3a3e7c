/*
 * he.h -- C ABI of the rotation-free HE Conv/FC server path on MI355X (gfx950).
 *
 * The library evaluates the server side of the paper's Conv and FC procedures
 * (Alg. 1 "Proposed HE convolution procedure", server evaluation; Alg. 2
 * "Proposed FC evaluation procedure with HE", server evaluation) in the exact
 * BFV-style reading: R_q = Z_q[X]/(X^N + 1) over L RNS limbs of 30-bit primes,
 * plaintext modulus t, Delta = floor(Q / t).
 *
 *   conv:  c0^(n) = sum_j c0_j rho_j^(n) - Delta sh_j fhat_j^(n)        (Alg. 1)
 *          out_g  = residue class o_n of c0^(n) for the channels n of group g,
 *                   zero elsewhere, plus Delta sh'_g                       (Alg. 1)
 *   fc:    out_b  = first n_o' coefficients of c0 rho_b - Delta sh w_b,
 *                   plus Delta ((d_b + sh'_b) mod t)                       (Alg. 2)
 *
 * Packing follows Eq. (k_batch_new) / Eq. (i_batch) for conv, generalised to
 * c_o > c_i, zero padding and inputs wider than one polynomial:
 *   H_p = H + 2 pad, W_p = W + 2 pad, s = 2^floor(log2(N / (H_p W_p))),
 *   g_i = min(c_i, s), g_o = largest power of two <= min(c_o, s),
 *   K_in = ceil(c_i / g_i), K_out = ceil(c_o / g_o), o_n = (n mod g_o) s / g_o.
 *   Input poly j, coefficient s (y W_p + x) + m' holds channel j g_i + m' at
 *   padded pixel (y, x); output channel n at output pixel (oy, ox) is
 *   coefficient s (stride oy W_p + stride ox) + o_n of output poly n / g_o.
 * and Eq. (i(x) formula) / Eq. (w(x) formula) with Theorem 1 for FC, with
 *   n_o' = n_o rounded up to a power of two (or 2^floor(log2(N / n_i)) rows per
 *   block when n_i n_o' > N), n_i' = N / n_o', blocks = ceil(n_o / n_o'),
 *   input coefficient l n_o' holds input l.
 *
 * Conventions for every call:
 *  - Polynomials at the boundary are in coefficient form, u32, contiguous,
 *    limb-major (the limb axis sits just before the N axis), residues in
 *    [0, q_l).  Shares sh / sh' hold values in [0, t) and carry no limb axis.
 *  - Pointers named d_* are device memory owned by the caller; they must stay
 *    valid until the stream reaches the call.  Host pointers are read before
 *    the call returns.  The library owns contexts and layers.
 *  - Layer calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream).  Error codes are returned before any launch when the arguments
 *    are invalid; nothing is written in that case.
 *  - Contexts and layers are bound to the device that was current at creation.
 */
#ifndef HE_H
#define HE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    HE_OK = 0,
    HE_EINVAL = -1,        /* invalid argument or parameter set            */
    HE_EUNSUPPORTED = -2,  /* valid but outside what this build handles    */
    HE_ENOMEM = -3,        /* device or host allocation failed             */
    HE_EDEVICE = -4        /* a HIP runtime call or kernel launch failed   */
};

enum { HE_LAYER_CONV = 0, HE_LAYER_FC = 1 };

/* he_pack_filters flags: which inverse transform the conv layer will use. */
enum {
    HE_PACK_CLASS_INTT = 0,  /* default: inverse transform only the extracted
                                residue classes (Sec. III-A: only the valid
                                slots need to be computed)                    */
    HE_PACK_FULL_INTT = 1    /* full-length inverse NTT of every c0^(n), then
                                extraction (Alg. 1 as printed)                */
};

typedef struct he_ctx he_ctx;
typedef struct he_layer he_layer;

typedef struct {
    int32_t kind;                                 /* HE_LAYER_CONV or HE_LAYER_FC */
    uint32_t c_i, c_o, H, W, f, stride, pad;      /* conv                         */
    uint32_t n_i, n_o;                            /* fc                           */
} he_layer_desc;

typedef struct {
    int32_t kind;
    uint32_t N, L;
    uint32_t s, g_i, g_o, K_in, K_out, H_p, W_p, H_o, W_o;   /* conv            */
    uint32_t n_o_p, n_i_p, blocks;                          /* fc              */
    uint32_t flags;                                         /* pack flags      */
    uint64_t resident_bytes;                                /* device operands */
} he_layer_info;

/*
 * he_setup -- create a context for ring degree N (a power of two, 256..16384),
 * L limbs (1..8) and plaintext modulus t (2 <= t < every q).
 * primes: L distinct primes q < 2^30 with q = 1 (mod 2N), or NULL for the L
 * largest such primes in descending order.  Builds the twiddle tables on the
 * current device.  (Sec. II-A ring R_Q and RNS/CRT of Sec. I; parameters of
 * Sec. IV-A are replaced by the exact-integer set.)
 * Returns HE_EINVAL for a bad parameter set, HE_EDEVICE / HE_ENOMEM on
 * device failures.  *out is set only on HE_OK.
 */
int he_setup(uint32_t N, uint32_t L, const uint32_t *primes, uint32_t t, he_ctx **out);

/* Parameters of a context: primes[L] and Delta mod q_l (delta_l[L]); either may be NULL. */
int he_ctx_params(const he_ctx *ctx, uint32_t *N, uint32_t *L, uint32_t *t,
                  uint32_t *primes, uint32_t *delta_l);

/*
 * he_pack_filters -- server initialisation of one layer (Alg. 1 / Alg. 2,
 * server initialisation and the precomputed transforms of Sec. IV-A-1):
 * pack the filters (conv) or weight matrix (fc), then keep the NTT-domain
 * products operands resident on the device.
 *   weights  host int8: conv [c_o][c_i][f][f]; fc [n_o][n_i]
 *   rho      host u32 masks, values < t: conv [K_in][c_o][N]; fc [blocks][N]
 *   bias     host int32 [n_o] (fc only; NULL = zero; must be NULL for conv)
 *   flags    HE_PACK_CLASS_INTT or HE_PACK_FULL_INTT (conv only)
 * Synchronises the device before returning.  The layer is owned by the
 * library until he_free_layer.
 */
int he_pack_filters(he_ctx *ctx, const he_layer_desc *desc, const int8_t *weights,
                    const uint32_t *rho, const int32_t *bias, uint32_t flags,
                    he_layer **out);

/* Tiling of a packed layer (the quantities in the comment at the top). */
int he_layer_info_get(const he_layer *layer, he_layer_info *out);

/*
 * he_layer_geometry -- the tiling of a layer description before any packing:
 * s, g_i, g_o, K_in, K_out, padded and output sizes for conv (Eq. k_batch_new
 * and Eq. i_batch generalised by the rule at the top), n_o', n_i', blocks for
 * FC (Eq. w(x) formula, Theorem 1), and the bytes the packed layer would keep
 * resident.  The same rule he_pack_filters applies, so callers size their
 * buffers from it instead of re-deriving it.  Allocates nothing and touches no
 * device.  flags as for he_pack_filters (ignored for FC).  HE_EINVAL for a
 * description the ring cannot hold, HE_EUNSUPPORTED for s > 256.
 */
int he_layer_geometry(const he_ctx *ctx, const he_layer_desc *desc, uint32_t flags, he_layer_info *out);

/* Bytes of device workspace a layer call with batch B needs (see *_ws calls). */
size_t he_layer_workspace_bytes(const he_layer *layer, uint32_t B);

/* Bytes of workspace he_encrypt_c0 and he_poly_mul need for `rows` polynomial rows. */
size_t he_ctx_workspace_bytes(const he_ctx *ctx, uint32_t rows);

/*
 * he_workspace_reserve -- make the context-owned workspace of `stream` at
 * least `bytes` bytes (he_layer_workspace_bytes / he_ctx_workspace_bytes give
 * the sizes), and give the stream the 64 KiB counter block that the one-launch
 * layer form needs (created zeroed on the first reservation; every launch
 * leaves it zero).  The calls that use a context workspace (he_conv_layer,
 * he_fc_layer, he_conv_layer_ntt, he_fc_layer_ntt, he_encrypt_c0,
 * he_poly_mul) never allocate: they fail with HE_ENOMEM, before any launch,
 * when the stream's reserved workspace is smaller than they need.  Growing a
 * workspace synchronises the device before the old buffer is freed; it must
 * not run while another host thread issues calls on the same stream.  Calls
 * on one stream share its workspace (they run in stream order); calls on
 * different streams need their own reservations.
 */
int he_workspace_reserve(he_ctx *ctx, void *stream, size_t bytes);

/*
 * he_sync_check -- HE_EDEVICE if a one-launch layer call that used the counter
 * block of `stream` (its he_workspace_reserve reservation) gave up a bounded
 * wait for a work item it depends on (its output words are then undefined;
 * the flag is cleared), else HE_OK.  Synchronises the stream.  Each wait
 * depends only on items that started earlier in the same launch, so a wait
 * ends unless the device stalls for about a second.
 */
int he_sync_check(he_ctx *ctx, void *stream);

/*
 * he_conv_layer -- server evaluation of one Conv layer for B images
 * (Alg. 1, server evaluation, and the extraction loops that follow it).
 *   d_c0       [B][K_in][L][N]  c0 shares, residues < q_l
 *   d_sh       [B][K_in][N]     server input share, values < t; NULL on a
 *                               network's first layer (no share to remove)
 *   d_sh_next  [B][K_out][N]    fresh server share sh', values < t; NULL on
 *                               the last layer
 *   d_out      [B][K_out][L][N] c0^r, residues < q_l
 * Uses the workspace reserved for `stream` (he_workspace_reserve; HE_ENOMEM
 * if it is smaller than he_layer_workspace_bytes(layer, B)); allocates nothing.
 */
int he_conv_layer(he_ctx *ctx, const he_layer *layer, uint32_t B,
                  const uint32_t *d_c0, const uint32_t *d_sh, const uint32_t *d_sh_next,
                  uint32_t *d_out, void *stream);

/* As he_conv_layer with a caller-owned device workspace of at least
 * he_layer_workspace_bytes(layer, B) bytes (256-byte aligned).  Allocates nothing. */
int he_conv_layer_ws(he_ctx *ctx, const he_layer *layer, uint32_t B,
                     const uint32_t *d_c0, const uint32_t *d_sh, const uint32_t *d_sh_next,
                     uint32_t *d_out, void *d_workspace, size_t workspace_bytes, void *stream);

/*
 * he_conv_layer_noalloc -- he_conv_layer for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  Same arguments and output words as he_conv_layer, but
 * the workspace is a static device array of HE_NOALLOC_SCRATCH_BYTES bytes
 * (one per GPU, held until the process ends, its address looked up once per
 * device by he_setup), so the call needs no he_workspace_reserve and calls no
 * allocator.  HE_ENOMEM, before any launch, when he_layer_workspace_bytes(
 * layer, B) exceeds HE_NOALLOC_SCRATCH_BYTES.  Every call on one GPU shares
 * that array and nothing in it is expected to start at any value: calls that
 * overlap on one GPU (two streams, two host threads, two contexts) race and
 * must be ordered by the caller.  Kernel timing (he_profile_*) does not see
 * this form's launches.
 */
#define HE_NOALLOC_SCRATCH_BYTES (32u << 20)
int he_conv_layer_noalloc(he_ctx *ctx, const he_layer *layer, uint32_t B,
                          const uint32_t *d_c0, const uint32_t *d_sh, const uint32_t *d_sh_next,
                          uint32_t *d_out, void *stream);

/*
 * he_fc_layer -- server evaluation of one FC layer for B inputs (Alg. 2,
 * server evaluation; Theorem 1 places output b n_o' + k at coefficient k of
 * block b).
 *   d_c0       [B][L][N]               c0 of the packed input (Eq. i(x) formula)
 *   d_sh       [B][N] values < t, or NULL
 *   d_sh_next  [B][blocks][n_o'] values < t, or NULL (last layer)
 *   d_out      [B][blocks][L][n_o']    first n_o' coefficients of c0^r per block
 */
int he_fc_layer(he_ctx *ctx, const he_layer *layer, uint32_t B,
                const uint32_t *d_c0, const uint32_t *d_sh, const uint32_t *d_sh_next,
                uint32_t *d_out, void *stream);

int he_fc_layer_ws(he_ctx *ctx, const he_layer *layer, uint32_t B,
                   const uint32_t *d_c0, const uint32_t *d_sh, const uint32_t *d_sh_next,
                   uint32_t *d_out, void *d_workspace, size_t workspace_bytes, void *stream);

/*
 * The same layer split at its NTT-domain inputs, as the paper's protocol runs
 * it (Sec. IV-A-1): the client obtains NTT(c0) during encryption and sends it;
 * the server computes NTT(sh) of its own share, which it can do as soon as it
 * draws the share, before the layer's c0 arrives.
 *
 * he_layer_inputs_ntt -- forward NTTs of c0 and/or sh (either may be NULL) of
 * B images into the layer's NTT-domain input buffer d_x [B][2 K_in][L][N]
 * (device, 16-byte aligned, caller-owned): c0 rows at [b][j], sh rows at
 * [b][K_in + j]; K_in = 1 for FC.  d_c0 and d_sh as for he_conv_layer /
 * he_fc_layer.  Rows not passed are left as they are.
 *
 * he_conv_layer_ntt / he_fc_layer_ntt -- the rest of the layer (MAC, inverse,
 * extraction, + Delta sh') from d_x; has_sh = 0 when the layer has no input
 * share (the sh rows of d_x are then not read).  d_sh_next, d_out as for
 * he_conv_layer / he_fc_layer.  Uses the workspace reserved for the stream.
 * he_conv_layer is he_layer_inputs_ntt followed by he_conv_layer_ntt (same words).
 */
int he_layer_inputs_ntt(he_ctx *ctx, const he_layer *layer, uint32_t B, const uint32_t *d_c0,
                        const uint32_t *d_sh, uint32_t *d_x, void *stream);
int he_conv_layer_ntt(he_ctx *ctx, const he_layer *layer, uint32_t B, const uint32_t *d_x, int has_sh,
                      const uint32_t *d_sh_next, uint32_t *d_out, void *stream);
int he_fc_layer_ntt(he_ctx *ctx, const he_layer *layer, uint32_t B, const uint32_t *d_x, int has_sh,
                    const uint32_t *d_sh_next, uint32_t *d_out, void *stream);

/*
 * Transform primitives on device polynomials, exposed for checking the ring
 * arithmetic (Sec. IV-A-1: products through NTTs and coefficient-wise
 * multiplications).  d_in / d_out: [rows][L][N] u32 residues < q_l; may alias.
 * The NTT-domain order is private to the library: only ntt followed by intt,
 * or he_poly_mul, have a defined meaning in coefficient form.
 */
int he_ntt_forward(he_ctx *ctx, uint32_t rows, const uint32_t *d_in, uint32_t *d_out, void *stream);
int he_ntt_inverse(he_ctx *ctx, uint32_t rows, const uint32_t *d_in, uint32_t *d_out, void *stream);
/* d_c[r] = d_a[r] * d_b[r] in Z_q[X]/(X^N + 1), per limb; [rows][L][N] each.
 * d_c must not alias d_a or d_b.  Uses the workspace reserved for the stream. */
int he_poly_mul(he_ctx *ctx, uint32_t rows, const uint32_t *d_a, const uint32_t *d_b,
                uint32_t *d_c, void *stream);

/*
 * Kernel timing (measurement aid).  While enabled for a kernel kind, every
 * launch of that kind made by the layer calls is bracketed by two HIP events
 * recorded on the call's stream.  he_profile_read synchronises on the recorded
 * events and returns the number of launches and their summed duration (ms)
 * since the last reset.  Kinds: HE_K_NTT_FWD, HE_K_MAC, HE_K_TAIL (residue-
 * class inverse + extraction), HE_K_INTT (full inverse + extraction),
 * HE_K_MAC_TAIL (MAC, residue-class inverse and extraction in one launch),
 * HE_K_LAYER (the whole layer in one launch: forward transforms, MAC, inverse
 * and extraction), HE_K_LAYER_ROWS (the same with one MAC + inverse item per
 * output row), HE_K_GROUP (a grouped launch, he_group_run; recorded on the
 * context of the group's first call), HE_K_MAC_MFMA (the batched MAC on the
 * matrix cores, HE_TUNE_MAC = 9).
 */
enum { HE_K_NTT_FWD = 1, HE_K_MAC = 2, HE_K_TAIL = 4, HE_K_INTT = 8, HE_K_MAC_TAIL = 16, HE_K_LAYER = 32,
       HE_K_LAYER_ROWS = 64, HE_K_GROUP = 128, HE_K_MAC_MFMA = 256 };
int he_profile_enable(he_ctx *ctx, uint32_t kind_mask);
int he_profile_read(he_ctx *ctx, uint32_t kind, uint64_t *launches, double *total_ms);
int he_profile_reset(he_ctx *ctx);

/*
 * Client role (the client side of Alg. 1 / Alg. 2 on the device).
 *
 * he_pack_operands -- a layer whose resident NTT-domain operands are two given
 * polynomial sets instead of (rho, -Delta fhat): a, b host u32 residues,
 * conv [K_in][c_o][L][N], fc [blocks][L][N], coefficient form, each below its
 * limb's prime (HE_EINVAL otherwise).  Calling he_conv_layer / he_fc_layer on
 * it with d_c0 = a per-limb input set X and d_sh = a [0, t) input set Y gives
 * sum_j X_j a_j + Y_j b_j with the same extraction.  With a = p1, b = p2
 * (the masks of the server initialisation) and X = v, Y = i this is the
 * client's c1^r (Alg. 1 / Alg. 2 client evaluation); pass d_sh_next = NULL.
 *
 * he_client_masks -- the client's layer of the same form built on the device
 * from a server layer (he_pack_filters) and the client's key and noise: p1 =
 * rho b + e1 and p2 = Delta (fhat + rho) + e2 for every (j, n) (Alg. 1 / Alg. 2
 * server initialisation), kept NTT-domain like he_pack_operands(p1, p2).  b:
 * device [L][N] residues (public key part); e1, e2: device int32, conv
 * [K_in][c_o][N], fc [blocks][N], small signed.  The server layer is only read.
 *
 * he_encrypt_c0 -- c0 of the encryption of -msg (Alg. 1 / Alg. 2 client
 * encryption, Eq. encryption negated): out[r] = -(v[r] b + Delta msg[r] + e0[r])
 * mod q_l.  v, e0: device int32 [rows][N] (small signed), b: device [L][N]
 * residues (public key part), msg: device [rows][N] values < t, out:
 * [rows][L][N].  With v = s, b = a, msg = 0, e0 = -e it is key generation
 * b = -a s + e (Sec. II-A).  Uses the workspace reserved for the stream.
 *
 * he_decrypt -- msg[r][k] = round(t x / Q) mod t, x the CRT lift of
 * x0[r][.][k] + x1[r][.][k] (x1 may be NULL): the scale-and-round of the share
 * sum (Alg. 1 / Alg. 2 last client line, Eq. decryption in the exact reading).
 * x0, x1: device [rows][L][M] residues; msg: [rows][M]; M <= N (0 means N),
 * e.g. M = n_o' for FC outputs.  Correct for share sums within Q/(4t) of
 * Delta times a message.
 */
int he_pack_operands(he_ctx *ctx, const he_layer_desc *desc, const uint32_t *a, const uint32_t *b,
                     uint32_t flags, he_layer **out);
int he_client_masks(he_ctx *ctx, const he_layer *server, const uint32_t *d_b, const int32_t *d_e1,
                    const int32_t *d_e2, he_layer **out);
int he_encrypt_c0(he_ctx *ctx, uint32_t rows, const int32_t *d_v, const uint32_t *d_b,
                  const uint32_t *d_msg, const int32_t *d_e0, uint32_t *d_out, void *stream);
int he_decrypt(he_ctx *ctx, uint32_t rows, uint32_t M, const uint32_t *d_x0, const uint32_t *d_x1,
               uint32_t *d_msg, void *stream);

/*
 * Layer sequences (runtime): an ordered list of layer calls with their device
 * buffers, run as one host call or captured once into a HIP graph and replayed.
 * Steps run in order on one stream and share one sequence-owned workspace, so a
 * sequence is for one stream at a time.  Buffers must stay valid while the
 * sequence exists.  Capture needs a non-null stream; no timing events are
 * recorded into the graph (the context's timing setting is left unchanged);
 * after capture no step can be added.
 */
typedef struct he_seq he_seq;
int he_seq_create(he_ctx *ctx, he_seq **out);
/* Append a conv or FC call (kind taken from the layer); arguments as he_conv_layer / he_fc_layer. */
int he_seq_add(he_seq *seq, const he_layer *layer, uint32_t B, const uint32_t *d_c0,
               const uint32_t *d_sh, const uint32_t *d_sh_next, uint32_t *d_out);
int he_seq_run(he_seq *seq, void *stream);
int he_seq_capture(he_seq *seq, void *stream);
int he_seq_replay(he_seq *seq, void *stream);
uint32_t he_seq_length(const he_seq *seq);
void he_seq_free(he_seq *seq);

/*
 * Grouped launch: independent layer calls -- any layers, contexts (ring
 * degrees, limb counts) and batch sizes on one device -- evaluated by ONE
 * kernel launch.  Each call is the server evaluation of he_conv_layer /
 * he_fc_layer (Alg. 1 / Alg. 2, with the NTT-domain products of Sec. IV-A-1)
 * and gives the same output words.  The launch walks a device-side list of
 * work items: forward-transform sub-blocks of every call, then MAC items
 * (image x channel tiles of one limb and slot range for batched conv calls,
 * so that a resident operand word is read once per tile of images), then the
 * residue-class inverse and extraction items; an item waits, through counters,
 * only for the items of its own call that it reads.
 *
 * he_layer_call: one call, arguments as he_conv_layer / he_fc_layer (the kind
 * is the layer's).  Conv layers must be packed in the residue-class form with
 * 2 <= s <= 256 and N/s <= 4096; FC layers need n_o' <= 1024; N is 4096,
 * 8192 or 16384 (HE_EUNSUPPORTED otherwise, naming the call).
 *
 * he_group_create -- plans the items, allocates the group's device job list,
 * workspace (he_layer_workspace_bytes of every call) and zeroed counters, and
 * uploads the list (synchronous).  The buffers of the calls are baked in: they
 * must stay valid, and keep their sizes, while the group exists.  flags:
 * HE_GROUP_MAC_AUTO (image tiles for conv calls of B >= 4), HE_GROUP_MAC_PER_IMAGE
 * (one image per MAC item), HE_GROUP_MAC_TILED (image tiles wherever the shape
 * allows).  *out = NULL on failure.
 * he_group_run -- one launch on `stream`, with the group's device current (as
 * for every layer call); allocates nothing (it may be captured into a HIP
 * graph).  The counters return to zero by the end of each launch; launches of
 * one group must not overlap (one stream at a time).
 * he_group_check -- synchronises the stream; HE_EDEVICE if an item of an earlier
 * launch gave up waiting (about a second; its call's words are then undefined;
 * the flag is cleared), else HE_OK.
 * he_group_items -- work items per phase (NTT, MAC, inverse), the number of
 * calls whose MAC runs in image tiles, and the workspace bytes.
 * he_group_tune -- the autotuner's knob of a group: the items of a phase go
 * to the 8 XCDs in chunks of 2^c consecutive items, round robin (neighbouring
 * items of one call share an L2; calls of different cost spread over every
 * XCD).  Times one launch per candidate c in 2..8 (median of three after a
 * warm-up, on `stream`, synchronising), keeps the fastest and returns it in
 * *chunk_log (may be NULL); the launches write the calls' outputs (the same
 * words each time).  Then as he_group_check.  Default before tuning: c = 6.
 * he_group_set_chunk -- sets c (0..10) directly.
 */
typedef struct {
    he_ctx *ctx;
    const he_layer *layer;
    uint32_t B;
    const uint32_t *d_c0, *d_sh, *d_sh_next;
    uint32_t *d_out;
} he_layer_call;
typedef struct he_group he_group;
enum { HE_GROUP_MAC_AUTO = 0, HE_GROUP_MAC_PER_IMAGE = 1, HE_GROUP_MAC_TILED = 2 };
int he_group_create(const he_layer_call *calls, uint32_t n, uint32_t flags, he_group **out);
int he_group_run(he_group *g, void *stream);
int he_group_check(he_group *g, void *stream);
int he_group_items(const he_group *g, uint32_t *items, uint32_t *tiled_jobs, size_t *workspace_bytes);
int he_group_tune(he_group *g, void *stream, uint32_t *chunk_log);
int he_group_set_chunk(he_group *g, uint32_t chunk_log);
void he_group_free(he_group *g);

/*
 * Serving runtime: continuous batching of layer requests (the server of Alg. 1
 * / Alg. 2 answering many clients).  Layers are registered once; a request
 * names a layer, its arrival time in seconds from the start of the run, and
 * resident device buffers laid out as for one image of he_conv_layer /
 * he_fc_layer (d_sh / d_sh_next may be NULL as there).  he_server_run replays
 * the time-ordered trace in real time: a generator thread submits each request
 * at its arrival time and a dispatcher thread admits the oldest pending
 * request whenever one of `streams` stream slots is free and its transient
 * memory (workspace, plus gather / scatter staging when batched) fits in the
 * free part of an hbm_budget_bytes pool allocated at creation; up to max_batch
 * pending requests of the same layer (and the same share pattern) ride along.
 * Batches on different slots run concurrently.  A request whose memory can
 * never fit fails with HE_ENOMEM; a request whose batch reports a device error
 * fails with HE_EDEVICE; timeout_s > 0 bounds the run.  Every request's output
 * words equal those of a lone layer call on its inputs.  streams = 1 and
 * max_batch = 1 give the plain first-come first-served one-request-per-launch
 * server.  Results: per request arrival, dispatch and completion times
 * (seconds), batch size and status.
 */
typedef struct he_server he_server;
typedef struct {
    uint32_t streams;            /* concurrent stream slots, 1..64                  */
    uint32_t max_batch;          /* requests of one layer per launch, 1..1024       */
    uint64_t hbm_budget_bytes;   /* pool for transient per-batch device memory      */
    double timeout_s;            /* abandon the run after this long (0: no limit)   */
} he_server_config;
int he_server_create(const he_server_config *cfg, he_server **out);
int he_server_add_layer(he_server *srv, he_ctx *ctx, const he_layer *layer, uint32_t *layer_id);
int he_server_add_request(he_server *srv, uint32_t layer_id, double arrival_s, const uint32_t *d_c0,
                          const uint32_t *d_sh, const uint32_t *d_sh_next, uint32_t *d_out);
/* As he_server_add_request, but the request is held until request `after` (an
 * index of an earlier added request, -1 for none) completes; it then arrives at
 * max(arrival_s, that completion time).  This models a client that issues its
 * next layer when the previous one returns.  If `after` fails, so does this. */
int he_server_add_request_after(he_server *srv, uint32_t layer_id, double arrival_s, int64_t after,
                                const uint32_t *d_c0, const uint32_t *d_sh, const uint32_t *d_sh_next,
                                uint32_t *d_out);
int he_server_run(he_server *srv);
uint32_t he_server_requests(const he_server *srv);
int he_server_results(const he_server *srv, double *arrival, double *dispatch, double *complete,
                      uint32_t *batch, int32_t *status);
void he_server_free(he_server *srv);

/*
 * Tuning.  Knobs: HE_TUNE_NTT_FWD / HE_TUNE_NTT_INV / HE_TUNE_TAIL take the
 * register radix log2 r in 2..5 (each thread keeps 2^r words and runs r stages
 * per LDS pass; 0 = automatic), HE_TUNE_MAC takes 0 (streaming per-image MAC),
 * 1 (register-blocked batched MAC), 2 (residue-class conv layers: MAC, inverse
 * and extraction fused, one workgroup per output row), 3 (residue-class conv
 * layers, B >= 2: LDS-staged batched MAC over image x channel tiles), 4 (as
 * 3, with neighbouring tiles on one XCD), 5 and 6 (as 3 and 4, each stage
 * moved from memory to LDS by DMA, three stages in flight), 7 (conv and FC:
 * the whole layer in one launch, forward transforms included, work items in
 * workgroup order that wait on counters), 8 (conv: one launch of whole-row
 * transforms and one MAC + inverse item per output row), 9 (residue-class conv
 * layers, B >= 2, c_o a multiple of 8, s >= 4 and N/s >= 16: the batched MAC on
 * the integer matrix cores, residues split into signed 8-bit digits whose
 * products are summed exactly; a tuner candidate) or -1 (automatic:
 * 7 for FC layers at B = 1 where the shape allows it (N 4096..16384,
 * n_o' <= 1024); for conv layers at B = 1, 2, except 0 for layers with
 * K_in >= 2 and at most 64 output rows K_out g_o L; 9 where that form is
 * allowed and B >= 8 with s >= 16, or B >= 32; otherwise at B >= 4, 5 for
 * residue-class layers and 1 for full-length ones).  The one-launch forms need
 * a counter block: the calls that use a reserved stream workspace,
 * he_conv_layer_noalloc, layer sequences and the server have one, a *_ws call
 * has one when its stream has a reservation; otherwise, and for a shape a
 * form does not allow, the automatic multi-launch form runs.  Every value
 * yields the same output words.
 * he_tune_force pins a knob for the whole context (tests
 * sweep all values with it).  he_autotune_layer tunes the knobs of one layer at
 * batch B one after another: each candidate is timed as a whole layer call on
 * scratch buffers (median of 5, caches evicted before each), and the fastest is
 * kept for later calls with that shape (at B = 1 the MAC form leaves the automatic
 * rule above only for a form at least 5 % faster).  Candidates are visible only to
 * the tuning thread while they are timed; the choices are published when tuning ends
 * (the MAC form is kept with the layer, per B).  It allocates and frees its scratch
 * (about 512 MiB plus one call's buffers) and synchronises the stream.
 * he_tune_get reads a kept transform choice back (key: knob, log2 of the transform
 * size, rows per launch); HE_EINVAL for HE_TUNE_MAC, whose choices live with layers.
 */
enum { HE_TUNE_NTT_FWD = 1, HE_TUNE_NTT_INV = 2, HE_TUNE_TAIL = 3, HE_TUNE_MAC = 4 };
int he_tune_force(he_ctx *ctx, uint32_t knob, int32_t value);
int he_autotune_layer(he_ctx *ctx, const he_layer *layer, uint32_t B, void *stream);
int he_tune_get(he_ctx *ctx, uint32_t knob, uint32_t key_size, uint32_t key_rows, int32_t *value);

/*
 * he_probe_rate -- measurement aid for the integer-ALU roofs: the whole chip's
 * throughput of one instruction mix with no memory traffic (eight 256-thread
 * workgroups per CU, 8 independent chains per thread, `iters` rounds).  Kinds:
 * HE_PROBE_BFLY / HE_PROBE_GSBFLY (the forward / inverse Shoup butterflies of
 * the NTT kernels, per butterfly), HE_PROBE_MAD64 (32x32 -> 64-bit
 * multiply-add of the MAC), HE_PROBE_ADD, HE_PROBE_MULLO, HE_PROBE_MULHI (one
 * 32-bit vector instruction each).  *ops_per_s: operations per second; *ms
 * (may be NULL): the timed launch.  Runs on the current device and the null
 * stream, synchronises.
 */
enum { HE_PROBE_BFLY = 1, HE_PROBE_GSBFLY = 2, HE_PROBE_MAD64 = 3, HE_PROBE_ADD = 4, HE_PROBE_MULLO = 5,
       HE_PROBE_MULHI = 6 };
int he_probe_rate(uint32_t kind, uint32_t iters, double *ops_per_s, double *ms);

void he_free_layer(he_layer *layer);
void he_free(he_ctx *ctx);
const char *he_strerror(int code);
/* Text of the last HIP error seen by the library (thread-local), or "". */
const char *he_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HE_H */
