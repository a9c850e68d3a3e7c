// Host side of the C ABI declared in include/he.h.
//
// Context: primes (rule: the L largest q < 2^30 with q = 1 mod 2N), a primitive
// 2N-th root psi per prime, Shoup twiddle tables in HBM ([L][N] words each),
// Delta = floor(Q / t) mod q_l computed without big integers as
// Delta = -(Q mod t) t^-1 (mod q_l), since q_l | Q.
// Layer: packed filters (Eq. k_batch_new generalised, or Eq. w(x) formula), then
// the NTT-domain operands kept resident: Op[n][l][J][N], J < K_in the masks
// rho_j^(n), J >= K_in the products -Delta fhat_j^(n), all times N^-1 and, in
// the residue-class form, times x_k^-o_n.

#include <hip/hip_runtime.h>

#include <chrono>
#include <functional>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <memory>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/he.h"
#include "he_internal.h"
#include "he_kernels.h"

// Workspace of he_conv_layer_noalloc: one array per device, alive until the process ends.  Host
// code never uses the name `scratch` as an address; it uses the per-device address that
// hipGetSymbolAddress returned when the first context was created on that device.
// The sync block of the one-launch layer form follows the workspace part (zero at load; every
// launch leaves it zero).
static __device__ __align__(256) uint8_t scratch[HE_NOALLOC_SCRATCH_BYTES + FZ_SYNC_WORDS * 4];

namespace {

thread_local std::string g_last_error;

int dev_fail(hipError_t e, const char *what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return HE_EDEVICE;
}

#define HE_HIP(call)                                              \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return dev_fail(e_, #call);         \
    } while (0)

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Look up the scratch array's address on `dev`, which must be the current device (once per device).
int scratch_bind(int dev) {
    if (dev < 0 || dev >= kMaxDevices) {
        g_last_error = "device index beyond " + std::to_string(kMaxDevices);
        return HE_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return HE_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return dev_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
    g_scratch_ptr[dev] = p;
    return HE_OK;
}

void *scratch_device_ptr(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[dev];
}

typedef unsigned __int128 u128;

uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }

uint64_t powmod(uint64_t a, uint64_t e, uint64_t m) {
    uint64_t r = 1 % m;
    a %= m;
    while (e) {
        if (e & 1) r = mulmod(r, a, m);
        a = mulmod(a, a, m);
        e >>= 1;
    }
    return r;
}

uint64_t invmod(uint64_t a, uint64_t p) { return powmod(a, p - 2, p); }   // p prime

bool is_prime_u64(uint64_t n) {
    if (n < 2) return false;
    static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (uint64_t p : bases)
        if (n % p == 0) return n == p;
    uint64_t d = n - 1;
    int r = 0;
    while ((d & 1) == 0) {
        d >>= 1;
        ++r;
    }
    for (uint64_t a : bases) {
        uint64_t x = powmod(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int i = 1; i < r; ++i) {
            x = mulmod(x, x, n);
            if (x == n - 1) {
                comp = false;
                break;
            }
        }
        if (comp) return false;
    }
    return true;
}

uint32_t bit_reverse(uint32_t x, int bits) {
    uint32_t r = 0;
    for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
    return r;
}

uint32_t shoup(uint32_t w, uint32_t q) { return (uint32_t)(((uint64_t)w << 32) / q); }

uint32_t log2u(uint32_t x) {
    uint32_t r = 0;
    while ((1u << r) < x) ++r;
    return r;
}

uint32_t pow2_floor(uint32_t x) {
    uint32_t r = 1;
    while ((r << 1) <= x) r <<= 1;
    return r;
}

struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
    uint32_t *sync = nullptr;   // zeroed counter block of the one-launch layer form (FZ_SYNC_WORDS words)
};

struct ProfRec {
    uint32_t kind;
    hipEvent_t start, stop;
};

}  // namespace

struct he_ctx {
    int device = 0;
    uint32_t N = 0, logN = 0, L = 0, t = 0;
    std::vector<uint32_t> primes, delta_l;
    LimbConsts lc;
    uint32_t *tw = nullptr, *twsh = nullptr, *twi = nullptr, *twish = nullptr, *xinv = nullptr;
    std::mutex mu;
    std::unordered_map<hipStream_t, Workspace> ws;
    uint32_t prof_mask = 0;
    std::vector<ProfRec> prof;
    // tuning: forced knob values (0 / -1 = automatic) and measured choices per launch shape
    DecConsts dc;
    int force_fwd = 0, force_inv = 0, force_tail = 0, force_mac = -1;
    std::map<std::tuple<int, uint32_t, uint32_t>, int> tuned;   // (knob, log size, rows) -> value
};

struct he_layer {
    he_ctx *ctx = nullptr;
    he_layer_info info;
    uint32_t *op = nullptr;        // [c_o or blocks][L][2 K_in][N]
    int32_t *bias = nullptr;       // fc: [blocks][n_o_p]
    uint32_t n_rows = 0;           // c_o (conv) or blocks (fc)
    // MAC form chosen by the autotuner per batch size (guarded by the context's mutex)
    mutable std::map<uint32_t, int> mac_choice;
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t layer_ws_bytes(const he_layer *ly, uint32_t B) {
    const he_layer_info &in = ly->info;
    const size_t N = in.N, L = in.L;
    if (in.kind == HE_LAYER_CONV) {
        const size_t xn = align256((size_t)B * 2 * in.K_in * L * N * 4);
        const size_t per = (in.flags == HE_PACK_FULL_INTT) ? N : N / in.s;
        return xn + align256((size_t)B * ly->n_rows * L * per * 4);
    }
    return align256((size_t)B * 2 * L * N * 4) + align256((size_t)B * in.blocks * L * N * 4);
}

// The workspace reserved for `st` (he_workspace_reserve); a call never allocates.  Fails with
// HE_ENOMEM, naming the bytes needed, when nothing or too little was reserved for the stream.
int ctx_workspace(he_ctx *ctx, hipStream_t st, size_t bytes, void **out, uint32_t **sync = nullptr) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->ws.find(st);
    if (it == ctx->ws.end() || it->second.bytes < bytes) {
        g_last_error = "workspace: " + std::to_string(bytes) + " bytes needed on this stream, " +
                       std::to_string(it == ctx->ws.end() ? 0 : it->second.bytes) +
                       " reserved (he_workspace_reserve, or pass a workspace to a *_ws call)";
        return HE_ENOMEM;
    }
    *out = it->second.ptr;
    if (sync) *sync = it->second.sync;
    return HE_OK;
}

// The sync block reserved for `st` (he_workspace_reserve), or null.
uint32_t *ctx_sync(he_ctx *ctx, hipStream_t st) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->ws.find(st);
    return it == ctx->ws.end() ? nullptr : it->second.sync;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Candidate knob values of a running autotune, visible only to the tuning thread, so that calls on
// other threads keep the published choices while candidates are timed.
struct TuneTrial {
    std::map<std::tuple<int, uint32_t, uint32_t>, int> knobs;
    const he_layer *mac_layer = nullptr;
    uint32_t mac_B = 0;
    int mac = -2;   // -2: none under trial
};
thread_local const TuneTrial *tl_trial = nullptr;
// Kernel timing is suppressed on this thread (autotune trials, graph capture).
thread_local bool tl_no_prof = false;

int knob(he_ctx *ctx, int which, uint32_t logsize, uint32_t rows) {
    const int forced = which == HE_TUNE_NTT_FWD ? ctx->force_fwd
                       : which == HE_TUNE_NTT_INV ? ctx->force_inv
                                                  : ctx->force_tail;
    if (forced > 0) return forced;
    const auto key = std::make_tuple(which, logsize, rows);
    if (tl_trial) {
        auto it = tl_trial->knobs.find(key);
        if (it != tl_trial->knobs.end()) return it->second;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->tuned.find(key);
    return it == ctx->tuned.end() ? 0 : it->second;
}

// The MAC form kept for this layer at batch B: a trial value of a running autotune on this thread,
// else the tuner's published choice, else -1 (automatic).
int mac_tuned(he_ctx *ctx, const he_layer *ly, uint32_t B) {
    if (tl_trial && tl_trial->mac != -2 && tl_trial->mac_layer == ly && tl_trial->mac_B == B) return tl_trial->mac;
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ly->mac_choice.find(B);
    return it == ly->mac_choice.end() ? -1 : it->second;
}

// Conv MAC variant of a layer at batch B: 0 streaming (then tail), 1 register-blocked
// batched (then tail), 2 fused MAC + residue-class tail, 3 LDS-staged batched (then tail),
// 4 as 3 with XCD-contiguous workgroup order, 5 and 6 as 3 and 4 with the stages moved to LDS
// by DMA, 9 on the matrix cores (then tail).  A tuned or forced value is used when the layer's
// shape allows it; otherwise, and by default, B = 1 takes the fused form (the streaming one for
// layers with K_in >= 2 and at most 64 output rows) and B >= 4 a batched one (9 where allowed
// from B = 8 with s >= 16 and from B = 32 at any s, else 5 for the residue-class form, 1 for
// the full-length form).
bool mac_tiled_ok(const he_layer *ly, uint32_t B) {
    const he_layer_info &in = ly->info;
    const bool cls = in.flags == HE_PACK_CLASS_INTT;
    return B >= 2 && (!cls || (in.s >= 2 && in.s <= 128));
}

bool mac_fused_ok(const he_ctx *ctx, const he_layer *ly) {
    const he_layer_info &in = ly->info;
    const uint32_t logm = ctx->logN - log2u(in.s);
    return in.kind == HE_LAYER_CONV && in.flags == HE_PACK_CLASS_INTT && logm >= 4 && in.s <= 256 && in.N >= 256;
}

bool mac_lds_ok(const he_layer *ly, uint32_t B) {
    const he_layer_info &in = ly->info;
    return B >= 2 && in.kind == HE_LAYER_CONV && in.flags == HE_PACK_CLASS_INTT && in.s >= 2 && in.N >= 256;
}

// the matrix-core batched MAC: residue-class conv layers with c_o a multiple of 8, s >= 4,
// N / s >= 16 and at most 32768 products in a block sum (2 K_in s, the input share included)
bool mac_mfma_layer_ok(const he_layer *ly, uint32_t B) {
    const he_layer_info &in = ly->info;
    return mac_lds_ok(ly, B) && mac_mfma_ok(B, ly->n_rows, 2 * in.K_in, in.N, in.s);
}

// The item geometry of this layer at batch B in the one-launch / grouped forms (kernels_fused.hip),
// before the plan, in f; false when the shape is outside them.
bool fused_layer_shape(const he_ctx *ctx, const he_layer *ly, uint32_t B, bool rows, FusedLayer &f) {
    const he_layer_info &in = ly->info;
    std::memset(&f, 0, sizeof(f));
    f.kind = in.kind == HE_LAYER_CONV ? FZ_KIND_CONV : FZ_KIND_FC;
    if (in.kind == HE_LAYER_CONV && in.flags != HE_PACK_CLASS_INTT) return false;
    f.B = B;
    f.K_in = in.K_in;
    f.Jtot = 2 * in.K_in;
    f.Juse = f.Jtot;
    f.rows = ly->n_rows;
    f.g_o = in.g_o;
    f.K_out = in.K_out;
    f.L = in.L;
    f.logN = ctx->logN;
    f.s_log = in.kind == HE_LAYER_CONV ? log2u(in.s) : 0;
    f.n_o_p = in.n_o_p;
    f.rows_form = rows ? 1u : 0u;
    if (!fused_layer_ok(f)) return false;
    f.ntt_c0 = f.ntt_sh = in.K_in;
    return true;
}

// The one-launch layer form for this layer at batch B: its item geometry in *jb when the shape
// allows it and its counters fit a sync block.  Its MAC reads the resident operands once per
// image, so the automatic rule keeps it for B = 1.
bool layer_one_launch_ok(const he_ctx *ctx, const he_layer *ly, uint32_t B, FusedLayer *jb, bool rows = false) {
    FusedLayer f;
    if (!fused_layer_shape(ctx, ly, B, rows, f)) return false;
    if (FZ_SB_HDR + fused_layer_plan(f) > FZ_SYNC_WORDS) return false;
    if (jb) *jb = f;
    return true;
}

// The multi-launch MAC form of a conv layer (values 0..6) for a forced or tuned value mk (-1:
// the automatic rule).
int mac_variant_multi(he_ctx *ctx, const he_layer *ly, uint32_t B, int mk) {
    const bool tiled_ok = mac_tiled_ok(ly, B), fused_ok = mac_fused_ok(ctx, ly);
    if (mk == 3 || mk == 4 || mk == 5 || mk == 6) return mac_lds_ok(ly, B) ? mk : 0;
    if (mk == 9) return mac_mfma_layer_ok(ly, B) ? 9 : 0;
    if (mk == 2) return fused_ok ? 2 : 0;
    if (mk == 1) return tiled_ok ? 1 : 0;
    if (mk == 0) return 0;
    if (B == 1 && fused_ok) {
        // a layer with several input polys and output rows for at most a quarter of the CUs
        // streams its MAC over many workgroups faster than the fused launch's few, even with
        // the tail as a second launch (what the autotuner picks for such layers)
        const he_layer_info &in = ly->info;
        return (in.K_in >= 2 && 4 * in.K_out * in.g_o * in.L <= 256) ? 0 : 2;
    }
    // the matrix-core form where it was measured faster without tuning: blocks of 16 slots and
    // more from B = 8, every block length from B = 32 (x1 / x2 / x4 stacks at B = 8, 16, 64)
    if (B >= 8 && mac_mfma_layer_ok(ly, B) && (ly->info.s >= 16 || B >= 32)) return 9;
    if (B >= 4 && mac_lds_ok(ly, B)) return 5;
    return tiled_ok && B >= 4 ? 1 : 0;
}

// The form of a layer call at batch B: 7 = the one-launch layer (conv or FC; by default for an FC
// layer at B = 1 when the shape allows it), 8 = the one-launch conv layer with one MAC + inverse
// item per output row, else the multi-launch MAC form of a conv layer (0..6), -1 for the
// multi-launch FC.  For conv layers at B = 1 the automatic rule keeps the multi-launch forms: a
// hand-over between workgroups inside a launch costs about as much as a launch boundary on this
// device, and the forward transforms slow down under the overlapped operand stream.
int mac_variant(he_ctx *ctx, const he_layer *ly, uint32_t B) {
    int mk = ctx->force_mac;
    if (mk < 0) mk = mac_tuned(ctx, ly, B);
    const bool conv = ly->info.kind == HE_LAYER_CONV;
    if (mk == 8 && layer_one_launch_ok(ctx, ly, B, nullptr, true)) return 8;
    if ((mk == 7 || mk == 8 || (mk < 0 && B == 1 && !conv)) && layer_one_launch_ok(ctx, ly, B, nullptr)) return 7;
    if (!conv) return -1;
    return mac_variant_multi(ctx, ly, B, (mk == 7 || mk == 8) ? -1 : mk);
}

// Times one kernel launch with dispatch-recorded events when profiling is on for its kind.
struct ProfScope {
    he_ctx *ctx;
    uint32_t kind;
    LaunchEv le;
    ProfScope(he_ctx *c, uint32_t k) : ctx(c), kind(k) {
        if ((ctx->prof_mask & kind) && !tl_no_prof) {
            if (hipEventCreate(&le.start) != hipSuccess || hipEventCreate(&le.stop) != hipSuccess)
                le.start = le.stop = nullptr;
        }
    }
    const LaunchEv *ev() const { return le.start ? &le : nullptr; }
    hipError_t done(hipError_t e) {
        if (le.start) {
            std::lock_guard<std::mutex> lk(ctx->mu);
            ctx->prof.push_back({kind, le.start, le.stop});
            le.start = le.stop = nullptr;
        }
        return e;
    }
};

}  // namespace


namespace {

// Tiling of a layer description (the rule in include/he.h); cls gets o_n per channel (conv).
int layer_geometry(const he_ctx *ctx, const he_layer_desc *desc, uint32_t flags, he_layer_info *info,
                   std::vector<uint32_t> *cls) {
    const uint32_t N = ctx->N;
    std::memset(info, 0, sizeof(*info));
    info->kind = desc->kind;
    info->N = N;
    info->L = ctx->L;
    if (desc->kind == HE_LAYER_CONV) {
        const uint32_t c_i = desc->c_i, c_o = desc->c_o, H = desc->H, W = desc->W, f = desc->f;
        if (!c_i || !c_o || !H || !W || !f || !desc->stride) return HE_EINVAL;
        const uint64_t Hp = (uint64_t)H + 2 * desc->pad, Wp = (uint64_t)W + 2 * desc->pad;
        if (f > Hp || f > Wp || Hp * Wp > N) return HE_EINVAL;
        const uint32_t s = pow2_floor((uint32_t)(N / (Hp * Wp)));
        if (s > 256) return HE_EUNSUPPORTED;
        info->s = s;
        info->g_i = c_i < s ? c_i : s;
        info->g_o = pow2_floor(c_o < s ? c_o : s);
        info->K_in = (c_i + info->g_i - 1) / info->g_i;
        info->K_out = (c_o + info->g_o - 1) / info->g_o;
        info->H_p = (uint32_t)Hp;
        info->W_p = (uint32_t)Wp;
        info->H_o = (uint32_t)((Hp - f) / desc->stride + 1);
        info->W_o = (uint32_t)((Wp - f) / desc->stride + 1);
        info->flags = flags;
        if (cls) {
            cls->resize(c_o);
            for (uint32_t n = 0; n < c_o; ++n) (*cls)[n] = (n % info->g_o) * (s / info->g_o);
        }
        return HE_OK;
    }
    if (desc->kind == HE_LAYER_FC) {
        const uint32_t n_i = desc->n_i, n_o = desc->n_o;
        if (!n_i || !n_o || n_i > N) return HE_EINVAL;
        uint32_t nop = 1;
        while (nop < n_o) nop <<= 1;
        if ((uint64_t)n_i * nop > N) nop = pow2_floor(N / n_i);
        info->n_o_p = nop;
        info->n_i_p = N / nop;
        info->blocks = (n_o + nop - 1) / nop;
        info->K_in = 1;
        info->flags = HE_PACK_FULL_INTT;
        return HE_OK;
    }
    return HE_EINVAL;
}

}  // namespace

// Library-internal: suppress kernel timing on the calling thread (graph capture); returns the
// previous setting.
__attribute__((visibility("hidden"))) bool he_prof_suppress(bool on) {
    const bool was = tl_no_prof;
    tl_no_prof = on;
    return was;
}

extern "C" {

const char *he_strerror(int code) {
    switch (code) {
        case HE_OK: return "ok";
        case HE_EINVAL: return "invalid argument";
        case HE_EUNSUPPORTED: return "unsupported";
        case HE_ENOMEM: return "out of memory";
        case HE_EDEVICE: return "device error";
        default: return "unknown error";
    }
}

const char *he_last_error(void) { return g_last_error.c_str(); }

int he_setup(uint32_t N, uint32_t L, const uint32_t *primes, uint32_t t, he_ctx **out) {
    if (!out) return HE_EINVAL;
    if (N < 256 || N > 16384 || (N & (N - 1))) return HE_EINVAL;
    if (L < 1 || L > HE_MAX_LIMBS) return HE_EINVAL;
    if (t < 2) return HE_EINVAL;
    std::vector<uint32_t> ps;
    if (primes) {
        for (uint32_t l = 0; l < L; ++l) {
            const uint32_t q = primes[l];
            if (q >= (1u << 30) || q % (2 * N) != 1 || !is_prime_u64(q) || t >= q) return HE_EINVAL;
            for (uint32_t p : ps)
                if (p == q) return HE_EINVAL;
            ps.push_back(q);
        }
    } else {
        uint64_t q = (((1ull << 30) - 1) / (2 * N)) * (2 * N) + 1;
        if (q >= (1ull << 30)) q -= 2 * N;
        while (ps.size() < L && q > 2 * N) {
            if (is_prime_u64(q)) ps.push_back((uint32_t)q);
            q -= 2 * N;
        }
        if (ps.size() < L) return HE_EINVAL;
        for (uint32_t p : ps)
            if (t >= p) return HE_EINVAL;
    }
    he_ctx *ctx = new (std::nothrow) he_ctx();
    if (!ctx) return HE_ENOMEM;
    hipGetDevice(&ctx->device);
    {
        const int src = scratch_bind(ctx->device);
        if (src != HE_OK) {
            delete ctx;
            return src;
        }
    }
    ctx->N = N;
    ctx->logN = log2u(N);
    ctx->L = L;
    ctx->t = t;
    ctx->primes = ps;
    std::memset(&ctx->lc, 0, sizeof(ctx->lc));
    uint64_t Qmodt = 1;
    for (uint32_t q : ps) Qmodt = Qmodt * (q % t) % t;
    std::vector<uint32_t> h_tw((size_t)L * N), h_twsh((size_t)L * N), h_twi((size_t)L * N), h_twish((size_t)L * N),
        h_xinv((size_t)L * N);
    const int bits = (int)ctx->logN;
    for (uint32_t l = 0; l < L; ++l) {
        const uint32_t q = ps[l];
        // primitive 2N-th root: g^((q-1)/2N) with psi^N = -1
        uint64_t psi = 0;
        for (uint64_t g = 2; g < q; ++g) {
            const uint64_t c = powmod(g, (q - 1) / (2 * N), q);
            if (powmod(c, N, q) == q - 1) {
                psi = c;
                break;
            }
        }
        if (!psi) {
            delete ctx;
            return HE_EINVAL;
        }
        const uint64_t psi_inv = invmod(psi, q);
        for (uint32_t i = 0; i < N; ++i) {
            const uint32_t e = bit_reverse(i, bits);
            const uint32_t w = (uint32_t)powmod(psi, e, q);
            const uint32_t wi = (uint32_t)powmod(psi_inv, e, q);
            h_tw[(size_t)l * N + i] = w;
            h_twsh[(size_t)l * N + i] = shoup(w, q);
            h_twi[(size_t)l * N + i] = wi;
            h_twish[(size_t)l * N + i] = shoup(wi, q);
            // x_k^-1 with x_k = psi^(2 brv(k) + 1), the k-th evaluation point
            h_xinv[(size_t)l * N + i] = (uint32_t)powmod(psi_inv, 2ull * e + 1, q);
        }
        LimbConst &c = ctx->lc.l[l];
        c.q = q;
        c.q2 = 2 * q;
        const uint64_t dl = (q - mulmod(Qmodt % q, invmod(t % q, q), q)) % q;   // floor(Q/t) mod q
        c.delta = (uint32_t)dl;
        c.delta_sh = shoup(c.delta, q);
        c.r32 = (uint32_t)((1ull << 32) % q);
        c.r32_sh = shoup(c.r32, q);
        c.bar = (uint32_t)((1ull << 32) / q);
        c.ninv = (uint32_t)invmod(N, q);
        c.ninv_sh = shoup(c.ninv, q);
        c.t_mod = t;
        ctx->delta_l.push_back(c.delta);
    }
    // decryption: (Q / q_l)^-1 mod q_l
    std::memset(&ctx->dc, 0, sizeof(ctx->dc));
    ctx->dc.t = t;
    for (uint32_t l = 0; l < L; ++l) {
        uint64_t prod = 1;
        for (uint32_t k = 0; k < L; ++k)
            if (k != l) prod = mulmod(prod, ps[k] % ps[l], ps[l]);
        ctx->dc.inv[l] = (uint32_t)invmod(prod, ps[l]);
        ctx->dc.inv_sh[l] = shoup(ctx->dc.inv[l], ps[l]);
    }
    const size_t bytes = (size_t)L * N * 4;
    uint32_t **bufs[5] = {&ctx->tw, &ctx->twsh, &ctx->twi, &ctx->twish, &ctx->xinv};
    std::vector<uint32_t> *hosts[5] = {&h_tw, &h_twsh, &h_twi, &h_twish, &h_xinv};
    for (int i = 0; i < 5; ++i) {
        hipError_t e = hipMalloc((void **)bufs[i], bytes);
        if (e == hipSuccess) e = hipMemcpy(*bufs[i], hosts[i]->data(), bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            he_free(ctx);
            return dev_fail(e, "he_setup tables");
        }
    }
    *out = ctx;
    return HE_OK;
}

int he_ctx_params(const he_ctx *ctx, uint32_t *N, uint32_t *L, uint32_t *t, uint32_t *primes, uint32_t *delta_l) {
    if (!ctx) return HE_EINVAL;
    if (N) *N = ctx->N;
    if (L) *L = ctx->L;
    if (t) *t = ctx->t;
    for (uint32_t l = 0; l < ctx->L; ++l) {
        if (primes) primes[l] = ctx->primes[l];
        if (delta_l) delta_l[l] = ctx->delta_l[l];
    }
    return HE_OK;
}

int he_tune_force(he_ctx *ctx, uint32_t which, int32_t value) {
    if (!ctx) return HE_EINVAL;
    switch (which) {
        case HE_TUNE_NTT_FWD: ctx->force_fwd = value; break;
        case HE_TUNE_NTT_INV: ctx->force_inv = value; break;
        case HE_TUNE_TAIL: ctx->force_tail = value; break;
        case HE_TUNE_MAC: ctx->force_mac = value; break;
        default: return HE_EINVAL;
    }
    return HE_OK;
}


int he_autotune_layer(he_ctx *ctx, const he_layer *ly, uint32_t B, void *stream) {
    if (!ctx || !ly || ly->ctx != ctx || B == 0) return HE_EINVAL;
    const he_layer_info &in = ly->info;
    hipStream_t st = (hipStream_t)stream;
    const uint32_t logN = ctx->logN, N = in.N, L = in.L;
    const bool conv = in.kind == HE_LAYER_CONV;
    // Scratch inputs, outputs and workspace of one call at batch B, plus a buffer whose
    // rewrite before every timed call evicts L2 and the last-level cache, so each
    // candidate is timed as a whole layer call from cold memory, as in a stream of
    // layers whose operands do not stay cached.  The words are zeros: no timing and no
    // kernel's addressing depends on the values.
    const size_t c0_b = align256((conv ? (size_t)B * in.K_in : (size_t)B) * L * N * 4);
    const size_t sh_b = align256((conv ? (size_t)B * in.K_in : (size_t)B) * N * 4);
    const size_t shn_b = align256(conv ? (size_t)B * in.K_out * N * 4 : (size_t)B * in.blocks * in.n_o_p * 4);
    const size_t out_b = align256(conv ? (size_t)B * in.K_out * L * N * 4 : (size_t)B * in.blocks * L * in.n_o_p * 4);
    const size_t ws_b = align256(layer_ws_bytes(ly, B));
    const size_t flush_b = (size_t)512 << 20;
    const size_t sync_b = (size_t)FZ_SYNC_WORDS * 4;   // the trials' own counter block (zeroed below)
    const size_t data_b = c0_b + sh_b + shn_b + out_b + ws_b + sync_b;
    char *buf = nullptr;
    if (hipMalloc((void **)&buf, data_b + flush_b) != hipSuccess) return HE_ENOMEM;
    const uint32_t *c0 = (const uint32_t *)buf;
    const uint32_t *sh = (const uint32_t *)(buf + c0_b);
    const uint32_t *shn = (const uint32_t *)(buf + c0_b + sh_b);
    uint32_t *out = (uint32_t *)(buf + c0_b + sh_b + shn_b);
    void *ws = buf + c0_b + sh_b + shn_b + out_b;
    uint32_t *tsync = (uint32_t *)(buf + c0_b + sh_b + shn_b + out_b + ws_b);
    char *flush = buf + data_b;
    hipEvent_t ea = nullptr, eb = nullptr;
    int rc = HE_OK;
    if (hipMemsetAsync(buf, 0, data_b, st) != hipSuccess || hipEventCreate(&ea) != hipSuccess ||
        hipEventCreate(&eb) != hipSuccess)
        rc = HE_EDEVICE;
    // candidates are set on this thread only; the choices are published once at the end
    TuneTrial trial;
    const TuneTrial *saved_trial = tl_trial;
    const bool saved_noprof = tl_no_prof;
    tl_trial = &trial;
    tl_no_prof = true;

    // median duration (ms) of one layer call after one untimed call
    auto time_layer = [&](bool with_sh, double *ms_out) -> int {
        constexpr int REPS = 5;
        float ms[REPS];
        for (int r = -1; r < REPS; ++r) {
            if (hipMemsetAsync(flush, r & 0xff, flush_b, st) != hipSuccess) return HE_EDEVICE;
            if (hipEventRecord(ea, st) != hipSuccess) return HE_EDEVICE;
            const int lrc = he_layer_call_sync(ctx, ly, B, c0, with_sh ? sh : nullptr, shn, out, ws, ws_b, tsync, st);
            if (lrc != HE_OK) return lrc;
            if (hipEventRecord(eb, st) != hipSuccess || hipEventSynchronize(eb) != hipSuccess) return HE_EDEVICE;
            if (r >= 0 && hipEventElapsedTime(&ms[r], ea, eb) != hipSuccess) return HE_EDEVICE;
        }
        std::sort(ms, ms + REPS);
        *ms_out = ms[REPS / 2];
        return HE_OK;
    };
    // try every candidate of one knob with the others at their current values; keep the fastest
    // (pref: a candidate kept unless another is faster by more than `margin` of its time).
    // set(c) puts candidate c under trial.
    auto pick = [&](const std::function<void(int)> &set, const std::vector<int> &cands, bool with_sh, int *chosen,
                    int pref = -1000, double margin = 0.0) -> int {
        double best = 1e30, pref_ms = -1.0;
        int arg = cands[0];
        for (int c : cands) {
            set(c);
            double ms = 0;
            const int r = time_layer(with_sh, &ms);
            if (r != HE_OK) return r;
            if (c == pref) pref_ms = ms;
            if (ms < best) {
                best = ms;
                arg = c;
            }
        }
        if (pref_ms >= 0.0 && best > pref_ms * (1.0 - margin)) arg = pref;
        set(arg);
        *chosen = arg;
        return HE_OK;
    };
    auto knob_setter = [&](int which, uint32_t key_size, uint32_t key_rows) {
        return std::function<void(int)>([&trial, which, key_size, key_rows](int c) {
            trial.knobs[std::make_tuple(which, key_size, key_rows)] = c;
        });
    };
    int chosen = 0;
    const std::vector<int> radix{2, 3, 4, 5};
    const uint32_t fwd_rows = (conv ? B * in.K_in : B) * L;
    // the forward launch's radix is timed under a multi-launch form (a one-launch layer has its own
    // forward items); a network's first layer has no input share: its forward launch has half the rows
    trial.mac_layer = ly;
    trial.mac_B = B;
    trial.mac = conv ? mac_variant_multi(ctx, ly, B, -1) : 0;
    if (rc == HE_OK) rc = pick(knob_setter(HE_TUNE_NTT_FWD, logN, fwd_rows), radix, false, &chosen);
    if (rc == HE_OK) rc = pick(knob_setter(HE_TUNE_NTT_FWD, logN, 2 * fwd_rows), radix, true, &chosen);
    trial.mac = -2;
    bool mac_done = false;
    int mac_pick = -1;
    if (conv) {
        const bool cls = in.flags == HE_PACK_CLASS_INTT;
        // every form the shape allows.  At batch one the candidates are the fused launch and the
        // streaming MAC then the tail; mac_variant's fixed rule (streaming for layers with several
        // input polys and few output rows) is kept unless the other form is 5 % faster, so that
        // layers timing cannot separate keep the rule's form
        std::vector<int> macs{0};
        if (mac_tiled_ok(ly, B)) macs.push_back(1);
        if (mac_fused_ok(ctx, ly)) macs.push_back(2);
        if (mac_lds_ok(ly, B))
            for (int m : {3, 4, 5, 6}) macs.push_back(m);
        if (mac_mfma_layer_ok(ly, B)) macs.push_back(9);
        if (layer_one_launch_ok(ctx, ly, B, nullptr)) macs.push_back(7);
        if (layer_one_launch_ok(ctx, ly, B, nullptr, true)) macs.push_back(8);
        trial.mac_layer = ly;
        trial.mac_B = B;
        trial.mac = -1;   // the automatic rule while the other knobs are tuned
        const uint32_t logm = logN - log2u(in.s);
        const uint32_t rows = B * in.K_out * in.g_o * L;
        // the tail's radix first, timed under a two-launch MAC form (the fused launch has its own
        // inverse), so that the MAC forms below are compared against a tuned tail; its key is
        // shared by the layers of one shape, and the first of them would otherwise see the default
        if (rc == HE_OK && cls && logm >= 4) {
            const int mv = mac_variant(ctx, ly, B);
            if (mv == 2 || mv == 7 || mv == 8) trial.mac = 0;
            rc = pick(knob_setter(HE_TUNE_TAIL, logm, rows), radix, true, &chosen);
            trial.mac = -1;
        }
        const int mac_pref = (B == 1 && macs.size() > 1) ? mac_variant(ctx, ly, B) : -1000;   // the rule's form
        if (rc == HE_OK && macs.size() > 1) {
            rc = pick([&trial](int c) { trial.mac = c; }, macs, true, &mac_pick, mac_pref, 0.05);
            mac_done = rc == HE_OK;
        }
        if (rc == HE_OK && !cls) rc = pick(knob_setter(HE_TUNE_NTT_INV, logN, rows), radix, true, &chosen);
    } else if (rc == HE_OK) {
        // FC: the multi-launch form's inverse radix, then that form against the one-launch form
        trial.mac_layer = ly;
        trial.mac_B = B;
        trial.mac = 0;
        rc = pick(knob_setter(HE_TUNE_NTT_INV, logN, B * in.blocks * L), radix, true, &chosen);
        if (rc == HE_OK && layer_one_launch_ok(ctx, ly, B, nullptr)) {
            trial.mac = -1;
            const int pref = mac_variant(ctx, ly, B) == 7 ? 7 : 0;
            rc = pick([&trial](int c) { trial.mac = c; }, std::vector<int>{0, 7}, true, &mac_pick, pref, 0.05);
            mac_done = rc == HE_OK;
        }
    }
    tl_trial = saved_trial;
    tl_no_prof = saved_noprof;
    if (rc == HE_OK) {
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (const auto &kv : trial.knobs) ctx->tuned[kv.first] = kv.second;
        if (mac_done) ly->mac_choice[B] = mac_pick;
    }
    hipStreamSynchronize(st);
    if (ea) hipEventDestroy(ea);
    if (eb) hipEventDestroy(eb);
    hipFree(buf);
    return rc;
}

int he_tune_get(he_ctx *ctx, uint32_t which, uint32_t key_size, uint32_t key_rows, int32_t *value) {
    if (!ctx || !value) return HE_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->tuned.find(std::make_tuple((int)which, key_size, key_rows));
    if (it == ctx->tuned.end()) return HE_EINVAL;
    *value = it->second;
    return HE_OK;
}

int he_profile_enable(he_ctx *ctx, uint32_t kind_mask) {
    if (!ctx) return HE_EINVAL;
    ctx->prof_mask = kind_mask;
    return HE_OK;
}

int he_profile_read(he_ctx *ctx, uint32_t kind, uint64_t *launches, double *total_ms) {
    if (!ctx) return HE_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    uint64_t n = 0;
    double tot = 0.0;
    for (const ProfRec &r : ctx->prof) {
        if (r.kind != kind) continue;
        HE_HIP(hipEventSynchronize(r.stop));
        float ms = 0.f;
        HE_HIP(hipEventElapsedTime(&ms, r.start, r.stop));
        tot += ms;
        ++n;
    }
    if (launches) *launches = n;
    if (total_ms) *total_ms = tot;
    return HE_OK;
}

int he_profile_reset(he_ctx *ctx) {
    if (!ctx) return HE_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (const ProfRec &r : ctx->prof) {
        hipEventSynchronize(r.stop);
        hipEventDestroy(r.start);
        hipEventDestroy(r.stop);
    }
    ctx->prof.clear();
    return HE_OK;
}

void he_free(he_ctx *ctx) {
    if (!ctx) return;
    he_profile_reset(ctx);
    hipFree(ctx->tw);
    hipFree(ctx->twsh);
    hipFree(ctx->twi);
    hipFree(ctx->twish);
    hipFree(ctx->xinv);
    for (auto &kv : ctx->ws) {
        if (kv.second.ptr) hipFree(kv.second.ptr);
        if (kv.second.sync) hipFree(kv.second.sync);
    }
    delete ctx;
}

void he_free_layer(he_layer *ly) {
    if (!ly) return;
    hipFree(ly->op);
    hipFree(ly->bias);
    delete ly;
}

int he_layer_info_get(const he_layer *ly, he_layer_info *out) {
    if (!ly || !out) return HE_EINVAL;
    *out = ly->info;
    return HE_OK;
}

size_t he_layer_workspace_bytes(const he_layer *ly, uint32_t B) { return ly ? layer_ws_bytes(ly, B) : 0; }

int he_layer_geometry(const he_ctx *ctx, const he_layer_desc *desc, uint32_t flags, he_layer_info *out) {
    if (!ctx || !desc || !out) return HE_EINVAL;
    if (flags != HE_PACK_CLASS_INTT && flags != HE_PACK_FULL_INTT) return HE_EINVAL;
    he_layer_info info;
    const int rc = layer_geometry(ctx, desc, flags, &info, nullptr);
    if (rc != HE_OK) return rc;
    const uint64_t rows = desc->kind == HE_LAYER_CONV ? desc->c_o : info.blocks;
    info.resident_bytes = rows * ctx->L * 2ull * info.K_in * ctx->N * 4 +
                          (desc->kind == HE_LAYER_FC ? (uint64_t)info.blocks * info.n_o_p * 4 : 0);
    *out = info;
    return HE_OK;
}

size_t he_ctx_workspace_bytes(const he_ctx *ctx, uint32_t rows) {
    if (!ctx) return 0;
    const size_t poly = align256((size_t)rows * ctx->L * ctx->N * 4);
    const size_t enc = poly + align256((size_t)ctx->L * ctx->N * 4);   // he_encrypt_c0: v rows + NTT(b)
    const size_t mul = 2 * poly;                                        // he_poly_mul: both transforms
    return enc > mul ? enc : mul;
}

int he_sync_check(he_ctx *ctx, void *stream) {
    if (!ctx) return HE_EINVAL;
    uint32_t *sync = ctx_sync(ctx, (hipStream_t)stream);
    if (!sync) return HE_OK;
    HE_HIP(hipStreamSynchronize((hipStream_t)stream));
    uint32_t err = 0;
    HE_HIP(hipMemcpy(&err, sync + FZ_SB_ERR, 4, hipMemcpyDeviceToHost));
    if (err == 0) return HE_OK;
    HE_HIP(hipMemset(sync + FZ_SB_ERR, 0, 4));
    g_last_error = "a one-launch layer call on this stream gave up waiting for an item it depends on";
    return HE_EDEVICE;
}

int he_workspace_reserve(he_ctx *ctx, void *stream, size_t bytes) {
    if (!ctx) return HE_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(ctx->mu);
    Workspace &w = ctx->ws[st];
    if (!w.sync) {
        // counters of the one-launch layer form: zero now, and zero again after every launch
        hipError_t e = hipMalloc((void **)&w.sync, (size_t)FZ_SYNC_WORDS * 4);
        if (e == hipSuccess) e = hipMemset(w.sync, 0, (size_t)FZ_SYNC_WORDS * 4);
        if (e != hipSuccess) {
            if (w.sync) hipFree(w.sync);
            w.sync = nullptr;
            g_last_error = std::string("sync block: ") + hipGetErrorString(e);
            return HE_ENOMEM;
        }
    }
    if (w.bytes >= bytes) return HE_OK;
    // the old buffer may still be read by work queued on any stream: let it drain first
    if (w.ptr) {
        HE_HIP(hipDeviceSynchronize());
        HE_HIP(hipFree(w.ptr));
    }
    w.ptr = nullptr;
    w.bytes = 0;
    const size_t want = align256(bytes > 0 ? bytes : 256);
    hipError_t e = hipMalloc(&w.ptr, want);
    if (e != hipSuccess) {
        w.ptr = nullptr;
        g_last_error = std::string("workspace hipMalloc: ") + hipGetErrorString(e);
        return HE_ENOMEM;
    }
    w.bytes = want;
    return HE_OK;
}

int he_pack_filters(he_ctx *ctx, const he_layer_desc *desc, const int8_t *weights, const uint32_t *rho,
                    const int32_t *bias, uint32_t flags, he_layer **out) {
    if (!ctx || !desc || !weights || !rho || !out) return HE_EINVAL;
    if (flags != HE_PACK_CLASS_INTT && flags != HE_PACK_FULL_INTT) return HE_EINVAL;
    const uint32_t N = ctx->N, L = ctx->L;
    he_layer_info info;
    std::vector<uint32_t> cls;
    if (desc->kind == HE_LAYER_CONV && bias) return HE_EINVAL;
    int grc = layer_geometry(ctx, desc, flags, &info, &cls);
    if (grc != HE_OK) return grc;
    uint32_t K_in = 0, n_rows = 0;
    std::vector<int16_t> fh;   // [K_in][n_rows][N]
    std::vector<int32_t> hbias;
    if (desc->kind == HE_LAYER_CONV) {
        const uint32_t c_i = desc->c_i, c_o = desc->c_o, f = desc->f;
        const uint32_t s = info.s;
        const uint64_t Wp = info.W_p;
        K_in = info.K_in;
        n_rows = c_o;
        fh.assign((size_t)K_in * c_o * N, 0);
        for (uint32_t n = 0; n < c_o; ++n) {
            const int64_t o_n = cls[n];
            for (uint32_t m = 0; m < c_i; ++m) {
                const uint32_t j = m / info.g_i, mp = m % info.g_i;
                for (uint32_t ky = 0; ky < f; ++ky)
                    for (uint32_t kx = 0; kx < f; ++kx) {
                        const int32_t w = weights[(((size_t)n * c_i + m) * f + ky) * f + kx];
                        const int64_t e = o_n - (int64_t)s * (ky * Wp + kx) - mp;
                        int16_t &dst = fh[((size_t)j * c_o + n) * N + (size_t)(e >= 0 ? e : N + e)];
                        dst = (int16_t)(dst + (e >= 0 ? w : -w));
                    }
            }
        }
    } else {
        const uint32_t n_i = desc->n_i, n_o = desc->n_o;
        const uint32_t nop = info.n_o_p;
        K_in = 1;
        n_rows = info.blocks;
        fh.assign((size_t)info.blocks * N, 0);
        hbias.assign((size_t)info.blocks * nop, 0);
        // Eq. (w(x) formula) per block: w_b = sum_k W_{k,0} X^k - sum_k sum_{l>=1} W_{k, n_i'-l} X^(l n_o' + k)
        for (uint32_t b = 0; b < info.blocks; ++b)
            for (uint32_t k = 0; k < nop; ++k) {
                const uint32_t row = b * nop + k;
                if (row >= n_o) continue;
                for (uint32_t col = 0; col < n_i; ++col) {
                    const int32_t w = weights[(size_t)row * n_i + col];
                    if (col == 0)
                        fh[(size_t)b * N + k] = (int16_t)w;
                    else
                        fh[(size_t)b * N + (size_t)(info.n_i_p - col) * nop + k] = (int16_t)(-w);
                }
                if (bias) hbias[(size_t)b * nop + k] = bias[row];
            }
    }

    he_layer *ly = new (std::nothrow) he_layer();
    if (!ly) return HE_ENOMEM;
    ly->ctx = ctx;
    ly->n_rows = n_rows;
    const uint32_t Jtot = 2 * K_in;
    const size_t op_words = (size_t)n_rows * L * Jtot * N;
    info.resident_bytes = op_words * 4 + hbias.size() * 4;
    ly->info = info;

    uint32_t *d_rho = nullptr, *d_cls = nullptr;
    int16_t *d_fh = nullptr;
    auto fail = [&](hipError_t e, const char *what) {
        hipFree(d_rho);
        hipFree(d_fh);
        hipFree(d_cls);
        he_free_layer(ly);
        return dev_fail(e, what);
    };
    hipError_t e;
    const size_t rho_words = (size_t)K_in * n_rows * N;
    if ((e = hipMalloc((void **)&ly->op, op_words * 4)) != hipSuccess) {
        he_free_layer(ly);
        g_last_error = "layer operands: out of device memory";
        return HE_ENOMEM;
    }
    if ((e = hipMalloc((void **)&d_rho, rho_words * 4)) != hipSuccess) return fail(e, "pack rho");
    if ((e = hipMalloc((void **)&d_fh, fh.size() * 2)) != hipSuccess) return fail(e, "pack fhat");
    if ((e = hipMemcpy(d_rho, rho, rho_words * 4, hipMemcpyHostToDevice)) != hipSuccess) return fail(e, "pack rho copy");
    if ((e = hipMemcpy(d_fh, fh.data(), fh.size() * 2, hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e, "pack fhat copy");
    if (!hbias.empty()) {
        if ((e = hipMalloc((void **)&ly->bias, hbias.size() * 4)) != hipSuccess) return fail(e, "pack bias");
        if ((e = hipMemcpy(ly->bias, hbias.data(), hbias.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
            return fail(e, "pack bias copy");
    }
    if (desc->kind == HE_LAYER_CONV && flags == HE_PACK_CLASS_INTT) {
        if ((e = hipMalloc((void **)&d_cls, cls.size() * 4)) != hipSuccess) return fail(e, "pack cls");
        if ((e = hipMemcpy(d_cls, cls.data(), cls.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
            return fail(e, "pack cls copy");
    }
    hipStream_t st = nullptr;
    if ((e = launch_expand_operands(d_rho, d_fh, ly->op, K_in, n_rows, L, N, ctx->lc, st)) != hipSuccess)
        return fail(e, "expand");
    RowMap m;
    m.J = Jtot;
    m.L = L;
    m.src_b = m.dst_b = (uint64_t)L * Jtot * N;
    m.src_j = m.dst_j = N;
    m.src_l = m.dst_l = (uint64_t)Jtot * N;
    if ((e = launch_ntt_fwd((int)ctx->logN, ly->op, ly->op, m, n_rows * Jtot * L, ctx->tw, ctx->twsh, ctx->lc, st)) !=
        hipSuccess)
        return fail(e, "operand ntt");
    if ((e = launch_scale_operands(ly->op, ctx->xinv, d_cls, Jtot, n_rows, L, N, ctx->lc, st)) != hipSuccess)
        return fail(e, "operand scale");
    if ((e = hipDeviceSynchronize()) != hipSuccess) return fail(e, "pack sync");
    hipFree(d_rho);
    hipFree(d_fh);
    hipFree(d_cls);
    *out = ly;
    return HE_OK;
}


int he_pack_operands(he_ctx *ctx, const he_layer_desc *desc, const uint32_t *a, const uint32_t *b, uint32_t flags,
                     he_layer **out) {
    if (!ctx || !desc || !a || !b || !out) return HE_EINVAL;
    if (flags != HE_PACK_CLASS_INTT && flags != HE_PACK_FULL_INTT) return HE_EINVAL;
    he_layer_info info;
    std::vector<uint32_t> cls;
    int rc = layer_geometry(ctx, desc, flags, &info, &cls);
    if (rc != HE_OK) return rc;
    const uint32_t N = ctx->N, L = ctx->L, K_in = info.K_in, Jtot = 2 * K_in;
    const uint32_t n_rows = desc->kind == HE_LAYER_CONV ? desc->c_o : info.blocks;
    // residues must be below their limb's prime
    const size_t per_op = (size_t)K_in * n_rows * L * N;
    for (size_t i = 0; i < per_op; ++i) {
        const uint32_t q = ctx->primes[(i / N) % L];
        if (a[i] >= q || b[i] >= q) return HE_EINVAL;
    }
    he_layer *ly = new (std::nothrow) he_layer();
    if (!ly) return HE_ENOMEM;
    ly->ctx = ctx;
    ly->n_rows = n_rows;
    const size_t op_words = (size_t)n_rows * L * Jtot * N;
    std::vector<uint32_t> host(op_words);
    for (uint32_t n = 0; n < n_rows; ++n)
        for (uint32_t l = 0; l < L; ++l)
            for (uint32_t j = 0; j < K_in; ++j) {
                const size_t src = (((size_t)j * n_rows + n) * L + l) * N;
                std::memcpy(&host[(((size_t)n * L + l) * Jtot + j) * N], a + src, N * 4);
                std::memcpy(&host[(((size_t)n * L + l) * Jtot + K_in + j) * N], b + src, N * 4);
            }
    std::vector<int32_t> hbias;
    if (desc->kind == HE_LAYER_FC) hbias.assign((size_t)info.blocks * info.n_o_p, 0);
    info.resident_bytes = op_words * 4 + hbias.size() * 4;
    ly->info = info;
    uint32_t *d_cls = nullptr;
    hipError_t e;
    auto fail = [&](hipError_t err, const char *what) {
        hipFree(d_cls);
        he_free_layer(ly);
        return dev_fail(err, what);
    };
    if ((e = hipMalloc((void **)&ly->op, op_words * 4)) != hipSuccess) {
        he_free_layer(ly);
        return HE_ENOMEM;
    }
    if ((e = hipMemcpy(ly->op, host.data(), op_words * 4, hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e, "pack operands copy");
    if (!hbias.empty()) {
        if ((e = hipMalloc((void **)&ly->bias, hbias.size() * 4)) != hipSuccess) return fail(e, "pack bias");
        if ((e = hipMemcpy(ly->bias, hbias.data(), hbias.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
            return fail(e, "pack bias copy");
    }
    if (desc->kind == HE_LAYER_CONV && flags == HE_PACK_CLASS_INTT) {
        if ((e = hipMalloc((void **)&d_cls, cls.size() * 4)) != hipSuccess) return fail(e, "pack cls");
        if ((e = hipMemcpy(d_cls, cls.data(), cls.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
            return fail(e, "pack cls copy");
    }
    RowMap m;
    m.J = Jtot;
    m.L = L;
    m.src_b = m.dst_b = (uint64_t)L * Jtot * N;
    m.src_j = m.dst_j = N;
    m.src_l = m.dst_l = (uint64_t)Jtot * N;
    if ((e = launch_ntt_fwd((int)ctx->logN, ly->op, ly->op, m, n_rows * Jtot * L, ctx->tw, ctx->twsh, ctx->lc,
                            nullptr)) != hipSuccess)
        return fail(e, "operand ntt");
    if ((e = launch_scale_operands(ly->op, ctx->xinv, d_cls, Jtot, n_rows, L, N, ctx->lc, nullptr)) != hipSuccess)
        return fail(e, "operand scale");
    if ((e = hipDeviceSynchronize()) != hipSuccess) return fail(e, "pack sync");
    hipFree(d_cls);
    *out = ly;
    return HE_OK;
}

int he_client_masks(he_ctx *ctx, const he_layer *server, const uint32_t *d_b, const int32_t *d_e1,
                    const int32_t *d_e2, he_layer **out) {
    if (!ctx || !server || server->ctx != ctx || !d_b || !d_e1 || !d_e2 || !out) return HE_EINVAL;
    const he_layer_info &in = server->info;
    const uint32_t N = ctx->N, L = ctx->L, K_in = in.K_in, Jtot = 2 * K_in, n_rows = server->n_rows;
    he_layer *ly = new (std::nothrow) he_layer();
    if (!ly) return HE_ENOMEM;
    ly->ctx = ctx;
    ly->n_rows = n_rows;
    ly->info = in;
    const size_t op_words = (size_t)n_rows * L * Jtot * N;
    uint32_t *d_cls = nullptr, *bhat = nullptr;
    auto fail = [&](hipError_t err, const char *what) {
        hipFree(d_cls);
        hipFree(bhat);
        he_free_layer(ly);
        return dev_fail(err, what);
    };
    hipError_t e;
    if ((e = hipMalloc((void **)&ly->op, op_words * 4)) != hipSuccess || 
        (e = hipMalloc((void **)&bhat, (size_t)L * N * 4)) != hipSuccess) {
        hipFree(bhat);
        he_free_layer(ly);
        return HE_ENOMEM;
    }
    if (in.kind == HE_LAYER_FC) {
        // the client's share carries no bias
        const size_t nb = (size_t)in.blocks * in.n_o_p;
        if ((e = hipMalloc((void **)&ly->bias, nb * 4)) != hipSuccess) return fail(e, "client masks bias");
        if ((e = hipMemsetAsync(ly->bias, 0, nb * 4, nullptr)) != hipSuccess) return fail(e, "client masks bias");
        ly->info.resident_bytes = op_words * 4 + nb * 4;
    }
    // f NTT(e1), f NTT(e2) in the operand layout, f the server layer's factor
    if ((e = launch_mask_noise(d_e1, d_e2, ly->op, K_in, n_rows, L, N, ctx->lc, nullptr)) != hipSuccess)
        return fail(e, "client masks noise");
    RowMap m;
    m.J = Jtot;
    m.L = L;
    m.src_b = m.dst_b = (uint64_t)L * Jtot * N;
    m.src_j = m.dst_j = N;
    m.src_l = m.dst_l = (uint64_t)Jtot * N;
    if ((e = launch_ntt_fwd((int)ctx->logN, ly->op, ly->op, m, n_rows * Jtot * L, ctx->tw, ctx->twsh, ctx->lc,
                            nullptr)) != hipSuccess)
        return fail(e, "client masks noise ntt");
    if (in.kind == HE_LAYER_CONV && in.flags == HE_PACK_CLASS_INTT) {
        std::vector<uint32_t> cls(n_rows);
        for (uint32_t n = 0; n < n_rows; ++n) cls[n] = (n % in.g_o) * (in.s / in.g_o);
        if ((e = hipMalloc((void **)&d_cls, cls.size() * 4)) != hipSuccess) return fail(e, "client masks cls");
        if ((e = hipMemcpy(d_cls, cls.data(), cls.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
            return fail(e, "client masks cls copy");
    }
    if ((e = launch_scale_operands(ly->op, ctx->xinv, d_cls, Jtot, n_rows, L, N, ctx->lc, nullptr)) != hipSuccess)
        return fail(e, "client masks scale");
    // NTT(b), then the masks from the server's f NTT(rho), f NTT(-Delta fhat)
    RowMap mb;
    std::memset(&mb, 0, sizeof(mb));
    mb.J = 1;
    mb.L = L;
    mb.src_l = mb.dst_l = N;
    if ((e = launch_ntt_fwd((int)ctx->logN, d_b, bhat, mb, L, ctx->tw, ctx->twsh, ctx->lc, nullptr)) != hipSuccess)
        return fail(e, "client masks ntt(b)");
    if ((e = launch_mask_combine(server->op, bhat, ly->op, K_in, n_rows, L, N, ctx->lc, nullptr)) != hipSuccess)
        return fail(e, "client masks combine");
    if ((e = hipDeviceSynchronize()) != hipSuccess) return fail(e, "client masks sync");
    hipFree(d_cls);
    hipFree(bhat);
    *out = ly;
    return HE_OK;
}

int he_encrypt_c0(he_ctx *ctx, uint32_t rows, const int32_t *d_v, const uint32_t *d_b, const uint32_t *d_msg,
                  const int32_t *d_e0, uint32_t *d_out, void *stream) {
    if (!ctx) return HE_EINVAL;
    if (rows == 0) return HE_OK;
    if (!d_v || !d_b || !d_msg || !d_e0 || !d_out) return HE_EINVAL;
    const uint32_t N = ctx->N, L = ctx->L;
    hipStream_t st = (hipStream_t)stream;
    void *ws = nullptr;
    const size_t vb_bytes = align256((size_t)rows * L * N * 4);
    int rc = ctx_workspace(ctx, st, vb_bytes + align256((size_t)L * N * 4), &ws);
    if (rc != HE_OK) return rc;
    uint32_t *V = (uint32_t *)ws;
    uint32_t *Bh = (uint32_t *)((char *)ws + vb_bytes);
    RowMap m;
    m.J = 1;
    m.L = L;
    m.src_b = m.dst_b = (uint64_t)L * N;
    m.src_j = m.dst_j = 0;
    m.src_l = m.dst_l = N;
    EpiParams ep;
    std::memset(&ep, 0, sizeof(ep));
    ep.scale = 1;
    hipError_t e;
    if ((e = launch_lift_signed(d_v, V, rows, L, N, ctx->lc, st)) != hipSuccess) return dev_fail(e, "encrypt lift");
    if ((e = launch_ntt_fwd((int)ctx->logN, V, V, m, rows * L, ctx->tw, ctx->twsh, ctx->lc, st)) != hipSuccess)
        return dev_fail(e, "encrypt ntt v");
    if ((e = launch_ntt_fwd((int)ctx->logN, d_b, Bh, m, L, ctx->tw, ctx->twsh, ctx->lc, st)) != hipSuccess)
        return dev_fail(e, "encrypt ntt b");
    if ((e = launch_mul_bcast(V, Bh, V, rows, L, N, ctx->lc, st)) != hipSuccess) return dev_fail(e, "encrypt mul");
    if ((e = launch_ntt_inv((int)ctx->logN, V, V, m, rows * L, ctx->twi, ctx->twish, ctx->lc, EPI_STORE, ep, st)) !=
        hipSuccess)
        return dev_fail(e, "encrypt intt");
    if ((e = launch_encrypt_combine(V, d_msg, d_e0, d_out, rows, L, N, ctx->lc, st)) != hipSuccess)
        return dev_fail(e, "encrypt combine");
    return HE_OK;
}

int he_decrypt(he_ctx *ctx, uint32_t rows, uint32_t M, const uint32_t *d_x0, const uint32_t *d_x1, uint32_t *d_msg,
               void *stream) {
    if (!ctx || M > ctx->N) return HE_EINVAL;
    if (rows == 0) return HE_OK;
    if (!d_x0 || !d_msg) return HE_EINVAL;
    if (M == 0) M = ctx->N;
    hipError_t e = launch_decrypt(d_x0, d_x1, d_msg, rows, ctx->L, M, ctx->lc, ctx->dc, (hipStream_t)stream);
    return e == hipSuccess ? HE_OK : dev_fail(e, "decrypt");
}

namespace {

size_t x_bytes(const he_layer *ly, uint32_t B) {
    const he_layer_info &in = ly->info;
    return align256((size_t)B * 2 * in.K_in * in.L * in.N * 4);
}

// a1: forward NTT of the c0 rows (b, j, l) and/or the sh rows (one coefficient row per (b, j),
// read for every limb) into the NTT-domain input buffer x [B][2 K_in][L][N]: c0 at J < K_in,
// sh at J >= K_in.  One launch.
hipError_t inputs_ntt(he_ctx *ctx, const he_layer *ly, uint32_t B, const uint32_t *d_c0, const uint32_t *d_sh,
                      uint32_t *x, hipStream_t st) {
    const he_layer_info &in = ly->info;
    const uint32_t N = in.N, L = in.L, K_in = in.K_in, Jtot = 2 * K_in;
    const int logN = (int)ctx->logN;
    RowMap mc;
    mc.J = K_in;
    mc.L = L;
    mc.src_b = (uint64_t)K_in * L * N;
    mc.src_j = (uint64_t)L * N;
    mc.src_l = N;
    mc.dst_b = (uint64_t)Jtot * L * N;
    mc.dst_j = (uint64_t)L * N;
    mc.dst_l = N;
    RowMap ms = mc;
    ms.src_b = (uint64_t)K_in * N;
    ms.src_j = N;
    ms.src_l = 0;
    FwdJobs jobs;
    int nj = 0;
    if (d_c0) {
        jobs.src[nj] = d_c0;
        jobs.dst[nj] = x;
        jobs.map[nj] = mc;
        ++nj;
    }
    if (d_sh) {
        jobs.src[nj] = d_sh;
        jobs.dst[nj] = x + (size_t)K_in * L * N;
        jobs.map[nj] = ms;
        ++nj;
    }
    if (nj == 0) return hipSuccess;
    if (nj == 1) {
        jobs.src[1] = jobs.src[0];
        jobs.dst[1] = jobs.dst[0];
        jobs.map[1] = jobs.map[0];
    }
    jobs.rows0 = B * K_in * L;
    const uint32_t rows = jobs.rows0 * nj;
    ProfScope ps(ctx, HE_K_NTT_FWD);
    const hipError_t e = launch_ntt_fwd2(logN, knob(ctx, HE_TUNE_NTT_FWD, (uint32_t)logN, rows), jobs, rows, ctx->tw,
                                         ctx->twsh, ctx->lc, st, ps.ev());
    return ps.done(e);
}

// a2-a4 of a conv layer from the NTT-domain inputs x; mac: MAC-output workspace.
int conv_from_x(he_ctx *ctx, const he_layer *ly, uint32_t B, const uint32_t *xn, bool has_sh,
                const uint32_t *d_sh_next, uint32_t *d_out, uint32_t *mac, hipStream_t st) {
    const he_layer_info &in = ly->info;
    const uint32_t N = in.N, L = in.L, K_in = in.K_in, Jtot = 2 * K_in, c_o = ly->n_rows;
    const int logN = (int)ctx->logN;
    hipError_t e;
    // a2: coefficient-wise MAC over the input rows
    const uint32_t Juse = has_sh ? Jtot : K_in;
    const bool cls = in.flags == HE_PACK_CLASS_INTT;
    int mk = mac_variant(ctx, ly, B);
    if (mk == 7 || mk == 8) mk = mac_variant_multi(ctx, ly, B, -1);   // no sync block here: the multi-launch rule
    if (mk == 2) {
        // a2 + a3 + a4 in one launch: MAC, residue-class inverse, extraction, + Delta sh'
        ProfScope ps(ctx, HE_K_MAC_TAIL);
        e = launch_mac_tail(xn, ly->op, d_out, d_sh_next, B, Jtot, Juse, c_o, in.g_o, in.K_out, L, N, in.s, ctx->twi,
                            ctx->twish, ctx->lc, st, ps.ev());
        if ((e = ps.done(e)) != hipSuccess) return dev_fail(e, "conv mac + tail");
        return HE_OK;
    }
    {
        const bool tiled = mk == 1;
        ProfScope ps(ctx, mk == 9 ? HE_K_MAC_MFMA : HE_K_MAC);
        if (mk == 3 || mk == 4)
            e = launch_mac_lds(xn, ly->op, mac, B, Jtot, Juse, c_o, L, N, in.s, mk == 4, ctx->lc, st, ps.ev());
        else if (mk == 5 || mk == 6)
            e = launch_mac_dma(xn, ly->op, mac, B, Jtot, Juse, c_o, L, N, in.s, mk == 6, ctx->lc, st, ps.ev());
        else if (mk == 9)
            e = launch_mac_mfma(xn, ly->op, mac, B, Jtot, Juse, c_o, L, N, in.s, ctx->lc, st, ps.ev());
        else if (tiled)
            e = launch_mac_tiled(xn, ly->op, mac, B, Jtot, Juse, c_o, L, N, in.s, cls, ctx->lc, st, ps.ev());
        else if (cls)
            e = launch_mac_class(xn, ly->op, mac, B, Jtot, Juse, c_o, L, N, in.s, ctx->lc, st, ps.ev());
        else
            e = launch_mac_full(xn, ly->op, mac, B, Jtot, Juse, c_o, L, N, ctx->lc, st, ps.ev());
        if ((e = ps.done(e)) != hipSuccess) return dev_fail(e, "conv mac");
    }
    // a3 + a4: inverse transform, residue-class extraction, + Delta sh'
    if (cls) {
        const uint32_t logm = (uint32_t)logN - log2u(in.s);
        ProfScope ps(ctx, HE_K_TAIL);
        if (logm >= 4)
            e = launch_tail_rows(mac, d_out, d_sh_next, B, c_o, in.g_o, in.K_out, L, N, in.s, ctx->twi, ctx->twish,
                                 ctx->lc, st, ps.ev(), knob(ctx, HE_TUNE_TAIL, logm, B * in.K_out * in.g_o * L),
                                 mk == 9);
        else
            e = launch_tail_class(mac, d_out, d_sh_next, B, c_o, in.g_o, in.K_out, L, N, in.s, ctx->twi, ctx->twish,
                                  ctx->lc, st, ps.ev());
        if ((e = ps.done(e)) != hipSuccess) return dev_fail(e, "conv tail");
    } else {
        EpiParams ep;
        std::memset(&ep, 0, sizeof(ep));
        ep.c_o = c_o;
        ep.g_o = in.g_o;
        ep.K_out = in.K_out;
        ep.s_log = log2u(in.s);
        ep.out = d_out;
        ep.sh_next = d_sh_next;
        RowMap mi;
        std::memset(&mi, 0, sizeof(mi));
        mi.J = 1;
        mi.L = L;
        const uint32_t rows = B * in.K_out * in.g_o * L;
        ProfScope ps(ctx, HE_K_INTT);
        e = launch_ntt_inv(logN, mac, d_out, mi, rows, ctx->twi, ctx->twish, ctx->lc, EPI_CONV_CLASS, ep, st, ps.ev(),
                           knob(ctx, HE_TUNE_NTT_INV, (uint32_t)logN, rows));
        if ((e = ps.done(e)) != hipSuccess) return dev_fail(e, "conv inverse ntt");
    }
    return HE_OK;
}

// a2-a5 of an FC layer from the NTT-domain inputs x; mac: MAC-output workspace.
int fc_from_x(he_ctx *ctx, const he_layer *ly, uint32_t B, const uint32_t *xn, bool has_sh,
              const uint32_t *d_sh_next, uint32_t *d_out, uint32_t *mac, hipStream_t st) {
    const he_layer_info &in = ly->info;
    const uint32_t N = in.N, L = in.L;
    const int logN = (int)ctx->logN;
    hipError_t e;
    {
        ProfScope ps(ctx, HE_K_MAC);
        e = launch_mac_full(xn, ly->op, mac, B, 2, has_sh ? 2 : 1, in.blocks, L, N, ctx->lc, st, ps.ev());
        if ((e = ps.done(e)) != hipSuccess) return dev_fail(e, "fc mac");
    }
    EpiParams ep;
    std::memset(&ep, 0, sizeof(ep));
    ep.n_o_p = in.n_o_p;
    ep.blocks = in.blocks;
    ep.out = d_out;
    ep.sh_next = d_sh_next;
    ep.bias = ly->bias;
    RowMap mi;
    std::memset(&mi, 0, sizeof(mi));
    mi.J = 1;
    mi.L = L;
    const uint32_t rows = B * in.blocks * L;
    {
        ProfScope ps(ctx, HE_K_INTT);
        e = launch_ntt_inv(logN, mac, d_out, mi, rows, ctx->twi, ctx->twish, ctx->lc, EPI_FC_PREFIX, ep, st, ps.ev(),
                           knob(ctx, HE_TUNE_NTT_INV, (uint32_t)logN, rows));
        if ((e = ps.done(e)) != hipSuccess) return dev_fail(e, "fc inverse ntt");
    }
    return HE_OK;
}

}  // namespace

}  // extern "C"

namespace {

// a1-a5 of one layer call.  x_given: NTT-domain inputs (the *_ntt forms; ws then holds only the
// MAC output), else c0 / sh are transformed into ws.  sync: a zeroed sync block for the
// one-launch form, or null for the multi-launch forms.
int layer_exec(he_ctx *ctx, const he_layer *ly, uint32_t B, const uint32_t *d_c0, const uint32_t *d_sh,
               const uint32_t *x_given, bool has_sh, const uint32_t *d_sh_next, uint32_t *d_out, void *d_ws,
               uint32_t *sync, hipStream_t st) {
    const bool conv = ly->info.kind == HE_LAYER_CONV;
    uint32_t *xn = x_given ? const_cast<uint32_t *>(x_given) : (uint32_t *)d_ws;
    uint32_t *mac = x_given ? (uint32_t *)d_ws : (uint32_t *)((char *)d_ws + x_bytes(ly, B));
    FusedLayer jb;
    const int form = sync ? mac_variant(ctx, ly, B) : -1;
    if ((form == 7 || form == 8) && layer_one_launch_ok(ctx, ly, B, &jb, form == 8)) {
        jb.c0 = d_c0;
        jb.sh = d_sh;
        jb.sh_next = d_sh_next;
        jb.out = d_out;
        jb.op = ly->op;
        jb.bias = ly->bias;
        jb.x = xn;
        jb.h = mac;
        jb.Juse = has_sh ? jb.Jtot : jb.K_in;
        jb.ntt_c0 = x_given ? 0 : jb.K_in;
        jb.ntt_sh = (x_given || !d_sh) ? 0 : jb.K_in;
        fused_layer_plan(jb);
        ProfScope ps(ctx, form == 8 ? HE_K_LAYER_ROWS : HE_K_LAYER);
        hipError_t e = launch_fused_layer(jb, ctx->tw, ctx->twsh, ctx->twi, ctx->twish, ctx->xinv, ctx->lc, sync,
                                          st, ps.ev());
        if ((e = ps.done(e)) != hipSuccess) return dev_fail(e, conv ? "conv layer launch" : "fc layer launch");
        return HE_OK;
    }
    if (!x_given) {
        const hipError_t e = inputs_ntt(ctx, ly, B, d_c0, d_sh, xn, st);
        if (e != hipSuccess) return dev_fail(e, conv ? "conv forward ntt" : "fc forward ntt");
    }
    return conv ? conv_from_x(ctx, ly, B, xn, has_sh, d_sh_next, d_out, mac, st)
                : fc_from_x(ctx, ly, B, xn, has_sh, d_sh_next, d_out, mac, st);
}

int check_layer_args(const he_ctx *ctx, const he_layer *ly, int kind, const uint32_t *d_c0, const uint32_t *d_out,
                     const void *d_ws) {
    if (!ctx || !ly || ly->ctx != ctx || ly->info.kind != kind) return HE_EINVAL;
    if (!d_c0 || !d_out || !d_ws) return HE_EINVAL;
    if (!aligned16(d_c0) || !aligned16(d_ws)) return HE_EINVAL;
    if (kind == HE_LAYER_CONV && !aligned16(d_out)) return HE_EINVAL;
    return HE_OK;
}

}  // namespace

int he_layer_call_sync(he_ctx *ctx, const he_layer *ly, uint32_t B, const uint32_t *d_c0, const uint32_t *d_sh,
                       const uint32_t *d_sh_next, uint32_t *d_out, void *d_ws, size_t ws_bytes, uint32_t *sync,
                       void *stream) {
    if (!ly) return HE_EINVAL;
    if (B == 0) return (ctx && ly->ctx == ctx) ? HE_OK : HE_EINVAL;
    const int rc = check_layer_args(ctx, ly, ly->info.kind, d_c0, d_out, d_ws);
    if (rc != HE_OK) return rc;
    if (ws_bytes < layer_ws_bytes(ly, B)) return HE_EINVAL;
    return layer_exec(ctx, ly, B, d_c0, d_sh, nullptr, d_sh != nullptr, d_sh_next, d_out, d_ws, sync,
                      (hipStream_t)stream);
}

uint32_t *he_sync_block_alloc() {
    uint32_t *p = nullptr;
    if (hipMalloc((void **)&p, (size_t)FZ_SYNC_WORDS * 4) != hipSuccess) return nullptr;
    if (hipMemset(p, 0, (size_t)FZ_SYNC_WORDS * 4) != hipSuccess) {
        hipFree(p);
        return nullptr;
    }
    return p;
}

extern "C" {

int he_conv_layer_ws(he_ctx *ctx, const he_layer *ly, uint32_t B, const uint32_t *d_c0, const uint32_t *d_sh,
                     const uint32_t *d_sh_next, uint32_t *d_out, void *d_ws, size_t ws_bytes, void *stream) {
    if (!ctx || !ly || ly->ctx != ctx || ly->info.kind != HE_LAYER_CONV) return HE_EINVAL;
    return he_layer_call_sync(ctx, ly, B, d_c0, d_sh, d_sh_next, d_out, d_ws, ws_bytes,
                              ctx_sync(ctx, (hipStream_t)stream), stream);
}

int he_conv_layer(he_ctx *ctx, const he_layer *ly, uint32_t B, const uint32_t *d_c0, const uint32_t *d_sh,
                  const uint32_t *d_sh_next, uint32_t *d_out, void *stream) {
    if (!ctx || !ly || ly->ctx != ctx || ly->info.kind != HE_LAYER_CONV) return HE_EINVAL;
    if (B == 0) return HE_OK;
    void *ws = nullptr;
    uint32_t *sync = nullptr;
    const size_t need = layer_ws_bytes(ly, B);
    int rc = ctx_workspace(ctx, (hipStream_t)stream, need, &ws, &sync);
    if (rc != HE_OK) return rc;
    return he_layer_call_sync(ctx, ly, B, d_c0, d_sh, d_sh_next, d_out, ws, need, sync, stream);
}

int he_conv_layer_noalloc(he_ctx *ctx, const he_layer *ly, uint32_t B, const uint32_t *d_c0, const uint32_t *d_sh,
                          const uint32_t *d_sh_next, uint32_t *d_out, void *stream) {
    if (!ctx || !ly || ly->ctx != ctx || ly->info.kind != HE_LAYER_CONV) return HE_EINVAL;
    if (B == 0) return HE_OK;
    const size_t need = layer_ws_bytes(ly, B);
    if (need > (size_t)HE_NOALLOC_SCRATCH_BYTES) {
        g_last_error = "he_conv_layer_noalloc: " + std::to_string(need) + " bytes of scratch needed at B = " +
                       std::to_string(B) + ", the static scratch holds " +
                       std::to_string((size_t)HE_NOALLOC_SCRATCH_BYTES);
        return HE_ENOMEM;
    }
    void *ws = scratch_device_ptr(ctx->device);
    if (!ws) {
        g_last_error = "he_conv_layer_noalloc: no scratch address for this device";
        return HE_EDEVICE;
    }
    // timing events are created per launch when profiling is on; this form creates none
    const bool saved = tl_no_prof;
    tl_no_prof = true;
    uint32_t *sync = (uint32_t *)((char *)ws + HE_NOALLOC_SCRATCH_BYTES);
    const int rc = he_layer_call_sync(ctx, ly, B, d_c0, d_sh, d_sh_next, d_out, ws, (size_t)HE_NOALLOC_SCRATCH_BYTES,
                                      sync, stream);
    tl_no_prof = saved;
    return rc;
}

int he_fc_layer_ws(he_ctx *ctx, const he_layer *ly, uint32_t B, const uint32_t *d_c0, const uint32_t *d_sh,
                   const uint32_t *d_sh_next, uint32_t *d_out, void *d_ws, size_t ws_bytes, void *stream) {
    if (!ctx || !ly || ly->ctx != ctx || ly->info.kind != HE_LAYER_FC) return HE_EINVAL;
    return he_layer_call_sync(ctx, ly, B, d_c0, d_sh, d_sh_next, d_out, d_ws, ws_bytes,
                              ctx_sync(ctx, (hipStream_t)stream), stream);
}

int he_fc_layer(he_ctx *ctx, const he_layer *ly, uint32_t B, const uint32_t *d_c0, const uint32_t *d_sh,
                const uint32_t *d_sh_next, uint32_t *d_out, void *stream) {
    if (!ctx || !ly || ly->ctx != ctx || ly->info.kind != HE_LAYER_FC) return HE_EINVAL;
    if (B == 0) return HE_OK;
    void *ws = nullptr;
    uint32_t *sync = nullptr;
    const size_t need = layer_ws_bytes(ly, B);
    int rc = ctx_workspace(ctx, (hipStream_t)stream, need, &ws, &sync);
    if (rc != HE_OK) return rc;
    return he_layer_call_sync(ctx, ly, B, d_c0, d_sh, d_sh_next, d_out, ws, need, sync, stream);
}

int he_layer_inputs_ntt(he_ctx *ctx, const he_layer *ly, uint32_t B, const uint32_t *d_c0, const uint32_t *d_sh,
                        uint32_t *d_x, void *stream) {
    if (!ctx || !ly || ly->ctx != ctx || !d_x) return HE_EINVAL;
    if (B == 0 || (!d_c0 && !d_sh)) return HE_OK;
    if (!aligned16(d_x) || (d_c0 && !aligned16(d_c0))) return HE_EINVAL;
    const hipError_t e = inputs_ntt(ctx, ly, B, d_c0, d_sh, d_x, (hipStream_t)stream);
    return e == hipSuccess ? HE_OK : dev_fail(e, "layer input ntt");
}

int he_conv_layer_ntt(he_ctx *ctx, const he_layer *ly, uint32_t B, const uint32_t *d_x, int has_sh,
                      const uint32_t *d_sh_next, uint32_t *d_out, void *stream) {
    if (!ctx || !ly || ly->ctx != ctx || ly->info.kind != HE_LAYER_CONV) return HE_EINVAL;
    if (B == 0) return HE_OK;
    if (!d_x || !d_out || !aligned16(d_x) || !aligned16(d_out)) return HE_EINVAL;
    void *ws = nullptr;
    uint32_t *sync = nullptr;
    const size_t need = layer_ws_bytes(ly, B) - x_bytes(ly, B);
    int rc = ctx_workspace(ctx, (hipStream_t)stream, need > 0 ? need : 256, &ws, &sync);
    if (rc != HE_OK) return rc;
    return layer_exec(ctx, ly, B, nullptr, nullptr, d_x, has_sh != 0, d_sh_next, d_out, ws, sync,
                      (hipStream_t)stream);
}

int he_fc_layer_ntt(he_ctx *ctx, const he_layer *ly, uint32_t B, const uint32_t *d_x, int has_sh,
                    const uint32_t *d_sh_next, uint32_t *d_out, void *stream) {
    if (!ctx || !ly || ly->ctx != ctx || ly->info.kind != HE_LAYER_FC) return HE_EINVAL;
    if (B == 0) return HE_OK;
    if (!d_x || !d_out || !aligned16(d_x)) return HE_EINVAL;
    void *ws = nullptr;
    uint32_t *sync = nullptr;
    const size_t need = layer_ws_bytes(ly, B) - x_bytes(ly, B);
    int rc = ctx_workspace(ctx, (hipStream_t)stream, need, &ws, &sync);
    if (rc != HE_OK) return rc;
    return layer_exec(ctx, ly, B, nullptr, nullptr, d_x, has_sh != 0, d_sh_next, d_out, ws, sync,
                      (hipStream_t)stream);
}

int he_ntt_forward(he_ctx *ctx, uint32_t rows, const uint32_t *d_in, uint32_t *d_out, void *stream) {
    if (!ctx || (rows && (!d_in || !d_out))) return HE_EINVAL;
    RowMap m;
    m.J = 1;
    m.L = ctx->L;
    m.src_b = m.dst_b = (uint64_t)ctx->L * ctx->N;
    m.src_j = m.dst_j = 0;
    m.src_l = m.dst_l = ctx->N;
    hipError_t e = launch_ntt_fwd((int)ctx->logN, d_in, d_out, m, rows * ctx->L, ctx->tw, ctx->twsh, ctx->lc,
                                  (hipStream_t)stream);
    return e == hipSuccess ? HE_OK : dev_fail(e, "ntt forward");
}

int he_ntt_inverse(he_ctx *ctx, uint32_t rows, const uint32_t *d_in, uint32_t *d_out, void *stream) {
    if (!ctx || (rows && (!d_in || !d_out))) return HE_EINVAL;
    RowMap m;
    m.J = 1;
    m.L = ctx->L;
    m.src_b = m.dst_b = (uint64_t)ctx->L * ctx->N;
    m.src_j = m.dst_j = 0;
    m.src_l = m.dst_l = ctx->N;
    EpiParams ep;
    std::memset(&ep, 0, sizeof(ep));
    ep.scale = 1;
    hipError_t e = launch_ntt_inv((int)ctx->logN, d_in, d_out, m, rows * ctx->L, ctx->twi, ctx->twish, ctx->lc,
                                  EPI_STORE, ep, (hipStream_t)stream);
    return e == hipSuccess ? HE_OK : dev_fail(e, "ntt inverse");
}

int he_poly_mul(he_ctx *ctx, uint32_t rows, const uint32_t *d_a, const uint32_t *d_b, uint32_t *d_c, void *stream) {
    if (!ctx) return HE_EINVAL;
    if (rows == 0) return HE_OK;
    if (!d_a || !d_b || !d_c || d_c == d_a || d_c == d_b) return HE_EINVAL;
    const size_t words = (size_t)rows * ctx->L * ctx->N;
    void *ws = nullptr;
    int rc = ctx_workspace(ctx, (hipStream_t)stream, align256(words * 4) * 2, &ws);
    if (rc != HE_OK) return rc;
    uint32_t *A = (uint32_t *)ws;
    uint32_t *Bv = (uint32_t *)((char *)ws + align256(words * 4));
    if ((rc = he_ntt_forward(ctx, rows, d_a, A, stream)) != HE_OK) return rc;
    if ((rc = he_ntt_forward(ctx, rows, d_b, Bv, stream)) != HE_OK) return rc;
    hipError_t e = launch_pointwise_mul(A, Bv, A, rows, ctx->L, ctx->N, ctx->lc, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(e, "pointwise");
    return he_ntt_inverse(ctx, rows, A, d_c, stream);
}

}  // extern "C"

// ------------------------------------------------------------------ grouped launch
struct he_group {
    int device = 0;
    he_ctx *ctx0 = nullptr;              // the first call's context: timing (he_profile_*)
    std::vector<FusedJob> jobs;          // host copy of the device job list
    FusedJob *d_jobs = nullptr;
    LimbConsts *d_lc = nullptr;          // one per distinct context
    void *ws = nullptr;                  // every job's NTT-domain inputs and block sums
    uint32_t *sync = nullptr;            // header + every job's counters, zero between launches
    size_t ws_bytes = 0, sync_words = 0;
    uint32_t count[3] = {0, 0, 0};
    uint32_t chunk_log = 6;              // items per XCD chunk of a phase: 2^chunk_log (he_group_tune)
};

namespace {

void group_release(he_group *g) {
    if (!g) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(g->device);
    if (g->d_jobs) (void)hipFree(g->d_jobs);
    if (g->d_lc) (void)hipFree(g->d_lc);
    if (g->ws) (void)hipFree(g->ws);
    if (g->sync) (void)hipFree(g->sync);
    (void)hipSetDevice(cur);
    delete g;
}

}  // namespace

extern "C" {

int he_group_create(const he_layer_call *calls, uint32_t n, uint32_t flags, he_group **out) {
    if (!out || !calls || n == 0 || flags > HE_GROUP_MAC_TILED) return HE_EINVAL;
    *out = nullptr;
    std::unique_ptr<he_group, void (*)(he_group *)> g(new he_group, group_release);
    g->ctx0 = calls[0].ctx;
    if (!g->ctx0) return HE_EINVAL;
    g->device = g->ctx0->device;
    std::vector<he_ctx *> ctxs;
    std::vector<size_t> ws_off(n);
    size_t ws_total = 0, ctr_total = 0;
    g->jobs.resize(n);
    for (uint32_t i = 0; i < n; ++i) {
        const he_layer_call &c = calls[i];
        // the buffers of a layer call (the workspace is the group's own)
        if (!c.ctx || c.ctx->device != g->device || !c.layer || c.layer->ctx != c.ctx || c.B == 0 || !c.d_c0 ||
            !c.d_out || !aligned16(c.d_c0) || (c.layer->info.kind == HE_LAYER_CONV && !aligned16(c.d_out))) {
            g_last_error = "he_group_create: call " + std::to_string(i) + ": invalid arguments";
            return HE_EINVAL;
        }
        FusedLayer jb;
        if (!fused_layer_shape(c.ctx, c.layer, c.B, false, jb)) {
            g_last_error = "he_group_create: call " + std::to_string(i) +
                           ": layer shape outside the grouped launch (conv in the residue-class form with "
                           "2 <= s <= 256 and N/s <= 4096, or FC with n_o' <= 1024; N 4096..16384)";
            return HE_EUNSUPPORTED;
        }
        const he_layer_info &in = c.layer->info;
        jb.c0 = c.d_c0;
        jb.sh = c.d_sh;
        jb.sh_next = c.d_sh_next;
        jb.out = c.d_out;
        jb.op = c.layer->op;
        jb.bias = c.layer->bias;
        jb.Juse = c.d_sh ? jb.Jtot : jb.K_in;
        jb.ntt_c0 = jb.K_in;
        jb.ntt_sh = c.d_sh ? jb.K_in : 0;
        jb.grouped = 1;
        // image-tiled MAC items: a resident operand word read once per tile of images rather than
        // once per image (automatic from four images up)
        if (jb.kind == FZ_KIND_CONV && flags != HE_GROUP_MAC_PER_IMAGE && (c.B >= 4 || flags == HE_GROUP_MAC_TILED)) {
            MacLdsGeom gm;
            size_t lds_pad = 0;
            if (mac_lds_geometry(c.B, c.layer->n_rows, in.N, in.s, &gm, &lds_pad, 64) &&
                (size_t)gm.R * gm.cpb <= in.N / 4 && mac_dma_lds_bytes(gm) <= fused_group_lds_bytes()) {
                jb.mac_tiled = 1;
                jb.gm = gm;
            }
        }
        fused_layer_plan(jb);
        jb.ctr_stride = 32;   // one counter per 128-byte line
        ws_off[i] = ws_total;
        ws_total += layer_ws_bytes(c.layer, c.B);
        FusedJob &J = g->jobs[i];
        std::memset(&J, 0, sizeof(J));
        J.jb = jb;
        J.tw = c.ctx->tw;
        J.twsh = c.ctx->twsh;
        J.twi = c.ctx->twi;
        J.twish = c.ctx->twish;
        J.xinv = c.ctx->xinv;
        J.ctr_off = (uint32_t)ctr_total;
        ctr_total += (size_t)jb.n_ctr * jb.ctr_stride;
        if (ctr_total > (1u << 30)) return HE_EUNSUPPORTED;
        for (int p = 0; p < 3; ++p) J.first[p] = g->count[p];
        g->count[0] += jb.n_ntt;
        g->count[1] += jb.n_mac;
        g->count[2] += jb.n_inv;
        if (std::find(ctxs.begin(), ctxs.end(), c.ctx) == ctxs.end()) ctxs.push_back(c.ctx);
    }
    for (int p = 0; p < 3; ++p)
        if (g->count[p] > (1u << 28)) return HE_EUNSUPPORTED;
    int cur = 0;
    HE_HIP(hipGetDevice(&cur));
    HE_HIP(hipSetDevice(g->device));
    struct Restore {
        int d;
        ~Restore() { (void)hipSetDevice(d); }
    } restore{cur};
    g->ws_bytes = align256(ws_total > 0 ? ws_total : 256);
    g->sync_words = FZ_SB_HDR + ctr_total;
    if (hipMalloc(&g->ws, g->ws_bytes) != hipSuccess || hipMalloc((void **)&g->sync, g->sync_words * 4) != hipSuccess ||
        hipMalloc((void **)&g->d_lc, ctxs.size() * sizeof(LimbConsts)) != hipSuccess ||
        hipMalloc((void **)&g->d_jobs, n * sizeof(FusedJob)) != hipSuccess) {
        g_last_error = "he_group_create: out of device memory";
        return HE_ENOMEM;
    }
    HE_HIP(hipMemset(g->sync, 0, g->sync_words * 4));
    for (size_t k = 0; k < ctxs.size(); ++k)
        HE_HIP(hipMemcpy(g->d_lc + k, &ctxs[k]->lc, sizeof(LimbConsts), hipMemcpyHostToDevice));
    for (uint32_t i = 0; i < n; ++i) {
        FusedJob &J = g->jobs[i];
        const size_t k = std::find(ctxs.begin(), ctxs.end(), calls[i].ctx) - ctxs.begin();
        J.lc = g->d_lc + k;
        J.jb.x = (uint32_t *)((char *)g->ws + ws_off[i]);
        J.jb.h = (uint32_t *)((char *)g->ws + ws_off[i] + x_bytes(calls[i].layer, calls[i].B));
    }
    HE_HIP(hipMemcpy(g->d_jobs, g->jobs.data(), n * sizeof(FusedJob), hipMemcpyHostToDevice));
    *out = g.release();
    return HE_OK;
}

int he_group_run(he_group *g, void *stream) {
    if (!g) return HE_EINVAL;
    ProfScope ps(g->ctx0, HE_K_GROUP);
    hipError_t e = launch_fused_group(g->d_jobs, (uint32_t)g->jobs.size(), g->count, g->chunk_log, g->sync,
                                      (hipStream_t)stream, ps.ev());
    if ((e = ps.done(e)) != hipSuccess) return dev_fail(e, "grouped layer launch");
    return HE_OK;
}

int he_group_set_chunk(he_group *g, uint32_t chunk_log) {
    if (!g || chunk_log > 10) return HE_EINVAL;
    g->chunk_log = chunk_log;
    return HE_OK;
}

int he_group_tune(he_group *g, void *stream, uint32_t *chunk_log) {
    if (!g) return HE_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HE_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return HE_EDEVICE;
    }
    int rc = HE_OK;
    uint32_t best = g->chunk_log;
    float best_ms = 0.f;
    for (uint32_t c : {2u, 3u, 4u, 5u, 6u, 7u, 8u}) {
        g->chunk_log = c;
        float t[3];
        for (int r = -1; r < 3 && rc == HE_OK; ++r) {
            // a warm-up launch, then three timed ones (the median is kept)
            if (hipEventRecord(e0, st) != hipSuccess) rc = HE_EDEVICE;
            if (rc == HE_OK && launch_fused_group(g->d_jobs, (uint32_t)g->jobs.size(), g->count, c, g->sync, st) !=
                                   hipSuccess)
                rc = HE_EDEVICE;
            if (rc == HE_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
                rc = HE_EDEVICE;
            float ms = 0.f;
            if (rc == HE_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = HE_EDEVICE;
            if (r >= 0) t[r] = ms;
        }
        if (rc != HE_OK) break;
        std::sort(t, t + 3);
        if (best_ms == 0.f || t[1] < best_ms) {
            best_ms = t[1];
            best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    g->chunk_log = best;
    if (rc != HE_OK) {
        g_last_error = "he_group_tune: a timed launch failed";
        return rc;
    }
    if (chunk_log) *chunk_log = best;
    return he_group_check(g, stream);
}

int he_group_check(he_group *g, void *stream) {
    if (!g) return HE_EINVAL;
    HE_HIP(hipStreamSynchronize((hipStream_t)stream));
    uint32_t err = 0;
    HE_HIP(hipMemcpy(&err, g->sync + FZ_SB_ERR, 4, hipMemcpyDeviceToHost));
    if (err == 0) return HE_OK;
    HE_HIP(hipMemset(g->sync + FZ_SB_ERR, 0, 4));
    g_last_error = "a grouped launch gave up waiting for an item it depends on";
    return HE_EDEVICE;
}

int he_group_items(const he_group *g, uint32_t *items, uint32_t *tiled_jobs, size_t *workspace_bytes) {
    if (!g) return HE_EINVAL;
    if (items)
        for (int p = 0; p < 3; ++p) items[p] = g->count[p];
    if (tiled_jobs) {
        uint32_t k = 0;
        for (const FusedJob &J : g->jobs) k += J.jb.mac_tiled ? 1u : 0u;
        *tiled_jobs = k;
    }
    if (workspace_bytes) *workspace_bytes = g->ws_bytes;
    return HE_OK;
}

void he_group_free(he_group *g) { group_release(g); }

}  // extern "C"
