// Layer sequences: a recorded list of conv / FC layer calls that runs as one
// host call, or as one replay of a captured HIP graph.
//
// A sequence owns one device workspace sized for its largest step; its steps
// run in order on one stream, so they share it.  Capture records the kernels of
// every step into a hipGraph (no memset nodes: the layer kernels write every
// output word), and replay launches that graph on the caller's stream.

#include <hip/hip_runtime.h>

#include <new>
#include <string>
#include <vector>

#include "../../include/he.h"
#include "he_internal.h"
#include "he_kernels.h"

namespace {

struct Step {
    int kind;
    const he_layer *ly;
    uint32_t B;
    const uint32_t *c0, *sh, *shn;
    uint32_t *out;
};

}  // namespace

struct he_seq {
    he_ctx *ctx = nullptr;
    std::vector<Step> steps;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    uint32_t *sync = nullptr;   // counter block of the one-launch layer form (steps run in stream order)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

int grow(he_seq *s, size_t need) {
    if (need <= s->ws_bytes) return HE_OK;
    if (s->exec) return HE_EINVAL;   // a captured graph holds the old workspace address
    if (s->ws) hipFree(s->ws);
    s->ws = nullptr;
    s->ws_bytes = 0;
    if (hipMalloc(&s->ws, need) != hipSuccess) return HE_ENOMEM;
    s->ws_bytes = need;
    return HE_OK;
}

int run_steps(he_seq *s, hipStream_t st) {
    for (const Step &p : s->steps) {
        const int rc = he_layer_call_sync(s->ctx, p.ly, p.B, p.c0, p.sh, p.shn, p.out, s->ws, s->ws_bytes, s->sync, st);
        if (rc != HE_OK) return rc;
    }
    return HE_OK;
}

}  // namespace

extern "C" {

int he_seq_create(he_ctx *ctx, he_seq **out) {
    if (!ctx || !out) return HE_EINVAL;
    he_seq *s = new (std::nothrow) he_seq();
    if (!s) return HE_ENOMEM;
    s->ctx = ctx;
    s->sync = he_sync_block_alloc();
    if (!s->sync) {
        delete s;
        return HE_ENOMEM;
    }
    *out = s;
    return HE_OK;
}

int he_seq_add(he_seq *s, const he_layer *ly, uint32_t B, const uint32_t *d_c0, const uint32_t *d_sh,
               const uint32_t *d_sh_next, uint32_t *d_out) {
    if (!s || !ly || !d_c0 || !d_out) return HE_EINVAL;
    if (s->exec) return HE_EINVAL;
    he_layer_info info;
    if (he_layer_info_get(ly, &info) != HE_OK) return HE_EINVAL;
    int rc = grow(s, he_layer_workspace_bytes(ly, B));
    if (rc != HE_OK) return rc;
    s->steps.push_back({info.kind, ly, B, d_c0, d_sh, d_sh_next, d_out});
    return HE_OK;
}

int he_seq_run(he_seq *s, void *stream) {
    if (!s) return HE_EINVAL;
    return run_steps(s, (hipStream_t)stream);
}

int he_seq_capture(he_seq *s, void *stream) {
    if (!s || !stream) return HE_EINVAL;   // the null stream cannot be captured
    if (s->exec) return HE_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    // no timing events inside a graph: timing is suppressed on this thread during the capture
    // only, so the context's profiling setting is left as the caller set it
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return HE_EDEVICE;
    const bool was = he_prof_suppress(true);
    int rc = run_steps(s, st);
    he_prof_suppress(was);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    if (rc != HE_OK) {
        if (g) hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess || !g) return HE_EDEVICE;
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        hipGraphDestroy(g);
        return HE_EDEVICE;
    }
    s->graph = g;
    s->exec = x;
    return HE_OK;
}

int he_seq_replay(he_seq *s, void *stream) {
    if (!s || !s->exec) return HE_EINVAL;
    return hipGraphLaunch(s->exec, (hipStream_t)stream) == hipSuccess ? HE_OK : HE_EDEVICE;
}

uint32_t he_seq_length(const he_seq *s) { return s ? (uint32_t)s->steps.size() : 0; }

void he_seq_free(he_seq *s) {
    if (!s) return;
    if (s->exec) hipGraphExecDestroy(s->exec);
    if (s->graph) hipGraphDestroy(s->graph);
    if (s->ws) hipFree(s->ws);
    if (s->sync) hipFree(s->sync);
    delete s;
}

}  // extern "C"
