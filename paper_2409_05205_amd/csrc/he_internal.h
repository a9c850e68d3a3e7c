// Library-internal entry points shared by the runtime (he_runtime.hip) and the server
// (he_server.hip); not part of the C ABI.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "../../include/he.h"

// A conv or FC layer call (kind taken from the layer) on a caller workspace, with an explicit
// sync block for the one-launch form: FZ_SYNC_WORDS zeroed words that no concurrent call uses
// (null: the multi-launch forms).  Arguments otherwise as he_conv_layer_ws / he_fc_layer_ws.
int he_layer_call_sync(he_ctx *ctx, const he_layer *ly, uint32_t B, const uint32_t *d_c0, const uint32_t *d_sh,
                       const uint32_t *d_sh_next, uint32_t *d_out, void *d_ws, size_t ws_bytes, uint32_t *sync,
                       void *stream);

// Allocate one zeroed sync block on the current device (hipMalloc + hipMemset); null on failure.
uint32_t *he_sync_block_alloc();
