// Library-internal entry of the batched form (not part of the C ABI).
#pragma once
#include <stddef.h>

#include "parparaw.h"

namespace pp {

// pp_batch_bind with pinned host staging for the descriptor upload: when
// stage_bytes holds the descriptors, they are copied there first so the
// upload is asynchronous; the staging must stay untouched until the copy has
// run on `stream`. NULL staging: the same as pp_batch_bind.
pp_status_t batch_bind_staged(pp_batch_t* bt, void* d_ws, size_t ws_bytes, void* h_stage, size_t stage_bytes,
                              void* stream);

}  // namespace pp
