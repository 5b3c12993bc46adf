// Launch-shape autotuner: times every supported (block threads x bytes per
// thread) shape on the caller's own workload with HIP events and reports the
// fastest. The shape sets the chunk size of Sec. 3.1 (bytes per thread) and
// the tile of the single-pass scan (threads x bytes), so it trades the work
// of the multi-state simulation and tagging against lookback depth and
// occupancy; which side wins depends on the input sizes and dialects, hence
// measuring instead of a fixed rule.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>

#include "parparaw.h"

namespace {

const pp_options_t kShapes[PP_NUM_SHAPES] = {{64, 512}, {64, 256}, {32, 512}, {32, 256}, {16, 256}};

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    bool ok = false;
    Timer() { ok = hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess; }
    ~Timer()
    {
        if (a) hipEventDestroy(a);
        if (b) hipEventDestroy(b);
    }
};

// Mean milliseconds of `reps` calls of launch() after `warmup` untimed ones.
template <class F>
pp_status_t time_it(F&& launch, hipStream_t s, int warmup, int reps, float* ms)
{
    Timer t;
    if (!t.ok) return PP_ERR_HIP;
    for (int i = 0; i < warmup; ++i) {
        pp_status_t st = launch();
        if (st != PP_OK) return st;
    }
    if (hipEventRecord(t.a, s) != hipSuccess) return PP_ERR_HIP;
    for (int i = 0; i < reps; ++i) {
        pp_status_t st = launch();
        if (st != PP_OK) return st;
    }
    if (hipEventRecord(t.b, s) != hipSuccess || hipEventSynchronize(t.b) != hipSuccess) return PP_ERR_HIP;
    float total = 0.f;
    if (hipEventElapsedTime(&total, t.a, t.b) != hipSuccess) return PP_ERR_HIP;
    *ms = total / (float)reps;
    return PP_OK;
}

}  // namespace

extern "C" pp_status_t pp_shape(int32_t i, pp_options_t* out)
{
    if (i < 0 || i >= PP_NUM_SHAPES || !out) return PP_ERR_ARG;
    *out = kShapes[i];
    return PP_OK;
}

extern "C" size_t pp_autotune_workspace_size(int64_t n)
{
    size_t m = 0;
    for (const pp_options_t& o : kShapes) m = std::max(m, pp_workspace_size(n, &o));
    return m;
}

extern "C" pp_status_t pp_parse_autotune(const uint8_t* d_in, int64_t n, const pp_dfa_t* dfa,
                                         const pp_schema_t* schema, const pp_outputs_t* out, void* d_ws,
                                         size_t ws_bytes, int32_t reps, void* stream, pp_options_t* best,
                                         float* ms)
{
    if (!best || reps < 1) return PP_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    float best_ms = 0.f;
    int found = -1;
    for (int i = 0; i < PP_NUM_SHAPES; ++i) {
        const pp_options_t o = kShapes[i];
        if (ms) ms[i] = -1.f;
        if (pp_workspace_size(n, &o) > ws_bytes) continue;  // too small a workspace: shape skipped
        float t = 0.f;
        pp_status_t st = time_it([&] { return pp_parse(d_in, n, dfa, schema, out, d_ws, ws_bytes, &o, stream); },
                                 s, 1, reps, &t);
        if (st == PP_ERR_UNSUPPORTED) continue;
        if (st != PP_OK) return st;
        if (ms) ms[i] = t;
        if (found < 0 || t < best_ms) found = i, best_ms = t;
    }
    if (found < 0) return PP_ERR_WORKSPACE;
    *best = kShapes[found];
    return PP_OK;
}

extern "C" size_t pp_batch_autotune_workspace_size(const pp_dfa_t* dfas, int32_t ndfas, const pp_batch_item_t* items,
                                                   int32_t count)
{
    size_t m = 0;
    for (const pp_options_t& o : kShapes) {
        pp_batch_t* b = nullptr;
        if (pp_batch_create(dfas, ndfas, items, count, &o, &b) != PP_OK) continue;
        m = std::max(m, pp_batch_workspace_size(b));
        pp_batch_destroy(b);
    }
    return m;
}

extern "C" pp_status_t pp_batch_autotune(const pp_dfa_t* dfas, int32_t ndfas, const pp_batch_item_t* items,
                                         int32_t count, void* d_ws, size_t ws_bytes, int32_t reps, void* stream,
                                         pp_options_t* best, float* ms)
{
    if (!best || reps < 1) return PP_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    float best_ms = 0.f;
    int found = -1;
    for (int i = 0; i < PP_NUM_SHAPES; ++i) {
        const pp_options_t o = kShapes[i];
        if (ms) ms[i] = -1.f;
        pp_batch_t* b = nullptr;
        pp_status_t st = pp_batch_create(dfas, ndfas, items, count, &o, &b);
        if (st == PP_ERR_UNSUPPORTED) continue;
        if (st != PP_OK) return st;
        if (pp_batch_workspace_size(b) > ws_bytes) {
            pp_batch_destroy(b);
            continue;
        }
        st = pp_batch_bind(b, d_ws, ws_bytes, stream);
        float t = 0.f;
        if (st == PP_OK) st = time_it([&] { return pp_batch_launch(b, stream); }, s, 1, reps, &t);
        // the descriptor upload of bind reads host memory owned by the batch:
        // finish the stream before the batch goes away
        if (hipStreamSynchronize(s) != hipSuccess && st == PP_OK) st = PP_ERR_HIP;
        pp_batch_destroy(b);
        if (st != PP_OK) return st;
        if (ms) ms[i] = t;
        if (found < 0 || t < best_ms) found = i, best_ms = t;
    }
    if (found < 0) return PP_ERR_WORKSPACE;
    *best = kShapes[found];
    return PP_OK;
}
