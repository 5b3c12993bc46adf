// Serving form: a request loop in front of the batched parser.
//
// A scheduler thread owns the device side:
//   admission  requests are admitted in arrival order while a slot is free
//              and their input and output blocks fit in the arena, a fixed
//              slice of HBM carved once at creation (serve_sched.h);
//   transfer   each admitted request's bytes go host -> device with
//              hipMemcpyAsync from the caller's pinned buffer on one of the
//              copy streams, round robin, and an event marks the end;
//   batching   whenever a compute stream is free, every request whose copy
//              has finished joins one batched launch (pp_batch_*) on it, so
//              requests that arrive while others are parsing join the next
//              launch, and copies overlap the parses;
//   completion the launch's result records come back to pinned host memory;
//              a request whose output capacity was too small is parsed again
//              with the exact sizes its result reports; the rest complete and
//              keep their outputs in the arena until the client releases them.
// Host and device meet only through events. Timestamps of device events are
// mapped onto the host's steady clock through a reference event recorded at
// creation.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "batch_internal.h"
#include "parparaw.h"
#include "serve_sched.h"

namespace {

using pp::sched::Core;
using pp::sched::Request;

constexpr int kMaxCopyStreams = 4;
constexpr int kMaxComputeStreams = 2;

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct DevPtrs {
    void* values[PP_MAX_COLUMNS];
    uint8_t* valid[PP_MAX_COLUMNS];
    int64_t* str_end[PP_MAX_COLUMNS];
};

struct Flight {
    pp_batch_t* batch = nullptr;
    std::vector<Request*> reqs;
    bool busy = false;
};

}  // namespace

struct pp_server {
    pp_server_config_t cfg{};
    std::vector<pp_dfa_t> dfas;
    int device = 0;
    char* d_arena = nullptr;
    char* d_bws[kMaxComputeStreams] = {};  // batch workspace per compute stream
    char* h_stage[kMaxComputeStreams] = {};  // pinned staging of a batch's descriptors, per compute stream
    size_t stage_bytes = 0;
    size_t bws_bytes = 0;
    hipStream_t copy[kMaxCopyStreams] = {};
    hipStream_t comp[kMaxComputeStreams] = {};
    hipEvent_t ev_base = nullptr;
    int64_t base_ns = 0;
    std::vector<hipEvent_t> ev_copy;  // per slot
    hipEvent_t ev_done[kMaxComputeStreams] = {};
    pp_result_t* h_results = nullptr;  // pinned, per slot
    std::vector<DevPtrs> ptrs;         // per slot
    Flight flights[kMaxComputeStreams];

    std::mutex mu;
    std::condition_variable cv;
    Core* core = nullptr;
    std::vector<Request*> copying;  // scheduler thread only
    std::thread th;
    std::atomic<bool> stop{false};
    std::atomic<int> hip_error{0};
    pp_server_stats_t stats{};
    int rr = 0;

    int64_t device_ns(hipEvent_t e)
    {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev_base, e) != hipSuccess) return now_ns();
        return base_ns + (int64_t)((double)ms * 1e6);
    }
    void fail(int code) { hip_error.store(code); }
    void loop();
    bool launch_batch(int s, std::vector<Request*>& reqs);
};

bool pp_server::launch_batch(int s, std::vector<Request*>& reqs)
{
    // build the batch; halve it until its workspace fits this stream's slice
    std::vector<pp_batch_item_t> items(reqs.size());
    for (size_t i = 0; i < reqs.size(); ++i) {
        Request* r = reqs[i];
        const auto& L = r->L;
        char* out = d_arena + r->out_off;
        DevPtrs& P = ptrs[(size_t)r->slot];
        for (int c = 0; c < r->ncols; ++c) {
            const bool skip = r->types[c] == PP_SKIP;
            P.values[c] = skip ? nullptr : out + L.values[c];
            P.valid[c] = skip ? nullptr : (uint8_t*)(out + L.valid[c]);
            P.str_end[c] = r->types[c] == PP_STRING ? (int64_t*)(out + L.str_end[c]) : nullptr;
        }
        pp_batch_item_t& it = items[i];
        it.d_in = (const uint8_t*)(d_arena + r->in_off);
        it.n = r->n;
        it.dialect = r->dialect;
        it.ncols = r->ncols;
        it.types = r->types;
        it.out.cap_records = r->cap_r;
        it.out.cap_fields = r->cap_f;
        it.out.d_record_offsets = (int64_t*)(out + L.rec);
        it.out.d_field_offsets = (int64_t*)(out + L.fld);
        it.out.d_column_ids = (int32_t*)(out + L.cid);
        it.out.d_values = P.values;
        it.out.d_valid = P.valid;
        it.out.d_str_end = P.str_end;
        it.out.d_result = (pp_result_t*)(out + L.result);
    }
    size_t take = items.size();
    pp_batch_t* b = nullptr;
    for (;;) {
        pp_status_t st = pp_batch_create(dfas.data(), (int32_t)dfas.size(), items.data(), (int32_t)take,
                                         &cfg.opts, &b);
        if (st != PP_OK) { fail(st); return false; }
        if (pp_batch_workspace_size(b) <= bws_bytes) break;
        pp_batch_destroy(b);
        b = nullptr;
        if (take == 1) { fail(PP_ERR_WORKSPACE); return false; }
        take = (take + 1) / 2;
    }
    // requests beyond what fits go back to the front of the ready queue
    if (take < reqs.size()) {
        std::lock_guard<std::mutex> g(mu);
        for (size_t i = reqs.size(); i-- > take;) core->unready_front(reqs[i]);
        reqs.resize(take);
    }
    // (stream s is idle: its previous batch, and the upload from its staging, have finished)
    if (pp::batch_bind_staged(b, d_bws[s], bws_bytes, h_stage[s], stage_bytes, comp[s]) != PP_OK ||
        pp_batch_launch(b, comp[s]) != PP_OK) {
        pp_batch_destroy(b);
        fail(PP_ERR_HIP);
        return false;
    }
    for (Request* r : reqs)
        if (hipMemcpyAsync(&h_results[r->slot], d_arena + r->out_off + r->L.result, sizeof(pp_result_t),
                           hipMemcpyDeviceToHost, comp[s]) != hipSuccess)
            fail(PP_ERR_HIP);
    if (hipEventRecord(ev_done[s], comp[s]) != hipSuccess) fail(PP_ERR_HIP);
    flights[s].batch = b;
    flights[s].reqs = reqs;
    flights[s].busy = true;
    {
        std::lock_guard<std::mutex> g(mu);
        stats.batches += 1;
        stats.batched_requests += (int64_t)reqs.size();
        if ((int64_t)reqs.size() > stats.max_batch) stats.max_batch = (int64_t)reqs.size();
    }
    return true;
}

void pp_server::loop()
{
    hipSetDevice(device);
    const size_t max_batch = cfg.max_batch > 0 ? (size_t)cfg.max_batch : (size_t)cfg.max_slots;
    while (!stop.load() && hip_error.load() == 0) {
        bool progress = false;
        // 1. admission (and re-allocation of overflowed outputs)
        std::vector<Request*> adm;
        {
            std::lock_guard<std::mutex> g(mu);
            adm = core->admit();
            const int64_t used = (int64_t)core->arena().used();
            if (used > stats.arena_peak_bytes) stats.arena_peak_bytes = used;
        }
        const int64_t t_adm = now_ns();
        for (Request* r : adm) {
            r->t_admit = t_adm;
            hipStream_t cs = copy[rr++ % cfg.copy_streams];
            if (r->n > 0 &&
                hipMemcpyAsync(d_arena + r->in_off, r->h_in, (size_t)r->n, hipMemcpyHostToDevice, cs) != hipSuccess)
                fail(PP_ERR_HIP);
            if (hipEventRecord(ev_copy[(size_t)r->slot], cs) != hipSuccess) fail(PP_ERR_HIP);
            copying.push_back(r);
            progress = true;
        }
        // 2. finished copies
        for (size_t i = 0; i < copying.size();) {
            Request* r = copying[i];
            const hipError_t q = hipEventQuery(ev_copy[(size_t)r->slot]);
            if (q == hipSuccess) {
                r->t_h2d = device_ns(ev_copy[(size_t)r->slot]);
                {
                    std::lock_guard<std::mutex> g(mu);
                    core->copied(r);
                }
                copying[i] = copying.back();
                copying.pop_back();
                progress = true;
            } else {
                if (q != hipErrorNotReady) fail(PP_ERR_HIP);
                ++i;
            }
        }
        // 3. finished batches
        for (int s = 0; s < cfg.compute_streams; ++s) {
            Flight& f = flights[s];
            if (!f.busy) continue;
            const hipError_t q = hipEventQuery(ev_done[s]);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) { fail(PP_ERR_HIP); break; }
            const int64_t t_done = device_ns(ev_done[s]);
            pp_batch_destroy(f.batch);
            f.batch = nullptr;
            f.busy = false;
            std::lock_guard<std::mutex> g(mu);
            for (Request* r : f.reqs) {
                r->result = h_results[r->slot];
                r->t_done = t_done;
                if (core->parsed(r)) {
                    stats.completed += 1;
                    stats.bytes_completed += r->n;
                } else {
                    stats.reparsed += 1;
                }
            }
            f.reqs.clear();
            progress = true;
            cv.notify_all();
        }
        // 4. new batches on free compute streams
        for (int s = 0; s < cfg.compute_streams; ++s) {
            if (flights[s].busy) continue;
            std::vector<Request*> reqs;
            {
                std::lock_guard<std::mutex> g(mu);
                reqs = core->take_ready(max_batch);
            }
            if (reqs.empty()) break;
            if (!launch_batch(s, reqs)) break;
            progress = true;
        }
        if (!progress) {
            std::unique_lock<std::mutex> lk(mu);
            bool gpu_work = !copying.empty();
            for (int s = 0; s < cfg.compute_streams; ++s) gpu_work = gpu_work || flights[s].busy;
            if (gpu_work)
                lk.unlock(), std::this_thread::sleep_for(std::chrono::microseconds(20));
            else
                cv.wait_for(lk, std::chrono::milliseconds(2));
        }
    }
    // drain what the device still runs before the owner frees memory
    for (int s = 0; s < cfg.compute_streams; ++s) {
        hipStreamSynchronize(comp[s]);
        if (flights[s].batch) pp_batch_destroy(flights[s].batch);
        flights[s].batch = nullptr;
        flights[s].busy = false;
    }
    for (int c = 0; c < cfg.copy_streams; ++c) hipStreamSynchronize(copy[c]);
    cv.notify_all();
}

static void server_free(pp_server* sv)
{
    if (!sv) return;
    for (int s = 0; s < kMaxComputeStreams; ++s) {
        if (sv->comp[s]) hipStreamDestroy(sv->comp[s]);
        if (sv->ev_done[s]) hipEventDestroy(sv->ev_done[s]);
    }
    for (int c = 0; c < kMaxCopyStreams; ++c)
        if (sv->copy[c]) hipStreamDestroy(sv->copy[c]);
    for (hipEvent_t e : sv->ev_copy)
        if (e) hipEventDestroy(e);
    if (sv->ev_base) hipEventDestroy(sv->ev_base);
    if (sv->h_results) hipHostFree(sv->h_results);
    for (int s = 0; s < kMaxComputeStreams; ++s)
        if (sv->h_stage[s]) hipHostFree(sv->h_stage[s]);
    if (sv->d_arena) hipFree(sv->d_arena);
    delete sv->core;
    delete sv;
}

extern "C" pp_status_t pp_server_create(const pp_server_config_t* cfg, const pp_dfa_t* dfas, int32_t ndfas,
                                        pp_server_t** out)
{
    if (!cfg || !out || !dfas || ndfas < 1) return PP_ERR_ARG;
    *out = nullptr;
    pp_server_config_t c = *cfg;
    if (c.copy_streams == 0) c.copy_streams = 4;  // several small copies in flight hide each one's setup
    if (c.compute_streams == 0) c.compute_streams = 2;
    if (c.max_slots <= 0 || c.copy_streams < 1 || c.copy_streams > kMaxCopyStreams || c.compute_streams < 1 ||
        c.compute_streams > kMaxComputeStreams || c.max_batch < 0 || c.hbm_budget_bytes < (64u << 20))
        return PP_ERR_ARG;
    {  // validates the DFAs and the launch shape
        pp_batch_t* probe = nullptr;
        pp_status_t st = pp_batch_create(dfas, ndfas, nullptr, 0, &c.opts, &probe);
        if (st != PP_OK) return st;
        pp_batch_destroy(probe);
    }
    pp_server* sv = new (std::nothrow) pp_server();
    if (!sv) return PP_ERR_ARG;
    sv->cfg = c;
    sv->dfas.assign(dfas, dfas + ndfas);
    if (hipGetDevice(&sv->device) != hipSuccess) { server_free(sv); return PP_ERR_HIP; }
    // Batch workspace per compute stream: descriptor tables plus 68 bytes
    // (lookback words and tile map entry) per work item, for a batch whose
    // inputs fill the whole budget at the smallest tile (4 KiB).
    const size_t budget = c.hbm_budget_bytes;
    sv->bws_bytes = pp::sched::align_up(
        (1u << 20) + (size_t)ndfas * 4096 + (size_t)c.max_slots * 4096 + (budget / 4096 + (size_t)c.max_slots) * 68);
    const size_t reserved = sv->bws_bytes * (size_t)c.compute_streams;
    if (reserved + (32u << 20) > budget) { server_free(sv); return PP_ERR_ARG; }
    const size_t arena = (budget - reserved) / pp::sched::kAlign * pp::sched::kAlign;
    sv->core = new (std::nothrow) Core(arena, c.max_slots);
    if (!sv->core) { server_free(sv); return PP_ERR_ARG; }
    if (hipMalloc((void**)&sv->d_arena, budget) != hipSuccess) {
        sv->d_arena = nullptr;
        server_free(sv);
        return PP_ERR_HIP;
    }
    for (int s = 0; s < c.compute_streams; ++s) sv->d_bws[s] = sv->d_arena + arena + (size_t)s * sv->bws_bytes;
    bool ok = true;
    for (int s = 0; s < c.compute_streams && ok; ++s)
        ok = hipStreamCreateWithFlags(&sv->comp[s], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreate(&sv->ev_done[s]) == hipSuccess;
    for (int k = 0; k < c.copy_streams && ok; ++k)
        ok = hipStreamCreateWithFlags(&sv->copy[k], hipStreamNonBlocking) == hipSuccess;
    sv->ev_copy.assign((size_t)c.max_slots, nullptr);
    for (int k = 0; k < c.max_slots && ok; ++k) ok = hipEventCreate(&sv->ev_copy[(size_t)k]) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&sv->h_results, sizeof(pp_result_t) * (size_t)c.max_slots) == hipSuccess;
    // descriptors of a batch: a few KiB per request plus 4 bytes per work item
    sv->stage_bytes = std::min<size_t>(sv->bws_bytes, (size_t)16 << 20);
    for (int s = 0; s < c.compute_streams && ok; ++s)
        ok = hipHostMalloc((void**)&sv->h_stage[s], sv->stage_bytes) == hipSuccess;
    ok = ok && hipEventCreate(&sv->ev_base) == hipSuccess && hipEventRecord(sv->ev_base, sv->comp[0]) == hipSuccess &&
         hipEventSynchronize(sv->ev_base) == hipSuccess;
    if (!ok) { server_free(sv); return PP_ERR_HIP; }
    sv->base_ns = now_ns();
    sv->ptrs.resize((size_t)c.max_slots);
    sv->th = std::thread([sv] { sv->loop(); });
    *out = sv;
    return PP_OK;
}

extern "C" pp_status_t pp_server_submit(pp_server_t* sv, const pp_server_request_t* rq, uint64_t* id)
{
    if (!sv || !rq || !id) return PP_ERR_ARG;
    if (rq->dialect < 0 || rq->dialect >= (int32_t)sv->dfas.size()) return PP_ERR_ARG;
    if (rq->ncols < 0 || rq->ncols > PP_MAX_COLUMNS || (rq->ncols > 0 && !rq->types)) return PP_ERR_SCHEMA;
    if (sv->hip_error.load()) return PP_ERR_HIP;
    Request r;
    r.h_in = rq->h_in;
    r.n = rq->n;
    r.dialect = rq->dialect;
    r.ncols = rq->ncols;
    if (rq->ncols > 0) memcpy(r.types, rq->types, sizeof(int32_t) * (size_t)rq->ncols);
    r.cap_r = rq->cap_records;
    r.cap_f = rq->cap_fields;
    r.t_arrival = now_ns();
    pp_status_t st;
    {
        std::lock_guard<std::mutex> g(sv->mu);
        st = sv->core->submit(r, id);
        if (st == PP_OK) sv->stats.submitted += 1;
    }
    sv->cv.notify_all();
    return st;
}

extern "C" pp_status_t pp_server_poll(pp_server_t* sv, pp_server_completion_t* out, int32_t max, int32_t* got)
{
    if (!sv || !got || max < 0 || (max > 0 && !out)) return PP_ERR_ARG;
    *got = 0;
    std::lock_guard<std::mutex> g(sv->mu);
    std::vector<Request*> done = sv->core->take_done((size_t)max);
    for (size_t i = 0; i < done.size(); ++i) {
        Request* r = done[i];
        pp_server_completion_t& c = out[i];
        memset(&c, 0, sizeof c);
        c.id = r->id;
        c.result = r->result;
        c.n = r->n;
        if (r->has_out) {
            char* o = sv->d_arena + r->out_off;
            const DevPtrs& P = sv->ptrs[(size_t)r->slot];
            c.out.cap_records = r->cap_r;
            c.out.cap_fields = r->cap_f;
            c.out.d_record_offsets = (int64_t*)(o + r->L.rec);
            c.out.d_field_offsets = (int64_t*)(o + r->L.fld);
            c.out.d_column_ids = (int32_t*)(o + r->L.cid);
            c.out.d_values = P.values;
            c.out.d_valid = P.valid;
            c.out.d_str_end = P.str_end;
            c.out.d_result = (pp_result_t*)(o + r->L.result);
        }
        c.t_arrival_ns = r->t_arrival;
        c.t_admit_ns = r->t_admit;
        c.t_h2d_done_ns = r->t_h2d;
        c.t_parse_done_ns = r->t_done;
    }
    *got = (int32_t)done.size();
    return sv->hip_error.load() ? PP_ERR_HIP : PP_OK;
}

extern "C" pp_status_t pp_server_release(pp_server_t* sv, uint64_t id)
{
    if (!sv) return PP_ERR_ARG;
    pp_status_t st;
    {
        std::lock_guard<std::mutex> g(sv->mu);
        st = sv->core->release(id);
    }
    sv->cv.notify_all();
    return st;
}

extern "C" pp_status_t pp_server_wait(pp_server_t* sv, int64_t timeout_us)
{
    if (!sv) return PP_ERR_ARG;
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv.wait_for(lk, std::chrono::microseconds(timeout_us > 0 ? timeout_us : 0),
                    [sv] { return sv->core->done_count() > 0 || sv->hip_error.load() != 0; });
    return sv->hip_error.load() ? PP_ERR_HIP : PP_OK;
}

extern "C" pp_status_t pp_server_get_stats(pp_server_t* sv, pp_server_stats_t* st)
{
    if (!sv || !st) return PP_ERR_ARG;
    std::lock_guard<std::mutex> g(sv->mu);
    *st = sv->stats;
    st->arena_bytes = (int64_t)sv->core->arena().capacity();
    st->arena_used_bytes = (int64_t)sv->core->arena().used();
    st->pending = (int64_t)sv->core->pending_count();
    st->hip_error = sv->hip_error.load();
    return PP_OK;
}

extern "C" void pp_server_destroy(pp_server_t* sv)
{
    if (!sv) return;
    sv->stop.store(true);
    sv->cv.notify_all();
    if (sv->th.joinable()) sv->th.join();
    server_free(sv);
}
