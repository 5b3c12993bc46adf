// serve_sched.h -- host bookkeeping of the serving loop: a first-fit arena over a
// fixed device-memory budget, FIFO admission bounded by slots and budget, and
// the per-request state machine. No HIP calls: the device side (copies,
// batched launches, events) lives in serve.hip and drives this class, and a
// CPU test drives it with simulated completions.
#pragma once

#include <stdint.h>

#include <deque>
#include <map>
#include <memory>
#include <unordered_map>
#include <vector>

#include "parparaw.h"

namespace pp {
namespace sched {

constexpr uint64_t kAlign = 256;
inline uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, capacity): a free list ordered by offset,
// neighbours coalesced on free. Offsets and sizes are multiples of kAlign.
class Arena {
  public:
    explicit Arena(uint64_t capacity) : cap_(capacity / kAlign * kAlign)
    {
        if (cap_) free_[0] = cap_;
    }
    uint64_t capacity() const { return cap_; }
    uint64_t used() const { return used_; }
    // largest block that one allocation could get right now
    uint64_t largest_free() const
    {
        uint64_t m = 0;
        for (const auto& f : free_) m = f.second > m ? f.second : m;
        return m;
    }
    bool alloc(uint64_t bytes, uint64_t* off)
    {
        const uint64_t need = align_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            const uint64_t o = it->first, len = it->second;
            free_.erase(it);
            if (len > need) free_[o + need] = len - need;
            live_[o] = need;
            used_ += need;
            *off = o;
            return true;
        }
        return false;
    }
    // returns false for an offset that is not a live allocation
    bool release(uint64_t off)
    {
        auto lv = live_.find(off);
        if (lv == live_.end()) return false;
        uint64_t o = off, len = lv->second;
        live_.erase(lv);
        used_ -= len;
        auto next = free_.lower_bound(o);
        if (next != free_.end() && o + len == next->first) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == o) {
                prev->second += len;
                return true;
            }
        }
        free_[o] = len;
        return true;
    }
    size_t live_count() const { return live_.size(); }
    size_t free_count() const { return free_.size(); }

  private:
    uint64_t cap_;
    uint64_t used_ = 0;
    std::map<uint64_t, uint64_t> free_;           // offset -> length
    std::unordered_map<uint64_t, uint64_t> live_;  // offset -> length
};

// Byte layout of one request's output block (each part kAlign-aligned).
struct OutLayout {
    uint64_t rec = 0, fld = 0, cid = 0, result = 0;
    uint64_t values[PP_MAX_COLUMNS] = {}, valid[PP_MAX_COLUMNS] = {}, str_end[PP_MAX_COLUMNS] = {};
    uint64_t total = 0;
};

inline OutLayout out_layout(int64_t cap_r, int64_t cap_f, int ncols, const int32_t* types)
{
    OutLayout L;
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t at = o;
        o += align_up(bytes ? bytes : 1);
        return at;
    };
    L.result = take(sizeof(pp_result_t));
    L.rec = take((uint64_t)(cap_r + 1) * 8);
    L.fld = take((uint64_t)(cap_f + 1) * 8);
    L.cid = take((uint64_t)cap_f * 4);
    for (int c = 0; c < ncols; ++c) {
        if (types[c] == PP_SKIP) continue;
        L.values[c] = take((uint64_t)cap_r * 8);
        L.valid[c] = take((uint64_t)cap_r);
        if (types[c] == PP_STRING) L.str_end[c] = take((uint64_t)cap_r * 8);
    }
    L.total = o;
    return L;
}

enum class State { Pending, Copying, Ready, Parsing, Retry, Done };

struct Request {
    uint64_t id = 0;
    const uint8_t* h_in = nullptr;
    int64_t n = 0;
    int32_t dialect = 0;
    int32_t ncols = 0;
    int32_t types[PP_MAX_COLUMNS] = {};
    int64_t cap_r = 0, cap_f = 0;
    State st = State::Pending;
    int slot = -1;
    bool retried = false;
    uint64_t in_off = 0, out_off = 0;
    bool has_in = false, has_out = false;
    OutLayout L;
    pp_result_t result = {};
    int64_t t_arrival = 0, t_admit = 0, t_h2d = 0, t_done = 0;
};

// Admission and bookkeeping. Every call is made with the owner's lock held.
class Core {
  public:
    Core(uint64_t arena_bytes, int max_slots) : arena_(arena_bytes), free_slots_()
    {
        for (int s = max_slots - 1; s >= 0; --s) free_slots_.push_back(s);
    }
    Arena& arena() { return arena_; }

    // Footprint of a request: its input and its output block.
    static uint64_t footprint(int64_t n, int64_t cap_r, int64_t cap_f, int ncols, const int32_t* types)
    {
        return align_up((uint64_t)(n ? n : 1)) + out_layout(cap_r, cap_f, ncols, types).total;
    }

    // Validates and queues; PP_ERR_BUDGET when the request could never fit.
    pp_status_t submit(const Request& r, uint64_t* id)
    {
        if (r.n < 0 || r.cap_r < 0 || r.cap_f < 0 || r.ncols < 0 || r.ncols > PP_MAX_COLUMNS ||
            (r.n > 0 && !r.h_in))
            return PP_ERR_ARG;
        for (int c = 0; c < r.ncols; ++c)
            if (r.types[c] < PP_INT64 || r.types[c] > PP_SKIP) return PP_ERR_SCHEMA;
        if (footprint(r.n, r.cap_r, r.cap_f, r.ncols, r.types) > arena_.capacity()) return PP_ERR_BUDGET;
        auto q = std::make_unique<Request>(r);
        q->id = next_id_++;
        q->st = State::Pending;
        *id = q->id;
        pending_.push_back(q.get());
        all_[q->id] = std::move(q);
        return PP_OK;
    }

    // Re-allocates the output blocks of requests that overflowed their
    // capacity (oldest first); then admits pending requests in arrival order
    // while a slot is free and both blocks fit. A request that does not fit
    // blocks the ones behind it, so admission never reorders.
    std::vector<Request*> admit()
    {
        std::vector<Request*> now;
        while (!retry_.empty()) {
            Request* r = retry_.front();
            if (!alloc_out(r)) break;
            retry_.pop_front();
            r->st = State::Ready;
            ready_.push_back(r);
        }
        while (!pending_.empty() && !free_slots_.empty()) {
            Request* r = pending_.front();
            uint64_t in_off;
            if (!arena_.alloc((uint64_t)r->n, &in_off)) break;
            r->in_off = in_off;
            r->has_in = true;
            if (!alloc_out(r)) {
                arena_.release(in_off);
                r->has_in = false;
                break;
            }
            pending_.pop_front();
            r->slot = free_slots_.back();
            free_slots_.pop_back();
            r->st = State::Copying;
            now.push_back(r);
        }
        return now;
    }

    void copied(Request* r)
    {
        r->st = State::Ready;
        ready_.push_back(r);
    }

    // Ready requests in the order they became ready, at most max of them.
    std::vector<Request*> take_ready(size_t max)
    {
        std::vector<Request*> b;
        while (!ready_.empty() && b.size() < max) {
            Request* r = ready_.front();
            ready_.pop_front();
            r->st = State::Parsing;
            b.push_back(r);
        }
        return b;
    }
    size_t ready_count() const { return ready_.size(); }
    // puts a request taken by take_ready back at the front of the queue
    void unready_front(Request* r)
    {
        r->st = State::Ready;
        ready_.push_front(r);
    }

    // A parse ended with r->result filled in. Capacity overflow on the first
    // attempt re-parses with the exact sizes the result reports, if those fit
    // the budget at all; anything else completes the request (its input block
    // is freed, the outputs stay).
    // Returns true when the request completed.
    bool parsed(Request* r)
    {
        if (r->result.status == PP_RESULT_CAPACITY && !r->retried &&
            footprint(r->n, r->result.num_records, r->result.num_fields, r->ncols, r->types) <=
                arena_.capacity()) {
            r->retried = true;
            arena_.release(r->out_off);
            r->has_out = false;
            r->cap_r = r->result.num_records;
            r->cap_f = r->result.num_fields;
            if (alloc_out(r)) {
                r->st = State::Ready;
                ready_.push_back(r);
            } else {
                r->st = State::Retry;
                retry_.push_back(r);
            }
            return false;
        }
        if (r->has_in) arena_.release(r->in_off);
        r->has_in = false;
        r->st = State::Done;
        done_.push_back(r);
        return true;
    }

    // Completed requests not yet handed to the client, oldest first.
    std::vector<Request*> take_done(size_t max)
    {
        std::vector<Request*> v;
        while (!done_.empty() && v.size() < max) {
            v.push_back(done_.front());
            done_.pop_front();
        }
        return v;
    }

    // Frees a completed request's outputs and its slot.
    pp_status_t release(uint64_t id)
    {
        auto it = all_.find(id);
        if (it == all_.end() || it->second->st != State::Done) return PP_ERR_ARG;
        Request* r = it->second.get();
        for (auto d = done_.begin(); d != done_.end(); ++d)
            if (*d == r) {  // released before it was polled
                done_.erase(d);
                break;
            }
        if (r->has_out) arena_.release(r->out_off);
        free_slots_.push_back(r->slot);
        all_.erase(it);
        return PP_OK;
    }

    Request* find(uint64_t id)
    {
        auto it = all_.find(id);
        return it == all_.end() ? nullptr : it->second.get();
    }
    size_t pending_count() const { return pending_.size(); }
    size_t done_count() const { return done_.size(); }
    size_t live_requests() const { return all_.size(); }
    size_t free_slot_count() const { return free_slots_.size(); }
    bool idle() const { return pending_.empty() && ready_.empty() && retry_.empty(); }

  private:
    bool alloc_out(Request* r)
    {
        r->L = out_layout(r->cap_r, r->cap_f, r->ncols, r->types);
        uint64_t off;
        if (!arena_.alloc(r->L.total, &off)) return false;
        r->out_off = off;
        r->has_out = true;
        return true;
    }

    Arena arena_;
    std::vector<int> free_slots_;
    uint64_t next_id_ = 1;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> all_;
    std::deque<Request*> pending_, ready_, retry_, done_;
};

}  // namespace sched
}  // namespace pp
