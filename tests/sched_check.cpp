// CPU checks of the serving loop's host bookkeeping (serve_sched.h): the
// arena against a byte-map model, and admission, batching, re-parse and
// release driven by simulated device completions. Prints "ok <name>" per
// check and exits nonzero on the first failure.
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <set>
#include <vector>

#include "serve_sched.h"

using namespace pp::sched;

#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #c); \
            exit(1);                                                    \
        }                                                               \
    } while (0)

// Random alloc/free against a model that marks every owned 256-byte unit:
// blocks never overlap, stay in bounds, used() is exact, and after freeing
// everything the arena is one free block again.
static void arena_model()
{
    std::mt19937_64 rng(7);
    const uint64_t cap = 1 << 20;
    Arena a(cap);
    std::vector<int> owner(cap / kAlign, -1);
    std::vector<std::pair<uint64_t, uint64_t>> live;  // off, len
    uint64_t used = 0;
    for (int step = 0; step < 20000; ++step) {
        if (live.empty() || rng() % 3) {
            const uint64_t want = 1 + rng() % (cap / 16);
            uint64_t off;
            const uint64_t len = align_up(want);
            // first fit in the model: lowest offset with len free units
            uint64_t expect = UINT64_MAX;
            for (uint64_t u = 0, run = 0; u < owner.size(); ++u) {
                run = owner[u] < 0 ? run + 1 : 0;
                if (run * kAlign == len) { expect = (u + 1 - run) * kAlign; break; }
            }
            const bool ok = a.alloc(want, &off);
            CHECK(ok == (expect != UINT64_MAX));
            if (!ok) continue;
            CHECK(off == expect);
            for (uint64_t u = off / kAlign; u < (off + len) / kAlign; ++u) {
                CHECK(owner[u] < 0);
                owner[u] = step;
            }
            live.push_back({off, len});
            used += len;
        } else {
            const size_t k = rng() % live.size();
            auto [off, len] = live[k];
            CHECK(a.release(off));
            CHECK(!a.release(off));  // double free is refused
            for (uint64_t u = off / kAlign; u < (off + len) / kAlign; ++u) owner[u] = -1;
            live[k] = live.back();
            live.pop_back();
            used -= len;
        }
        CHECK(a.used() == used);
        CHECK(a.live_count() == live.size());
    }
    for (auto [off, len] : live) CHECK(a.release(off));
    CHECK(a.used() == 0 && a.free_count() == 1 && a.largest_free() == cap);
    printf("ok arena_model\n");
}

static Request req(int64_t n, int64_t cap_r, int64_t cap_f)
{
    Request r;
    static const uint8_t dummy = 0;
    r.h_in = &dummy;
    r.n = n;
    r.ncols = 2;
    r.types[0] = PP_INT64;
    r.types[1] = PP_STRING;
    r.cap_r = cap_r;
    r.cap_f = cap_f;
    return r;
}

static void finish(Core& c, Request* r, int64_t R, int64_t F)
{
    r->result = pp_result_t{};
    r->result.num_records = R;
    r->result.num_fields = F;
    r->result.status = (R > r->cap_r || F > r->cap_f) ? PP_RESULT_CAPACITY : PP_RESULT_OK;
}

// Admission is FIFO, bounded by slots and by the budget; a request that does
// not fit blocks those behind it until memory is released.
static void admission_fifo()
{
    const uint64_t fp = Core::footprint(100000, 100, 200, 2, req(0, 0, 0).types);
    Core c(fp * 3, 8);  // room for three requests of this size
    uint64_t id[5];
    for (int i = 0; i < 5; ++i) CHECK(c.submit(req(100000, 100, 200), &id[i]) == PP_OK);
    auto a = c.admit();
    CHECK(a.size() == 3 && a[0]->id == id[0] && a[1]->id == id[1] && a[2]->id == id[2]);
    CHECK(c.pending_count() == 2);
    CHECK(c.admit().empty());
    // a small request behind the big ones still waits its turn
    uint64_t small;
    CHECK(c.submit(req(10, 1, 2), &small) == PP_OK);
    CHECK(c.admit().empty());
    for (Request* r : a) c.copied(r);
    auto b = c.take_ready(16);
    CHECK(b.size() == 3);
    for (Request* r : b) {
        finish(c, r, 50, 100);
        CHECK(c.parsed(r));
    }
    // inputs are freed at completion, outputs stay until release; what the
    // freed inputs make room for is admitted, still in arrival order
    auto d = c.take_done(16);
    CHECK(d.size() == 3);
    CHECK(c.arena().used() < fp * 3 - 3 * 100000);
    std::vector<Request*> e = c.admit();
    CHECK(c.release(id[0]) == PP_OK);
    CHECK(c.release(id[0]) == PP_ERR_ARG);
    CHECK(c.release(id[1]) == PP_OK && c.release(id[2]) == PP_OK);
    for (Request* r : c.admit()) e.push_back(r);
    CHECK(e.size() == 3 && e[0]->id == id[3] && e[1]->id == id[4] && e[2]->id == small);
    printf("ok admission_fifo\n");
}

static void slots_bound()
{
    Core c(1ull << 30, 2);
    uint64_t id;
    for (int i = 0; i < 4; ++i) CHECK(c.submit(req(1000, 10, 20), &id) == PP_OK);
    auto a = c.admit();
    CHECK(a.size() == 2 && a[0]->slot != a[1]->slot);
    CHECK(c.admit().empty());
    c.copied(a[0]);
    auto b = c.take_ready(8);
    finish(c, b[0], 1, 2);
    CHECK(c.parsed(b[0]));
    CHECK(c.admit().empty());  // completed but not released: the slot is still held
    CHECK(c.release(b[0]->id) == PP_OK);
    auto d = c.admit();
    CHECK(d.size() == 1);
    printf("ok slots_bound\n");
}

static void budget_and_args()
{
    Core c(1 << 20, 4);
    uint64_t id;
    CHECK(c.submit(req(2 << 20, 1, 1), &id) == PP_ERR_BUDGET);
    CHECK(c.submit(req(-1, 1, 1), &id) == PP_ERR_ARG);
    Request bad = req(10, 1, 1);
    bad.types[1] = 99;
    CHECK(c.submit(bad, &id) == PP_ERR_SCHEMA);
    Request nul = req(10, 1, 1);
    nul.h_in = nullptr;
    CHECK(c.submit(nul, &id) == PP_ERR_ARG);
    CHECK(c.live_requests() == 0);
    printf("ok budget_and_args\n");
}

// Capacity overflow: the request is parsed again with the exact sizes, keeps
// its input and slot, and completes on the second pass.
static void reparse()
{
    Core c(1 << 24, 4);
    uint64_t id;
    CHECK(c.submit(req(5000, 2, 4), &id) == PP_OK);
    auto a = c.admit();
    c.copied(a[0]);
    auto b = c.take_ready(4);
    finish(c, b[0], 40, 80);
    CHECK(!c.parsed(b[0]));
    CHECK(b[0]->cap_r == 40 && b[0]->cap_f == 80 && b[0]->has_in);
    auto again = c.take_ready(4);
    CHECK(again.size() == 1 && again[0] == b[0]);
    finish(c, again[0], 40, 80);
    CHECK(c.parsed(again[0]));
    CHECK(c.take_done(4).size() == 1);
    CHECK(c.release(id) == PP_OK);
    CHECK(c.arena().used() == 0);
    // exact sizes beyond the whole budget: completes with CAPACITY, no outputs kept
    Core small(1 << 20, 2);
    CHECK(small.submit(req(1000, 1, 1), &id) == PP_OK);
    auto s = small.admit();
    small.copied(s[0]);
    auto t = small.take_ready(2);
    finish(small, t[0], 1 << 20, 1 << 22);
    CHECK(small.parsed(t[0]));
    CHECK(t[0]->result.status == PP_RESULT_CAPACITY);
    CHECK(small.release(id) == PP_OK && small.arena().used() == 0);
    printf("ok reparse\n");
}

// A long random schedule: every request completes exactly once, in-flight
// memory never exceeds the budget, and everything is freed at the end.
static void soak()
{
    std::mt19937_64 rng(11);
    const uint64_t budget = 64 << 20;
    Core c(budget, 16);
    std::set<uint64_t> open, completed;
    std::vector<Request*> inflight;
    int submitted = 0;
    for (int step = 0; step < 20000; ++step) {
        const int op = (int)(rng() % 4);
        if (op == 0 && submitted < 3000) {
            const int64_t n = (int64_t)(1 + rng() % (4 << 20));
            uint64_t id;
            const int64_t R = n / 50 + 1;
            const bool under = rng() % 5 == 0;  // a fifth give too small a capacity
            if (c.submit(req(n, under ? R / 2 : R, under ? R : 2 * R), &id) == PP_OK) {
                open.insert(id);
                ++submitted;
            }
        } else if (op == 1) {
            for (Request* r : c.admit()) c.copied(r);
        } else if (op == 2) {
            for (Request* r : c.take_ready(1 + rng() % 6)) inflight.push_back(r);
            while (!inflight.empty() && rng() % 2) {
                Request* r = inflight.back();
                inflight.pop_back();
                const int64_t R = r->n / 50 + 1;
                finish(c, r, R, 2 * R);
                c.parsed(r);
            }
        } else {
            for (Request* r : c.take_done(1 + rng() % 8)) {
                CHECK(r->result.status == PP_RESULT_OK);
                const uint64_t id = r->id;  // r is freed by release
                CHECK(!completed.count(id));
                completed.insert(id);
                CHECK(c.release(id) == PP_OK);
                open.erase(id);
            }
        }
        CHECK(c.arena().used() <= c.arena().capacity());
    }
    // drain
    for (int guard = 0; guard < 100000 && !open.empty(); ++guard) {
        for (Request* r : c.admit()) c.copied(r);
        for (Request* r : c.take_ready(64)) inflight.push_back(r);
        for (Request* r : inflight) {
            const int64_t R = r->n / 50 + 1;
            finish(c, r, R, 2 * R);
            c.parsed(r);
        }
        inflight.clear();
        for (Request* r : c.take_done(64)) {
            const uint64_t id = r->id;
            completed.insert(id);
            CHECK(c.release(id) == PP_OK);
            open.erase(id);
        }
    }
    CHECK(open.empty());
    CHECK((int)completed.size() == submitted);
    CHECK(c.arena().used() == 0 && c.live_requests() == 0 && c.free_slot_count() == 16);
    printf("ok soak %d requests\n", submitted);
}

int main()
{
    arena_model();
    admission_fifo();
    slots_bound();
    budget_and_args();
    reparse();
    soak();
    return 0;
}
