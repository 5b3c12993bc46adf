// Batched form: many independent buffers with their own dialects, schemas and
// outputs in one kernel launch (capturable in a HIP graph).
//
// The host builds descriptor tables once (pp_batch_create) and uploads them
// into the caller's workspace (pp_batch_bind):
//   [header: ticket counter, 256 B]
//   [byte tables per dialect, 4 KiB each]
//   [one BufDesc per buffer]
//   [column descriptors of all buffers]
//   [tile map: owning buffer of every (buffer, tile) work item]
//   [lookback words: kWordsPerTile per work item]
// A launch resets the counters, the lookback words and every buffer's result
// record (batch_init), then runs batch_tiles with one workgroup per work item,
// in two launches on the stream: buffers whose DFA has at most 4 states (one
// v_perm_b32 and one table dword per byte) first, then the others (8-state
// vectors). Work items are numbered buffer after buffer and tile after tile,
// the first class's buffers before the second's; each launch has its own
// ticket counter, and a workgroup takes the next ticket when it starts, so
// the tiles a work item waits on in its buffer's lookback carry smaller
// tickets and belong to workgroups that are already running.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "parparaw.h"
#include "batch_internal.h"
#include "dfa_check.h"
#include "tile.h"

namespace pp {

struct BufDesc {
    TileArgs a;
    int64_t tile_base;  // ticket of this buffer's first tile
};

struct BatchParams {
    unsigned int* counter;   // two ticket counters: <= 4-state launch, 8-state launch
    const BufDesc* bufs;
    const uint32_t* tilemap;
    int64_t first_tile;      // work items [first_tile, first_tile + total_tiles) of this launch
    int64_t total_tiles;
    int32_t count;
};

// A workgroup-uniform struct read from global memory into scalar registers
// (the compiler cannot prove descriptor memory unclobbered, so it would
// otherwise keep every field in vector registers).
template <class T>
__device__ __forceinline__ T load_uniform(const T* p)
{
    static_assert(sizeof(T) % 4 == 0, "dword-sized struct");
    T out;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(p);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k) dst[k] = __builtin_amdgcn_readfirstlane(src[k]);
    return out;
}

// One workgroup per (buffer, tile) work item. Each workgroup takes a ticket
// at start, so tickets follow start order and a tile only ever waits on
// tiles of its buffer with smaller tickets, which are already running. (A
// persistent loop over tickets was measured to raise register use from 105
// to 176 VGPRs, halving occupancy, for no gain.)
template <int NT, int B, bool NS8>
__global__ __launch_bounds__(NT, 4) void batch_tiles(BatchParams bp)
{
    __shared__ TileSmem<NT, B> sm;
    __shared__ uint32_t s_ticket;
    if (threadIdx.x == 0) s_ticket = atomicAdd(bp.counter + (NS8 ? 1 : 0), 1u);
    __syncthreads();
    // uniform across the workgroup: keep it (and the descriptor) in scalar registers
    const uint32_t tk = __builtin_amdgcn_readfirstlane(s_ticket);
    if ((int64_t)tk >= bp.total_tiles) return;
    const int64_t t = bp.first_tile + (int64_t)tk;
    const uint32_t buf = __builtin_amdgcn_readfirstlane(bp.tilemap[t]);
    const BufDesc d = load_uniform(&bp.bufs[buf]);
    const uint32_t local = (uint32_t)(t - d.tile_base);
    parse_tile<NT, B, NS8>(d.a, local, sm);
}

__global__ void batch_init(BatchParams bp, u64* words, size_t nwords)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = i; k < nwords; k += stride) words[k] = 0ull;
    for (size_t b = i; b < (size_t)bp.count; b += stride) {
        const TileArgs& a = bp.bufs[b].a;
        pp_result_t* r = a.result;
        r->first_invalid_offset = -1;
        r->num_conversion_errors = 0;
        r->num_ragged_records = 0;
        r->min_record_fields = -1;  // all ones: the unsigned minimum starts at its top
        r->max_record_fields = 0;
        r->num_records = 0;
        r->num_fields = 0;
        r->final_state = a.start_state;
        r->status = ((a.accept_mask >> a.start_state) & 1u) ? PP_RESULT_OK : PP_RESULT_NON_ACCEPTING_END;
        if (a.cap_records >= 0) a.record_offsets[0] = 0;
        if (a.cap_fields >= 0) a.field_offsets[0] = 0;
    }
    if (i == 0) {
        bp.counter[0] = 0u;
        bp.counter[1] = 0u;
    }
}

static pp_status_t batch_check_dfa(const pp_dfa_t* d) { return check_dfa_tables(d); }

// Per-byte rows: next state of every state, and (next*8 | tag<<6) of every
// state, one byte per state (Table 1's group rows expanded to bytes): one
// dword per byte for DFAs of at most 4 states, two (states 0-3, 4-7) for
// larger ones.
static void build_tables(const pp_dfa_t* d, uint32_t* t)
{
    const bool ns8 = d->num_states > 4;
    memset(t, 0, 1024 * sizeof(uint32_t));
    for (int b = 0; b < 256; ++b) {
        const int g = d->group_of[b];
        uint32_t lo = 0, hi = 0, clo = 0, chi = 0;
        for (int s = 0; s < 8; ++s) {
            const bool real = s < d->num_states;
            const uint32_t nx = real ? d->next[g][s] : (uint32_t)s;
            const uint32_t tg = real ? d->tag[g][s] : 0u;
            const uint32_t cb = (nx * 8u) | (tg << 6);
            if (s < 4) { lo |= nx << (8 * s); clo |= cb << (8 * s); }
            else { hi |= nx << (8 * (s - 4)); chi |= cb << (8 * (s - 4)); }
        }
        if (ns8) {
            t[2 * b] = lo;
            t[2 * b + 1] = hi;
            t[512 + 2 * b] = clo;
            t[512 + 2 * b + 1] = chi;
        } else {
            t[b] = lo;
            t[512 + b] = clo;
        }
    }
}

}  // namespace pp

using namespace pp;

struct pp_batch {
    int nt, b;
    int32_t count, ndfas;
    int64_t total_tiles;
    int64_t tiles4;  // work items of buffers whose DFA has at most 4 states (numbered first)
    size_t off_tables, off_bufs, off_cols, off_map, off_words, ws_size;
    std::vector<pp_dfa_t> dfas;
    std::vector<BufDesc> bufs;     // device pointers filled in at bind
    std::vector<ColDesc> cols;
    std::vector<int64_t> col_base;  // first column descriptor of each buffer
    std::vector<uint32_t> tilemap;
    std::vector<uint32_t> tables;
    std::vector<char> blob;         // host image of the descriptor part of the workspace
    void* d_ws = nullptr;
};

struct pp_batch_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

extern "C" pp_status_t pp_batch_create(const pp_dfa_t* dfas, int32_t ndfas, const pp_batch_item_t* items,
                                       int32_t count, const pp_options_t* opts, pp_batch_t** out)
{
    if (!out || ndfas < 1 || count < 0 || (count > 0 && !items) || !dfas) return PP_ERR_ARG;
    *out = nullptr;
    int nt = 512, b = 64;
    if (opts && opts->block_threads) nt = opts->block_threads;
    if (opts && opts->bytes_per_thread) b = opts->bytes_per_thread;
    if (opts && opts->tile_order != 0) return PP_ERR_ARG;  // tiles of a batch go in order
    if (!((nt == 512 && b == 64) || (nt == 256 && b == 64) || (nt == 256 && b == 32) || (nt == 512 && b == 32) ||
          (nt == 256 && b == 16)))
        return PP_ERR_ARG;
    for (int d = 0; d < ndfas; ++d) {
        pp_status_t st = batch_check_dfa(&dfas[d]);
        if (st != PP_OK) return st;
    }
    pp_batch* bt = new (std::nothrow) pp_batch();
    if (!bt) return PP_ERR_ARG;
    bt->nt = nt;
    bt->b = b;
    bt->count = count;
    bt->ndfas = ndfas;
    bt->dfas.assign(dfas, dfas + ndfas);
    bt->tables.resize((size_t)ndfas * 1024);
    for (int d = 0; d < ndfas; ++d) build_tables(&dfas[d], &bt->tables[(size_t)d * 1024]);
    const int64_t tb = (int64_t)nt * b;
    int64_t tiles = 0;
    bt->bufs.resize(count);
    bt->col_base.resize(count);
    for (int i = 0; i < count; ++i) {
        const pp_batch_item_t& it = items[i];
        const pp_outputs_t& o = it.out;
        pp_status_t st = PP_OK;
        if (it.n < 0 || (it.n > 0 && !it.d_in) || it.dialect < 0 || it.dialect >= ndfas) st = PP_ERR_ARG;
        else if (it.ncols < 0 || it.ncols > PP_MAX_COLUMNS || (it.ncols > 0 && !it.types)) st = PP_ERR_SCHEMA;
        else if (o.cap_records < 0 || o.cap_fields < 0 || !o.d_record_offsets || !o.d_field_offsets ||
                 !o.d_result || (o.cap_fields > 0 && !o.d_column_ids))
            st = PP_ERR_ARG;
        else if (it.n >= (1ll << 55)) st = PP_ERR_UNSUPPORTED;
        if (st != PP_OK) { delete bt; return st; }
        bt->col_base[i] = (int64_t)bt->cols.size();
        for (int c = 0; c < it.ncols; ++c) {
            const int32_t ty = it.types[c];
            if (ty < PP_INT64 || ty > PP_SKIP) { delete bt; return PP_ERR_SCHEMA; }
            ColDesc cd;
            memset(&cd, 0, sizeof cd);
            cd.type = ty;
            if (ty != PP_SKIP && o.cap_records > 0) {
                if (!o.d_values || !o.d_valid || !o.d_values[c] || !o.d_valid[c] ||
                    (ty == PP_STRING && (!o.d_str_end || !o.d_str_end[c]))) {
                    delete bt;
                    return PP_ERR_ARG;
                }
                cd.values = o.d_values[c];
                cd.valid = o.d_valid[c];
                cd.str_end = ty == PP_STRING ? o.d_str_end[c] : nullptr;
            }
            bt->cols.push_back(cd);
        }
        const pp_dfa_t& d = dfas[it.dialect];
        BufDesc& bd = bt->bufs[i];
        memset(&bd, 0, sizeof bd);
        TileArgs& a = bd.a;
        a.in = it.d_in;
        a.n = it.n;
        a.cap_records = o.cap_records;
        a.cap_fields = o.cap_fields;
        a.record_offsets = o.d_record_offsets;
        a.field_offsets = o.d_field_offsets;
        a.column_ids = o.d_column_ids;
        a.result = o.d_result;
        a.ctl_out = o.d_control_bitmap;
        a.ncols = it.ncols;
        a.num_states = d.num_states;
        a.start_state = d.start_state;
        a.invalid_state = d.invalid_state;
        a.accept_mask = d.accept_mask;
        a.num_tiles = (int32_t)((it.n + tb - 1) / tb);
        // the dialect index travels in the tables pointer, fixed up at bind
        a.tables = reinterpret_cast<const uint32_t*>((uintptr_t)it.dialect);
    }
    // work items: the buffers of <= 4-state DFAs first, then the others
    for (int pass = 0; pass < 2; ++pass) {
        for (int i = 0; i < count; ++i) {
            BufDesc& bd = bt->bufs[i];
            if ((bd.a.num_states > 4) != (pass == 1)) continue;
            bd.tile_base = tiles;
            tiles += bd.a.num_tiles;
        }
        if (pass == 0) bt->tiles4 = tiles;
    }
    // one workgroup per work item; the dispatch counts work-items in 32 bits
    if (tiles * nt > 0xffffffffll) { delete bt; return PP_ERR_UNSUPPORTED; }
    bt->total_tiles = tiles;
    bt->tilemap.resize((size_t)tiles);
    for (int i = 0; i < count; ++i)
        for (int64_t k = 0; k < bt->bufs[i].a.num_tiles; ++k) bt->tilemap[(size_t)(bt->bufs[i].tile_base + k)] = i;
    size_t off = 256;
    bt->off_tables = off;
    off = align_up(off + (size_t)ndfas * 4096, 256);
    bt->off_bufs = off;
    off = align_up(off + (size_t)count * sizeof(BufDesc), 256);
    bt->off_cols = off;
    off = align_up(off + bt->cols.size() * sizeof(ColDesc), 256);
    bt->off_map = off;
    off = align_up(off + (size_t)tiles * sizeof(uint32_t), 256);
    bt->off_words = off;
    off += (size_t)tiles * kWordsPerTile * sizeof(u64);
    bt->ws_size = off;
    *out = bt;
    return PP_OK;
}

extern "C" size_t pp_batch_workspace_size(const pp_batch_t* bt) { return bt ? bt->ws_size : 0; }

extern "C" int64_t pp_batch_num_tiles(const pp_batch_t* bt) { return bt ? bt->total_tiles : -1; }

extern "C" pp_status_t pp_batch_bind(pp_batch_t* bt, void* d_ws, size_t ws_bytes, void* stream)
{
    return pp::batch_bind_staged(bt, d_ws, ws_bytes, nullptr, 0, stream);
}

pp_status_t pp::batch_bind_staged(pp_batch_t* bt, void* d_ws, size_t ws_bytes, void* h_stage, size_t stage_bytes,
                                  void* stream)
{
    if (!bt || !d_ws || !ws_aligned(d_ws)) return PP_ERR_ARG;
    if (ws_bytes < bt->ws_size) return PP_ERR_WORKSPACE;
    char* ws = (char*)d_ws;
    // descriptors with device pointers into this workspace
    std::vector<BufDesc> bufs = bt->bufs;
    for (int i = 0; i < bt->count; ++i) {
        TileArgs& a = bufs[i].a;
        const uintptr_t dialect = (uintptr_t)a.tables;
        a.tables = (const uint32_t*)(ws + bt->off_tables + dialect * 4096);
        a.cols = (const ColDesc*)(ws + bt->off_cols) + bt->col_base[i];
        a.words = (u64*)(ws + bt->off_words) + (size_t)bufs[i].tile_base * kWordsPerTile;
    }
    bt->blob.assign(bt->off_words, 0);
    memcpy(bt->blob.data() + bt->off_tables, bt->tables.data(), bt->tables.size() * sizeof(uint32_t));
    if (!bufs.empty()) memcpy(bt->blob.data() + bt->off_bufs, bufs.data(), bufs.size() * sizeof(BufDesc));
    if (!bt->cols.empty()) memcpy(bt->blob.data() + bt->off_cols, bt->cols.data(), bt->cols.size() * sizeof(ColDesc));
    if (!bt->tilemap.empty())
        memcpy(bt->blob.data() + bt->off_map, bt->tilemap.data(), bt->tilemap.size() * sizeof(uint32_t));
    // from pinned staging when the caller has some (an asynchronous copy),
    // else from the batch's own pageable copy
    const void* src = bt->blob.data();
    if (h_stage && stage_bytes >= bt->blob.size()) {
        memcpy(h_stage, bt->blob.data(), bt->blob.size());
        src = h_stage;
    }
    if (hipMemcpyAsync(d_ws, src, bt->blob.size(), hipMemcpyHostToDevice, (hipStream_t)stream) != hipSuccess)
        return PP_ERR_HIP;
    bt->d_ws = d_ws;
    return PP_OK;
}

template <bool NS8>
static void launch_batch(const pp_batch_t* bt, const BatchParams& bp, hipStream_t s)
{
    const dim3 grid((unsigned)bp.total_tiles);
    if (bt->nt == 512 && bt->b == 64) hipLaunchKernelGGL((batch_tiles<512, 64, NS8>), grid, dim3(512), 0, s, bp);
    else if (bt->nt == 256 && bt->b == 64) hipLaunchKernelGGL((batch_tiles<256, 64, NS8>), grid, dim3(256), 0, s, bp);
    else if (bt->nt == 256 && bt->b == 32) hipLaunchKernelGGL((batch_tiles<256, 32, NS8>), grid, dim3(256), 0, s, bp);
    else if (bt->nt == 512 && bt->b == 32) hipLaunchKernelGGL((batch_tiles<512, 32, NS8>), grid, dim3(512), 0, s, bp);
    else hipLaunchKernelGGL((batch_tiles<256, 16, NS8>), grid, dim3(256), 0, s, bp);
}

extern "C" pp_status_t pp_batch_launch(const pp_batch_t* bt, void* stream)
{
    if (!bt || !bt->d_ws) return PP_ERR_ARG;
    char* ws = (char*)bt->d_ws;
    BatchParams bp;
    bp.counter = (unsigned int*)ws;
    bp.bufs = (const BufDesc*)(ws + bt->off_bufs);
    bp.tilemap = (const uint32_t*)(ws + bt->off_map);
    bp.first_tile = 0;
    bp.total_tiles = bt->total_tiles;
    bp.count = bt->count;
    hipStream_t s = (hipStream_t)stream;
    const size_t nwords = (size_t)bt->total_tiles * kWordsPerTile;
    const size_t work = std::max<size_t>(nwords, (size_t)bt->count);
    const int init_blocks = (int)std::min<size_t>(1024, std::max<size_t>(1, (work + 255) / 256));
    hipLaunchKernelGGL(batch_init, dim3(init_blocks), dim3(256), 0, s, bp, (u64*)(ws + bt->off_words), nwords);
    if (hipGetLastError() != hipSuccess) return PP_ERR_HIP;
    // <= 4-state buffers, then the others (each launch only if it has work)
    for (int cls = 0; cls < 2; ++cls) {
        bp.first_tile = cls ? bt->tiles4 : 0;
        bp.total_tiles = cls ? bt->total_tiles - bt->tiles4 : bt->tiles4;
        if (bp.total_tiles == 0) continue;
        if (cls == 0) launch_batch<false>(bt, bp, s);
        else launch_batch<true>(bt, bp, s);
        if (hipGetLastError() != hipSuccess) return PP_ERR_HIP;
    }
    return PP_OK;
}

extern "C" pp_status_t pp_batch_graph_create(const pp_batch_t* bt, pp_batch_graph_t** out)
{
    if (!bt || !out || !bt->d_ws) return PP_ERR_ARG;
    *out = nullptr;
    pp_batch_graph* g = new (std::nothrow) pp_batch_graph();
    if (!g) return PP_ERR_ARG;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) { delete g; return PP_ERR_HIP; }
    pp_status_t st = PP_OK;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) st = PP_ERR_HIP;
    if (st == PP_OK) {
        st = pp_batch_launch(bt, s);
        hipGraph_t graph = nullptr;
        if (hipStreamEndCapture(s, &graph) != hipSuccess || !graph) st = PP_ERR_HIP;
        g->graph = graph;
    }
    if (st == PP_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) st = PP_ERR_HIP;
    hipStreamDestroy(s);
    if (st != PP_OK) {
        pp_batch_graph_destroy(g);
        return st;
    }
    *out = g;
    return PP_OK;
}

extern "C" pp_status_t pp_batch_graph_launch(pp_batch_graph_t* g, void* stream)
{
    if (!g || !g->exec) return PP_ERR_ARG;
    return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? PP_OK : PP_ERR_HIP;
}

extern "C" void pp_batch_graph_destroy(pp_batch_graph_t* g)
{
    if (!g) return;
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    delete g;
}

extern "C" void pp_batch_destroy(pp_batch_t* bt) { delete bt; }
