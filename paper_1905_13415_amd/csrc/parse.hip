// Single-buffer launch of the parse pipeline (pp_parse): one workgroup per
// tile, tiles handed out in start order by an atomic ticket so that every
// predecessor a tile waits on in the lookback is already running.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "parparaw.h"
#include "dfa_check.h"
#include "tile.h"

namespace pp {

// Kernel arguments: the tile arguments plus what parse_init needs to build
// the workspace (DFA group tables and column descriptors).
struct Params {
    TileArgs a;
    unsigned int* counter;  // tile ticket
    uint32_t tile_order;    // 0: tiles in ticket order; else a permutation within blocks of 64
    uint32_t* tables;       // workspace copy of the byte tables (a.tables)
    ColDesc* colws;         // workspace copy of the column descriptors (a.cols)
    uint8_t group_of[256];
    uint8_t next[PP_MAX_GROUPS][PP_MAX_STATES];
    uint8_t tag[PP_MAX_GROUPS][PP_MAX_STATES];
    ColDesc cols[PP_MAX_COLUMNS];
};

// workspace: [ticket counter | pad] [byte tables, 4 KiB] [column descriptors] [kWordsPerTile words per tile]
constexpr size_t kWsHeader = 256, kWsTables = 4096, kWsCols = PP_MAX_COLUMNS * sizeof(ColDesc);

template <int NT, int B, bool NS8, int SH>
__global__ __launch_bounds__(NT, 4) void parse_tiles(Params p)
{
    __shared__ TileSmem<NT, B> sm;
    __shared__ uint32_t s_ticket;
    if (threadIdx.x == 0) s_ticket = atomicAdd(p.counter, 1u);
    tile_setup<NT, B, NS8>(p.a, sm);  // in flight together with the ticket
    __syncthreads();
    uint32_t tile = s_ticket;
    if (p.tile_order) {
        // Diagnostic order: ticket i of a complete block of 64 tiles takes the
        // block's tile (a i + c) mod 64, a odd (a permutation). A tile waits
        // only on tiles of its own block and of earlier ones; once the earlier
        // blocks are done, the at most 63 workgroups holding tickets of its
        // block leave resident slots free for the rest of the block's tickets,
        // so with 64 or more workgroups resident every wait ends (the host
        // checks the compute-unit count).
        const uint32_t base = tile & ~63u;
        if (base + 64u <= (uint32_t)p.a.num_tiles)
            tile = base + (((2u * p.tile_order + 1u) * (tile & 63u) + 37u * p.tile_order) & 63u);
    }
    parse_tile<NT, B, NS8, false, SH>(p.a, tile, sm);
}

// Resets the workspace and the result before a parse; writes the outputs of
// an empty input. Plain stores only, so the pair of launches can be captured.
__global__ void parse_init(Params p, size_t nwords)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (size_t k = i; k < nwords; k += (size_t)gridDim.x * blockDim.x) p.a.words[k] = 0ull;
    if (i < (size_t)p.a.ncols) p.colws[i] = p.cols[i];
    if (i < 256) {
        // per-byte transition rows from the DFA's group table (Table 1 layout):
        // next state of every state, and (next*8 | tag<<6) of every state
        const uint32_t b = (uint32_t)i;
        const uint32_t g = p.group_of[b];
        uint32_t lo = 0, hi = 0, clo = 0, chi = 0;
        for (int s = 0; s < 8; ++s) {
            const bool real = s < p.a.num_states;
            const uint32_t nx = real ? p.next[g][s] : (uint32_t)s;
            const uint32_t tg = real ? p.tag[g][s] : 0u;
            const uint32_t cb = (nx * 8u) | (tg << 6);
            if (s < 4) { lo |= nx << (8 * s); clo |= cb << (8 * s); }
            else { hi |= nx << (8 * (s - 4)); chi |= cb << (8 * (s - 4)); }
        }
        if (p.a.num_states > 4) {
            p.tables[2 * b] = lo; p.tables[2 * b + 1] = hi;
            p.tables[512 + 2 * b] = clo; p.tables[512 + 2 * b + 1] = chi;
        } else {
            p.tables[b] = lo;
            p.tables[512 + b] = clo;
        }
    }
    if (i == 0) {
        *p.counter = 0u;
        pp_result_t* r = p.a.result;
        r->first_invalid_offset = -1;
        r->num_conversion_errors = 0;
        r->num_ragged_records = 0;
        r->min_record_fields = -1;  // all ones: the unsigned minimum starts at its top
        r->max_record_fields = 0;
        r->num_records = 0;
        r->num_fields = 0;
        r->final_state = p.a.start_state;
        r->status = ((p.a.accept_mask >> p.a.start_state) & 1u) ? PP_RESULT_OK : PP_RESULT_NON_ACCEPTING_END;
        if (p.a.record_offsets && p.a.cap_records >= 0) p.a.record_offsets[0] = 0;
        if (p.a.field_offsets && p.a.cap_fields >= 0) p.a.field_offsets[0] = 0;
    }
}

// ---- host side ------------------------------------------------------------------------

struct Shape {
    int nt, b;
};
constexpr Shape kShapes[] = {{512, 64}, {256, 64}, {256, 32}, {512, 32}, {256, 16}};
constexpr Shape kDefaultShape = {512, 64};

static bool shape_of(const pp_options_t* o, Shape* s)
{
    Shape r = kDefaultShape;
    if (o && o->block_threads) r.nt = o->block_threads;
    if (o && o->bytes_per_thread) r.b = o->bytes_per_thread;
    for (const Shape& k : kShapes)
        if (k.nt == r.nt && k.b == r.b) { *s = r; return true; }
    return false;
}

static pp_status_t check_dfa(const pp_dfa_t* d) { return check_dfa_tables(d); }

template <int NT, int B>
static void launch_tiles(const Params& p, bool ns8, int sh, int64_t tiles, hipStream_t s)
{
    const dim3 g((unsigned)tiles), b(NT);
    if (sh) {
        if (ns8) hipLaunchKernelGGL((parse_tiles<NT, B, true, 1>), g, b, 0, s, p);
        else hipLaunchKernelGGL((parse_tiles<NT, B, false, 1>), g, b, 0, s, p);
    } else {
        if (ns8) hipLaunchKernelGGL((parse_tiles<NT, B, true, 0>), g, b, 0, s, p);
        else hipLaunchKernelGGL((parse_tiles<NT, B, false, 0>), g, b, 0, s, p);
    }
}

// The typed values of the records whose field count differs from ncols
// become the column defaults (records within the record capacity; the
// record offsets give each record's field count).
__global__ void reject_ragged(TileArgs a)
{
    const int64_t R0 = a.result->num_records;
    const int64_t R = R0 < a.cap_records ? R0 : a.cap_records;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R; r += stride) {
        if (a.record_offsets[r + 1] - a.record_offsets[r] == a.ncols) continue;
        for (int c = 0; c < a.ncols; ++c) {
            const ColDesc cd = a.cols[c];
            if (cd.type == PP_SKIP) continue;
            ((int64_t*)cd.values)[r] = 0;  // 0 and 0.0 share the bit pattern
            cd.valid[r] = 0;
            if (cd.type == PP_STRING) cd.str_end[r] = 0;
        }
    }
}

}  // namespace pp

using namespace pp;

extern "C" size_t pp_workspace_size(int64_t n, const pp_options_t* opts)
{
    Shape sh;
    if (n < 0 || !shape_of(opts, &sh)) return 0;
    const int64_t tb = (int64_t)sh.nt * sh.b;
    const int64_t tiles = (n + tb - 1) / tb;
    return kWsHeader + kWsTables + kWsCols + (size_t)tiles * kWordsPerTile * sizeof(u64);
}

// The parse behind pp_parse, pp_parse_utf16 and pp_infer_columns (count_only:
// no outputs beyond the result record, never CAPACITY). n symbols of
// 1 << symsh bytes each.
static pp_status_t parse_impl(const uint8_t* d_in, int64_t n, int symsh, const pp_dfa_t* dfa, const pp_schema_t* schema,
                              const pp_outputs_t* out, void* d_ws, size_t ws_bytes, const pp_options_t* opts,
                              void* stream, bool count_only)
{
    if (n < 0 || (n > 0 && !d_in) || !schema || !out || !d_ws || !out->d_result) return PP_ERR_ARG;
    if (symsh && (((uintptr_t)d_in) & 1)) return PP_ERR_ARG;  // code units are 2-byte aligned
    if (!ws_aligned(d_ws)) return PP_ERR_ARG;
    Shape sh;
    if (!shape_of(opts, &sh)) return PP_ERR_ARG;
    if (out->cap_records < 0 || out->cap_fields < 0) return PP_ERR_ARG;
    if (!out->d_record_offsets || !out->d_field_offsets) return PP_ERR_ARG;
    if (out->cap_fields > 0 && !out->d_column_ids) return PP_ERR_ARG;
    if (n >= (1ll << (55 - symsh))) return PP_ERR_UNSUPPORTED;
    pp_status_t st = check_dfa(dfa);
    if (st != PP_OK) return st;
    if (schema->ncols < 0 || schema->ncols > PP_MAX_COLUMNS) return PP_ERR_SCHEMA;
    if (schema->ncols > 0 && !schema->types) return PP_ERR_SCHEMA;
    if (schema->flags & ~PP_SCHEMA_REJECT_RAGGED) return PP_ERR_SCHEMA;
    if (ws_bytes < pp_workspace_size(n, opts)) return PP_ERR_WORKSPACE;
    const int32_t order = opts ? opts->tile_order : 0;
    if (order < 0) return PP_ERR_ARG;
    if (order > 0) {  // permuted blocks need 64 workgroups resident (one per compute unit suffices)
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return PP_ERR_HIP;
        if (cus < 64) return PP_ERR_UNSUPPORTED;
    }

    Params p;
    memset(&p, 0, sizeof p);
    p.tile_order = (uint32_t)order;
    TileArgs& a = p.a;
    a.in = d_in;
    a.n = n;
    a.cap_records = out->cap_records;
    a.cap_fields = out->cap_fields;
    a.record_offsets = out->d_record_offsets;
    a.field_offsets = out->d_field_offsets;
    a.column_ids = out->d_column_ids;
    a.result = out->d_result;
    a.ctl_out = out->d_control_bitmap;
    p.counter = (unsigned int*)d_ws;
    p.tables = (uint32_t*)((char*)d_ws + kWsHeader);
    p.colws = (ColDesc*)((char*)d_ws + kWsHeader + kWsTables);
    a.tables = p.tables;
    a.cols = p.colws;
    a.words = (u64*)((char*)d_ws + kWsHeader + kWsTables + kWsCols);
    const int64_t tb = (int64_t)sh.nt * sh.b;
    const int64_t tiles = (n + tb - 1) / tb;
    // the dispatch counts work-items in 32 bits
    if (tiles * sh.nt > 0xffffffffll) return PP_ERR_UNSUPPORTED;
    a.num_tiles = (int32_t)tiles;
    a.ncols = schema->ncols;
    a.num_states = dfa->num_states;
    a.start_state = dfa->start_state;
    a.invalid_state = dfa->invalid_state;
    a.accept_mask = dfa->accept_mask;
    a.count_only = count_only ? 1 : 0;
    memcpy(p.group_of, dfa->group_of, 256);
    for (int g = 0; g < PP_MAX_GROUPS; ++g)
        for (int s = 0; s < PP_MAX_STATES; ++s) {
            const bool real = g < dfa->num_groups && s < dfa->num_states;
            p.next[g][s] = real ? dfa->next[g][s] : (uint8_t)(s < dfa->num_states ? s : 0);
            p.tag[g][s] = real ? dfa->tag[g][s] : 0;
        }
    for (int c = 0; c < schema->ncols; ++c) {
        const int32_t ty = schema->types[c];
        if (ty < PP_INT64 || ty > PP_SKIP) return PP_ERR_SCHEMA;
        p.cols[c].type = ty;
        if (ty == PP_SKIP) continue;
        if (out->cap_records > 0) {
            if (!out->d_values || !out->d_valid || !out->d_values[c] || !out->d_valid[c]) return PP_ERR_ARG;
            if (ty == PP_STRING && (!out->d_str_end || !out->d_str_end[c])) return PP_ERR_ARG;
            p.cols[c].values = out->d_values[c];
            p.cols[c].valid = out->d_valid[c];
            p.cols[c].str_end = ty == PP_STRING ? out->d_str_end[c] : nullptr;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    const size_t nwords = (size_t)tiles * kWordsPerTile;
    const int init_blocks = (int)std::min<size_t>(1024, std::max<size_t>(1, (nwords + 255) / 256));
    hipLaunchKernelGGL(parse_init, dim3(init_blocks), dim3(256), 0, s, p, nwords);
    if (hipGetLastError() != hipSuccess) return PP_ERR_HIP;
    if (tiles == 0) return PP_OK;
    const bool ns8 = dfa->num_states > 4;
    if (sh.nt == 512 && sh.b == 64) launch_tiles<512, 64>(p, ns8, symsh, tiles, s);
    else if (sh.nt == 256 && sh.b == 64) launch_tiles<256, 64>(p, ns8, symsh, tiles, s);
    else if (sh.nt == 256 && sh.b == 32) launch_tiles<256, 32>(p, ns8, symsh, tiles, s);
    else if (sh.nt == 512 && sh.b == 32) launch_tiles<512, 32>(p, ns8, symsh, tiles, s);
    else launch_tiles<256, 16>(p, ns8, symsh, tiles, s);
    if (hipGetLastError() != hipSuccess) return PP_ERR_HIP;
    if ((schema->flags & PP_SCHEMA_REJECT_RAGGED) && schema->ncols > 0 && out->cap_records > 0) {
        hipLaunchKernelGGL(reject_ragged, dim3(1024), dim3(256), 0, s, a);
        if (hipGetLastError() != hipSuccess) return PP_ERR_HIP;
    }
    return PP_OK;
}

extern "C" pp_status_t pp_parse(const uint8_t* d_in, int64_t n, const pp_dfa_t* dfa,
                                const pp_schema_t* schema, const pp_outputs_t* out, void* d_ws,
                                size_t ws_bytes, const pp_options_t* opts, void* stream)
{
    return parse_impl(d_in, n, 0, dfa, schema, out, d_ws, ws_bytes, opts, stream, false);
}

// UTF-16 text (Sec. 4.2): the same launch over code units, narrowed to bytes
// as the tiles are staged; positions come out as byte offsets.
extern "C" size_t pp_workspace_size_utf16(int64_t n_units, const pp_options_t* opts)
{
    return pp_workspace_size(n_units, opts);
}

extern "C" pp_status_t pp_parse_utf16(const uint16_t* d_in, int64_t n_units, const pp_dfa_t* dfa,
                                      const pp_schema_t* schema, const pp_outputs_t* out, void* d_ws,
                                      size_t ws_bytes, const pp_options_t* opts, void* stream)
{
    return parse_impl(reinterpret_cast<const uint8_t*>(d_in), n_units, 1, dfa, schema, out, d_ws, ws_bytes, opts,
                      stream, false);
}

extern "C" pp_status_t pp_infer_columns(const uint8_t* d_in, int64_t n, const pp_dfa_t* dfa, pp_result_t* d_result,
                                        void* d_ws, size_t ws_bytes, const pp_options_t* opts, void* stream)
{
    if (!d_ws || !d_result) return PP_ERR_ARG;
    // no outputs: capacities 0; the first entries of the offset arrays,
    // which the initialisation writes, go to spare words of the workspace
    // header (its first word is the tile ticket)
    pp_outputs_t o;
    memset(&o, 0, sizeof o);
    o.d_record_offsets = (int64_t*)((char*)d_ws + 128);
    o.d_field_offsets = (int64_t*)((char*)d_ws + 192);
    o.d_result = d_result;
    pp_schema_t sch = {0, 0, nullptr};
    return parse_impl(d_in, n, 0, dfa, &sch, &o, d_ws, ws_bytes, opts, stream, true);
}

// ---- entry point without allocation ---------------------------------------------
// The workspace of pp_parse_noalloc: one static device array per GPU the
// library runs on, held until the process ends. In host code `scratch` names
// a host-side stand-in, never the device memory: its device address is taken
// once per device (hipGetSymbolAddress, with that device current) and only
// that address is passed to kernels. parse_init clears every part of it the
// kernels read (tile ticket, lookback words; tables and column descriptors
// are rewritten) with plain stores, so a call needs no memset and leaves no
// state that the next call depends on.
namespace pp {
static __device__ __align__(256) uint8_t scratch[PP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch[kMaxDevices];

static pp_status_t scratch_of_current_device(void** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PP_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return PP_ERR_HIP;
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return PP_OK;
}
}  // namespace pp

extern "C" pp_status_t pp_parse_noalloc(const uint8_t* d_in, int64_t n, const pp_dfa_t* dfa,
                                        const pp_schema_t* schema, const pp_outputs_t* out,
                                        const pp_options_t* opts, void* stream)
{
    Shape sh;
    if (n < 0 || !shape_of(opts, &sh)) return PP_ERR_ARG;
    if (pp_workspace_size(n, opts) > PP_NOALLOC_SCRATCH_BYTES) return PP_ERR_WORKSPACE;
    void* ws = nullptr;
    const pp_status_t st = scratch_of_current_device(&ws);
    if (st != PP_OK) return st;
    return pp_parse(d_in, n, dfa, schema, out, ws, PP_NOALLOC_SCRATCH_BYTES, opts, stream);
}

extern "C" const char* pp_status_str(pp_status_t s)
{
    switch (s) {
    case PP_OK: return "ok";
    case PP_ERR_ARG: return "invalid argument";
    case PP_ERR_DFA: return "invalid DFA";
    case PP_ERR_SCHEMA: return "invalid schema";
    case PP_ERR_WORKSPACE: return "workspace too small";
    case PP_ERR_HIP: return "HIP launch failed";
    case PP_ERR_UNSUPPORTED: return "unsupported";
    case PP_ERR_BUDGET: return "larger than the device budget";
    }
    return "unknown status";
}
