// Single-pass parallel parse of delimiter-separated text on gfx950: the
// per-tile pipeline shared by the single-buffer and the batched kernels.
//
// One workgroup of NT threads owns a tile of NT*B input bytes; each thread
// owns a chunk of B bytes (the per-thread chunks of Sec. 3.1). Per tile, in
// one kernel:
//   1. stage the tile in LDS with 16-byte loads, after the 64 bytes that
//      precede it (where the tile's first field usually begins); every
//      thread keeps its chunk in registers;
//   2. multi-state pass (Sec. 3.1): per chunk, one DFA instance per state,
//      packed one byte per state in a register; a step is one v_perm_b32
//      (<= 4 states) or two (<= 8 states) that looks every instance up in
//      the byte's transition row: the chunk's state-transition vector;
//   3. exclusive composition scan ((a o b)_i = b[a_i], Sec. 3.1): wavefront
//      scan through DPP moves, block scan through LDS, device scan by
//      decoupled lookback (the single-pass scan the paper builds on, Sec. 2)
//      in which one wavefront polls 64 predecessor tiles at a time;
//   4. tag pass from the chunk's start state into register bitmaps of record
//      delimiters, field delimiters and control symbols (Sec. 3.1); it runs
//      under a guessed start state while the lookback is pending, and again
//      for chunks the guess got wrong;
//   5. record counts (+), field counts (+), column carries (the abs/rel
//      operator of Sec. 3.2) and the last delimiter position, scanned the
//      same way;
//   6. delimiter positions, column ids and record ends staged in LDS, then
//      written coalesced as field offsets, column ids and record offsets;
//   7. typed conversion (Sec. 3.3): a wavefront takes a block of 64 records
//      and a contiguous group of columns, a lane one record, and walks the
//      group's fields in order; every lane is at the same column, so the
//      type is wavefront-uniform and the stores into the typed column are
//      contiguous. This takes the place of the paper's radix-sort partition
//      by column tag: the (record, column) pair addresses the output slot
//      directly. The lanes of the first column group also count their
//      record's fields, for the fewest and most fields per record (column
//      count inference and validation, Sec. 4.3).
// Tiles with more fields or records than the LDS staging holds take a
// per-thread path for steps 6-7 that gives the same outputs.
//
// Symbols are bytes (SH = 0) or UTF-16 code units (SH = 1, Sec. 4.2). The
// DFAs' structural symbols are ASCII, and a code unit below 0x80 is that
// ASCII symbol while any other unit (both halves of a surrogate pair
// included) can only be data; so the staging narrows each unit to one byte
// (the unit itself below 0x80, else 0x80, which falls in the catch-all
// group) and the pipeline runs on one byte per symbol, with tiles and chunks
// holding whole code units by construction. Output positions are symbol
// indices shifted left by SH: byte offsets into the input either way.
// The input is read from HBM once; per-symbol metadata never leaves the chip;
// outputs are written with streaming stores.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "convert.h"
#include "convert_fast.h"
#include "parparaw.h"

namespace pp {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned long long u64;
constexpr uint32_t kTagControl = 1;

struct ColDesc {
    void* values;
    uint8_t* valid;
    int64_t* str_end;
    int32_t type;
    int32_t pad;
};

// Device pointers of the outputs and the input are plain (generic) pointers
// in the descriptors; at the access they are cast to the global address
// space so that loads and stores compile to global (not flat) instructions,
// which do not hold up waits on LDS results.
#define PP_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ PP_GLOBAL T* gptr(T* ptr)
{
    return (PP_GLOBAL T*)ptr;
}
template <class T>
__device__ __forceinline__ const PP_GLOBAL T* gptr(const T* ptr)
{
    return (const PP_GLOBAL T*)ptr;
}

// Element `idx` of an output array at a 32-bit byte offset from a
// wavefront-uniform base: the store takes the base in scalar registers and
// only the offset per lane. Outputs are never read back by the kernel, so
// the store is a streaming (nontemporal) one.
template <class T>
__device__ __forceinline__ void put(T* base, uint32_t idx, T v)
{
    PP_GLOBAL char* const g = reinterpret_cast<PP_GLOBAL char*>(gptr(base));
    uint32_t off = idx * (uint32_t)sizeof(T);
    // opaque here, so that the widening of the offset stays next to the store
    // and the store can take the scalar base with a 32-bit lane offset
    asm volatile("" : "+v"(off));
    __builtin_nontemporal_store(v, reinterpret_cast<PP_GLOBAL T*>(g + off));
}

// Everything one tile needs about its buffer, dialect and outputs.
struct TileArgs {
    const uint8_t* in;
    int64_t n;
    int64_t cap_records;
    int64_t cap_fields;
    int64_t* record_offsets;
    int64_t* field_offsets;
    int32_t* column_ids;
    pp_result_t* result;
    u64* words;              // kWordsPerTile lookback words per tile of this buffer
    const uint32_t* tables;  // 2 x 512 dwords: byte -> next states, byte -> (next*8 | tag<<6)
    const ColDesc* cols;     // ncols column descriptors
    int32_t num_tiles;
    int32_t ncols;
    int32_t num_states;
    int32_t start_state;
    int32_t invalid_state;
    uint32_t accept_mask;
    int32_t count_only;  // no outputs but the result record, whose status is then never CAPACITY
    uint32_t* ctl_out;   // optional control-symbol bitmap of the whole input (one bit per byte)
};



// ---- lookback words ----------------------------------------------------------
// Every word is self-contained, [status:2 | payload:62], written once per
// state by relaxed agent-scope atomics, so no ordering with other memory is
// needed. Aggregates and inclusive prefixes of the counts live in separate
// words: an aggregate is never overwritten, so a reader always finds either
// all four inclusive words or both aggregate words of a tile.
constexpr int kWordsPerTile = 8;
enum { W_STATE = 0, W_AGG0 = 1, W_AGG1 = 2, W_IREC = 3, W_IFLD = 4, W_ICOL = 5, W_ILAST = 6 };
constexpr u64 kAgg = 1ull << 62, kIncl = 2ull << 62;
constexpr u64 kPayload = (1ull << 62) - 1;
// inclusive payloads: col = abs:1 @61 | value; last = has:1 @61 | ctl:1 @60 |
// state after the delimiter:4 @56 | absolute position:56
constexpr u64 kColAbs = 1ull << 61;
constexpr u64 kColVal = kColAbs - 1;
constexpr u64 kLastHas = 1ull << 61, kLastCtl = 1ull << 60;
constexpr u64 kLastPos = (1ull << 56) - 1;

__device__ inline void publish(u64* w, u64 v)
{
    __hip_atomic_store(gptr(w), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline u64 peek(u64* w)
{
    return __hip_atomic_load(gptr(w), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline u64 ballot(bool x) { return __ballot(x); }

__device__ inline u64 shfl_xor64(u64 v, int d)
{
    uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, d);
    uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), d);
    return ((u64)hi << 32) | lo;
}

__device__ inline u64 readlane64(u64 v, int l)  // l wavefront-uniform
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((u64)hi << 32) | lo;
}

__device__ inline u64 readlane0_64(u64 v)
{
    // the builtin returns a signed int: take each half as unsigned before
    // widening, or a low half with bit 31 set would sign-extend over the high
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((u64)hi << 32) | lo;
}

// ---- state-transition vectors (Sec. 3.1) --------------------------------------
// Entry i (byte i) is the end state of the instance that started in state i.
// <= 4 states: one dword; <= 8 states: lo = states 0-3, hi = states 4-7.
template <bool NS8>
struct SV {
    uint32_t lo, hi;
};

template <bool NS8>
__device__ inline SV<NS8> sv_identity()
{
    return {0x03020100u, NS8 ? 0x07060504u : 0u};
}

// (a o b)_i = b[a_i]: v_perm_b32 picks byte sel of {src0:src1}, bytes 0-3
// from src1 and 4-7 from src0.
template <bool NS8>
__device__ inline SV<NS8> compose(SV<NS8> a, SV<NS8> b)
{
    SV<NS8> r;
    if constexpr (NS8) {
        r.lo = __builtin_amdgcn_perm(b.hi, b.lo, a.lo);
        r.hi = __builtin_amdgcn_perm(b.hi, b.lo, a.hi);
    } else {
        r.lo = __builtin_amdgcn_perm(0u, b.lo, a.lo);
        r.hi = 0;
    }
    return r;
}

template <bool NS8>
__device__ inline uint32_t sv_get(SV<NS8> v, uint32_t i)
{
    uint32_t w = (NS8 && i >= 4) ? v.hi : v.lo;
    return (w >> ((i & 3) * 8)) & 0xffu;
}

template <bool NS8>
__device__ inline uint32_t sv_to_nib(SV<NS8> v)
{
    uint32_t r = 0;
    for (int i = 0; i < 4; ++i) r |= ((v.lo >> (8 * i)) & 0xfu) << (4 * i);
    if constexpr (NS8)
        for (int i = 0; i < 4; ++i) r |= ((v.hi >> (8 * i)) & 0xfu) << (16 + 4 * i);
    return r;
}

template <bool NS8>
__device__ inline SV<NS8> sv_from_nib(uint32_t x)
{
    SV<NS8> v{0u, 0u};
    for (int i = 0; i < 4; ++i) v.lo |= ((x >> (4 * i)) & 0xfu) << (8 * i);
    if constexpr (NS8)
        for (int i = 0; i < 4; ++i) v.hi |= ((x >> (16 + 4 * i)) & 0xfu) << (8 * i);
    return v;
}

// The even bits of x into the low half and the odd bits into the high half,
// each in order (four swap steps of the standard bit de-interleave).
__device__ __forceinline__ uint32_t unzip_bits(uint32_t x)
{
    uint32_t t;
    t = (x ^ (x >> 1)) & 0x22222222u;
    x ^= t ^ (t << 1);
    t = (x ^ (x >> 2)) & 0x0C0C0C0Cu;
    x ^= t ^ (t << 2);
    t = (x ^ (x >> 4)) & 0x00F000F0u;
    x ^= t ^ (t << 4);
    t = (x ^ (x >> 8)) & 0x0000FF00u;
    x ^= t ^ (t << 8);
    return x;
}

// ---- wavefront scans through DPP -------------------------------------------------
// A DPP move reads another lane's register within the same instruction (no LDS
// round trip). Controls (GFX9 encoding): row_shr:n = 0x110 + n within rows of
// 16 lanes; row_bcast:15 = 0x142 (lane 15 of each row to the next row, rows
// 1 and 3 written); row_bcast:31 = 0x143 (lane 31 to rows 2 and 3);
// wave_shr:1 = 0x138. Lanes whose source is outside the row (or wave), and
// rows the row mask leaves out, keep `old`, which the scans pass as the
// operator's identity.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_move(uint32_t old, uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWS, 0xF, false);
}

template <int CTRL, int ROWS, bool NS8>
__device__ __forceinline__ SV<NS8> dpp_sv(SV<NS8> v)
{
    const SV<NS8> id = sv_identity<NS8>();
    SV<NS8> r;
    r.lo = dpp_move<CTRL, ROWS>(id.lo, v.lo);
    r.hi = NS8 ? dpp_move<CTRL, ROWS>(id.hi, v.hi) : 0u;
    return r;
}

// Inclusive composition scan over the lanes (lane order = chunk order).
template <bool NS8>
__device__ __forceinline__ SV<NS8> wave_scan_sv(SV<NS8> x)
{
    x = compose(dpp_sv<0x111, 0xF, NS8>(x), x);
    x = compose(dpp_sv<0x112, 0xF, NS8>(x), x);
    x = compose(dpp_sv<0x114, 0xF, NS8>(x), x);
    x = compose(dpp_sv<0x118, 0xF, NS8>(x), x);
    x = compose(dpp_sv<0x142, 0xA, NS8>(x), x);
    x = compose(dpp_sv<0x143, 0xC, NS8>(x), x);
    return x;
}

// The previous lane's value (identity in lane 0).
template <bool NS8>
__device__ __forceinline__ SV<NS8> wave_prev_sv(SV<NS8> x)
{
    return dpp_sv<0x138, 0xF, NS8>(x);
}

// Ordered reduction over the 64 lanes, higher lanes on the left (the
// lookback's lane l holds the tile l places further back): DPP row shifts
// towards lane 0 within each row of 16 (a lane whose source lies outside its
// row receives the identity), then the four row totals read from lanes 0,
// 16, 32 and 48. Every lane must be active. Returns the total (uniform).
template <bool NS8>
__device__ __forceinline__ SV<NS8> wave_reduce_desc_sv(SV<NS8> x)
{
    x = compose(dpp_sv<0x101, 0xF, NS8>(x), x);
    x = compose(dpp_sv<0x102, 0xF, NS8>(x), x);
    x = compose(dpp_sv<0x104, 0xF, NS8>(x), x);
    x = compose(dpp_sv<0x108, 0xF, NS8>(x), x);
    SV<NS8> r[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        r[k].lo = (uint32_t)__builtin_amdgcn_readlane((int)x.lo, 16 * k);
        r[k].hi = NS8 ? (uint32_t)__builtin_amdgcn_readlane((int)x.hi, 16 * k) : 0u;
    }
    return compose(compose(compose(r[3], r[2]), r[1]), r[0]);
}

// One DFA step through the combined table: state*8 -> next state*8.
template <bool NS8>
__device__ inline uint32_t step_state(const uint32_t* tcomb, uint32_t b, uint32_t s8)
{
    uint32_t x;
    if constexpr (NS8) x = __builtin_amdgcn_ubfe(tcomb[2 * b + (s8 >> 5)], s8 & 31u, 8);
    else x = __builtin_amdgcn_ubfe(tcomb[b], s8, 8);
    return x & 0x38u;
}

// ---- count scan element within a tile (Sec. 3.2) ---------------------------------
// nr: record delimiters; nf: delimiters (fields closed); col: column carry,
// bit 31 = abs; last: tile-relative position + 1 of the last delimiter (0: none).
struct Cnt {
    uint32_t nr, nf, col, last;
};
constexpr uint32_t kCAbs = 1u << 31;

__device__ inline Cnt cnt_combine(Cnt a, Cnt b)
{
    Cnt r;
    r.nr = a.nr + b.nr;
    r.nf = a.nf + b.nf;
    r.col = (b.col & kCAbs) ? b.col : a.col + b.col;  // the abs/rel operator of Sec. 3.2
    r.last = b.last ? b.last : a.last;
    return r;
}

template <int CTRL, int ROWS>
__device__ __forceinline__ Cnt dpp_cnt(Cnt c)
{
    return {dpp_move<CTRL, ROWS>(0u, c.nr), dpp_move<CTRL, ROWS>(0u, c.nf), dpp_move<CTRL, ROWS>(0u, c.col),
            dpp_move<CTRL, ROWS>(0u, c.last)};
}

// Inclusive scan of the count elements over the lanes (identity: all zero).
__device__ __forceinline__ Cnt wave_scan_cnt(Cnt x)
{
    x = cnt_combine(dpp_cnt<0x111, 0xF>(x), x);
    x = cnt_combine(dpp_cnt<0x112, 0xF>(x), x);
    x = cnt_combine(dpp_cnt<0x114, 0xF>(x), x);
    x = cnt_combine(dpp_cnt<0x118, 0xF>(x), x);
    x = cnt_combine(dpp_cnt<0x142, 0xA>(x), x);
    x = cnt_combine(dpp_cnt<0x143, 0xC>(x), x);
    return x;
}

// ---- device-wide count prefix ------------------------------------------------------
struct Tot {
    u64 rec, fld, col, last;
};

__device__ inline Tot tot_combine(Tot a, Tot b)
{
    Tot r;
    r.rec = a.rec + b.rec;
    r.fld = a.fld + b.fld;
    r.col = (b.col & kColAbs) ? b.col : a.col + b.col;
    const u64 body = (b.last & kLastHas) ? b.last : a.last;
    r.last = (body & ~kLastCtl) | (b.last & kLastCtl);  // control bit of the last byte: from b
    return r;
}

template <int CTRL>
__device__ __forceinline__ u64 dpp64(u64 v)  // identity (0) from outside the row
{
    const uint32_t lo = dpp_move<CTRL, 0xF>(0u, (uint32_t)v), hi = dpp_move<CTRL, 0xF>(0u, (uint32_t)(v >> 32));
    return ((u64)hi << 32) | lo;
}

template <int CTRL>
__device__ __forceinline__ Tot dpp_tot(Tot t)
{
    return {dpp64<CTRL>(t.rec), dpp64<CTRL>(t.fld), dpp64<CTRL>(t.col), dpp64<CTRL>(t.last)};
}

// The ordered lane reduction above for count prefixes (the all-zero Tot is
// a left identity of tot_combine).
__device__ __forceinline__ Tot wave_reduce_desc_tot(Tot x)
{
    x = tot_combine(dpp_tot<0x101>(x), x);
    x = tot_combine(dpp_tot<0x102>(x), x);
    x = tot_combine(dpp_tot<0x104>(x), x);
    x = tot_combine(dpp_tot<0x108>(x), x);
    Tot r[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        r[k] = {readlane64(x.rec, 16 * k), readlane64(x.fld, 16 * k), readlane64(x.col, 16 * k),
                readlane64(x.last, 16 * k)};
    return tot_combine(tot_combine(tot_combine(r[3], r[2]), r[1]), r[0]);
}

// aggregate words: agg0 = nr:31 @31 | nf:31; agg1 = col:31 @31 | last:31 where
// col = abs:1 @30 | value:30 and last = has:1 @30 | ctl:1 @29 | state after:4 @25 | pos in tile:25
__device__ inline Tot tot_from_agg(u64 a0, u64 a1, int64_t tile_start)
{
    Tot t;
    t.rec = (a0 >> 31) & 0x7fffffffull;
    t.fld = a0 & 0x7fffffffull;
    const u64 c = (a1 >> 31) & 0x7fffffffull;
    t.col = ((c >> 30) & 1 ? kColAbs : 0ull) | (c & 0x3fffffffull);
    const u64 l = a1 & 0x7fffffffull;
    t.last = ((l >> 29) & 1) ? kLastCtl : 0ull;
    if ((l >> 30) & 1)
        t.last |= kLastHas | (((l >> 25) & 0xfull) << 56) | (u64)(tile_start + (int64_t)(l & 0x1ffffffull));
    return t;
}

// Reads input bytes for conversion: from the LDS tile when inside it, from
// HBM for the head of a field that began in an earlier tile.
// Bytes kept in LDS before a tile (not for the first tile of a buffer, whose
// fields never start earlier).
constexpr int kLdsBefore = 64;

// A numeric field that begins tiles back and is at least this many symbols
// long is converted after the tile's own conversion by the whole workgroup
// (the block-level collaboration of Sec. 3.3) instead of by one lane
// reading it symbol by symbol from HBM. (A field within the tile is shorter
// than a tile and its lane reads it from LDS.)
constexpr int64_t kLongField = 2048;
struct LongEntry {
    int64_t b, e, rec;  // symbol span (enclosing control symbols stripped), global record
    uint32_t meta;      // column | type << 16
    uint32_t pad;
};
constexpr int kDigCap = 800;  // significant digits a long float keeps (the slow path's Decimal)

// A UTF-16 code unit as the byte the pipeline parses.
__device__ __forceinline__ uint32_t narrow_unit(uint32_t u) { return u < 0x80u ? u : 0x80u; }

// Symbol `pos` of the input as a byte: from LDS when the tile's copy holds
// it, else from global memory (narrowed, for code units).
template <int SH>
struct ByteSrc {
    const uint8_t* lds;  // the tile; lds[-kLdsBefore, 0) hold the bytes before it
    const uint8_t* g;
    int64_t tile_start;
    __device__ uint32_t operator()(int64_t pos) const
    {
        int64_t r = pos - tile_start;
        if (r >= -kLdsBefore) return lds[r];
        if constexpr (SH) return narrow_unit(gptr(reinterpret_cast<const uint16_t*>(g))[pos]);
        else return gptr(g)[pos];
    }
};

// Two code units narrowed in place: a packed 16-bit minimum with 0x80.
__device__ __forceinline__ uint32_t narrow2(uint32_t w)
{
    typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
    const u16x2 cap = {0x80, 0x80};
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(u16x2, w), cap));
}

// Eight code units (16 bytes) narrowed to eight bytes: the low bytes of the
// narrowed pairs gathered. (The components are named: this compiler lowers a
// bit cast of a subscripted vector element as element 0.)
__device__ __forceinline__ uint2 narrow8(u32x4 v)
{
    return make_uint2(__builtin_amdgcn_perm(narrow2(v.y), narrow2(v.x), 0x06040200u),
                      __builtin_amdgcn_perm(narrow2(v.w), narrow2(v.z), 0x06040200u));
}

// The general conversions (any length, any position, exponents, more than
// 19 digits). Returns 1 converted, 0 not a value of the type. (Kept inline:
// out of line, the calls cost the whole kernel about 7% on the numeric
// workload.)
template <class Src>
__device__ inline int convert_general(int ty, const Src& src, int64_t b, int64_t e, u64* bits)
{
    if (ty == PP_FLOAT64) {
        double dv = 0.0;
        const int r = conv_float64(src, b, e, &dv);
        *bits = __builtin_bit_cast(u64, dv);
        return r;
    }
    int64_t iv = 0;
    int r;
    if (ty == PP_INT64) r = conv_int64(src, b, e, &iv);
    else if (ty == PP_TIMESTAMP_S) r = conv_timestamp(src, b, e, &iv);
    else r = conv_date(src, b, e, &iv);
    *bits = (u64)iv;
    return r;
}

// Strip the enclosing control symbols of field [b, e) and convert it into
// column c, record rec. ctl_first/ctl_last_sym: whether symbols b and e-1 are
// control symbols. Returns 1 on a conversion error.
template <int SH>
__device__ inline int store_field(const TileArgs& p, const ColDesc* cols, const ByteSrc<SH>& src, int c, int ty,
                                  int64_t rec, int64_t b, int64_t e, bool ctl_first, bool ctl_last_sym)
{
    int64_t begin = b, end = e;
    if (end > begin && ctl_first) ++begin;
    if (end - 1 >= begin && ctl_last_sym) --end;
    const bool store = rec < p.cap_records;
    const ColDesc cd = cols[c];
    if (ty == PP_STRING) {
        if (store) {
            gptr((int64_t*)cd.values)[rec] = begin << SH;
            gptr(cd.str_end)[rec] = end << SH;
            gptr(cd.valid)[rec] = 1;
        }
        return 0;
    }
    if (end == begin) {  // empty: the column default, not an error (Sec. 4.3)
        if (store) {
            gptr((int64_t*)cd.values)[rec] = 0;
            gptr(cd.valid)[rec] = 0;
        }
        return 0;
    }
    u64 bits = 0;
    const bool ok = convert_general(ty, src, begin, end, &bits) == 1;
    if (!ok) bits = 0ull;
    if (store) {
        gptr((u64*)cd.values)[rec] = bits;
        gptr(cd.valid)[rec] = ok;
    }
    return !ok;
}

__device__ inline void store_missing(const TileArgs& p, const ColDesc* cols, int c, int ty, int64_t rec)
{
    if (rec >= p.cap_records || ty == PP_SKIP) return;
    const ColDesc cd = cols[c];
    gptr((u64*)cd.values)[rec] = 0;  // 0 and 0.0 share the bit pattern
    gptr(cd.valid)[rec] = 0;
    if (ty == PP_STRING) gptr(cd.str_end)[rec] = 0;
}

// ---- the kernel ---------------------------------------------------------------
// Shared memory of one tile (sized for up to 8 states, so one allocation
// serves both state-vector widths).
template <int NT, int B>
struct TileSmem {
    static constexpr int TILE = NT * B;
    static constexpr int NW = NT / 64;
    static constexpr int FCAP = TILE / 6;   // delimiters staged per tile
    static constexpr int RCAP = TILE / 16;  // records staged per tile
    uint32_t tnext[512];  // byte -> next state of every state
    uint32_t tcomb[512];  // byte -> per state (next*8 | tag<<6)
    uint8_t after_delim[256];  // byte -> the state after it as a delimiter (0xff: depends on the state)
    uint8_t ctl_any[256];      // byte -> 1 if it is a control symbol (a quote) in some state
    // the tile at offset PRE, preceded by the PRE bytes before it (where the
    // tile's first field usually begins); +32: register windows read past the end
    static constexpr int PRE = kLdsBefore;
    __attribute__((aligned(16))) uint8_t bytes[PRE + TILE + 32];
    uint16_t pos[FCAP];     // tile-relative delimiter positions
    uint8_t colid[FCAP];    // column of the field each delimiter closes (below 255; else the per-thread path)
    uint16_t recend[RCAP];  // local field index of each record delimiter
    uint32_t ctl[TILE / 32];  // control-symbol bitmap of the tile
    double pow10[24];  // 10^k, k <= 22, for the decimal conversions
    uint32_t wsv[NW][2];
    Cnt wcnt[NW];
    uint32_t anyctl, s0, fin, last_sa, guess, colovf;
    // Long numeric fields queued for the workgroup pass: the tile's first
    // field when it is a number that began tiles back (fields within the
    // tile are shorter than a tile and read from LDS by their lane).
    static constexpr int LCAP = 1;
    LongEntry longq[LCAP];
    uint32_t nlong;
    u64 red[12];  // the pass's reductions
    // the buffer's input, record capacity and column descriptors for the
    // pass, kept here rather than in registers across the whole tile
    const uint8_t* lin;
    int64_t lcap;
    const ColDesc* lcols;
    pp_result_t* lres;
    u64 pref[4];
    u64 err, ragged, fmin, fmax;  // fmin/fmax: fewest/most fields of a record closed here
};

// A buffer's constants in LDS: the per-byte transition rows (built by the
// init kernel from the DFA's group table), the column descriptors and the
// powers of ten. Visible after the workgroup's next barrier.
template <int NT, int B, bool NS8>
__device__ __forceinline__ void tile_setup(const TileArgs& p, TileSmem<NT, B>& sm)
{
    const int tid = threadIdx.x;
    if (tid <= 22) sm.pow10[tid] = exact_pow10(tid);
    for (int k = tid; k < (NS8 ? 512 : 256); k += NT) {
        sm.tnext[k] = gptr(p.tables)[k];
        sm.tcomb[k] = gptr(p.tables)[512 + k];
    }
    // For each byte, the state the DFA enters when the byte closes a field or
    // record, if the same from every state in which it does (typical: the
    // start of the next field); else 0xff. States without a delimiter
    // transition on the byte carry no tag and drop out.
    for (int b = tid; b < 256; b += NT) {
        const uint32_t lo = gptr(p.tables)[512 + (NS8 ? 2 * b : b)];
        const uint32_t hi = NS8 ? gptr(p.tables)[512 + 2 * b + 1] : 0u;
        uint32_t a = 0xffu, any = 0u, same = 1u, ctl = 0u;
        for (int st = 0; st < (NS8 ? 8 : 4); ++st) {
            const uint32_t x = ((st < 4 ? lo : hi) >> (8 * (st & 3))) & 0xffu;
            ctl |= (x >> 6) == kTagControl;
            if (x & 0x80u) {  // tag bit 1: a field or record delimiter
                const uint32_t nx = (x >> 3) & 7u;
                same &= !any || nx == a;
                a = nx;
                any = 1u;
            }
        }
        sm.after_delim[b] = (uint8_t)(any && same ? a : 0xffu);
        sm.ctl_any[b] = (uint8_t)ctl;
    }
}

// ---- long numeric fields: the workgroup pass ----------------------------------------
__device__ inline u64 wave_min_u64(u64 v)
{
#pragma unroll
    for (int d = 32; d; d >>= 1) {
        const u64 o = shfl_xor64(v, d);
        v = o < v ? o : v;
    }
    return v;
}
__device__ inline u64 wave_max_u64(u64 v)
{
#pragma unroll
    for (int d = 32; d; d >>= 1) {
        const u64 o = shfl_xor64(v, d);
        v = o > v ? o : v;
    }
    return v;
}
__device__ inline u64 wave_sum_u64(u64 v)
{
#pragma unroll
    for (int d = 32; d; d >>= 1) v += shfl_xor64(v, d);
    return v;
}
__device__ inline uint32_t word_of(const u32x4& v, int q) { return q == 0 ? v.x : q == 1 ? v.y : q == 2 ? v.z : v.w; }

// The symbols [lo, hi) of the input, spread over the workgroup: those at the
// unaligned ends one at a time to sym_visit(i, c) (c the symbol's byte),
// the aligned middle four at a time to word_visit(i, w) (symbols i..i+3 as
// the bytes of w, low byte first), from 16-byte loads (four in flight per
// thread). Each thread visits its symbols in increasing position.
template <int NT, int SH, class SymVisit, class WordVisit>
__device__ inline void scan_symbols(const uint8_t* in, int64_t lo, int64_t hi, SymVisit&& sym_visit,
                                    WordVisit&& word_visit)
{
    const int tid = threadIdx.x;
    auto sym = [&](int64_t i) -> uint32_t {
        if constexpr (SH) return narrow_unit(gptr(reinterpret_cast<const uint16_t*>(in))[i]);
        else return gptr(in)[i];
    };
    if (hi <= lo) return;
    const uintptr_t base = (uintptr_t)in;
    const uintptr_t a = base + ((uintptr_t)lo << SH), z = base + ((uintptr_t)hi << SH);
    const uintptr_t a16 = (a + 15) & ~(uintptr_t)15, z16 = z & ~(uintptr_t)15;
    if (a16 >= z16) {
        for (int64_t i = lo + tid; i < hi; i += NT) sym_visit(i, sym(i));
        return;
    }
    const int64_t h1 = (int64_t)((a16 - base) >> SH), t0 = (int64_t)((z16 - base) >> SH);
    for (int64_t i = lo + tid; i < h1; i += NT) sym_visit(i, sym(i));
    constexpr int SPB = 16 >> SH;  // symbols per 16-byte block
    const int64_t nblk = (int64_t)((z16 - a16) >> 4);
    const u32x4* const blk = reinterpret_cast<const u32x4*>(a16);
    for (int64_t k0 = tid; k0 < nblk; k0 += 4 * NT) {
        u32x4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t k = k0 + (int64_t)u * NT;
            v[u] = k < nblk ? __builtin_nontemporal_load(gptr(blk) + k) : u32x4{0u, 0u, 0u, 0u};
        }
        auto block = [&](const u32x4& v, int64_t k) {
            const int64_t i0 = h1 + k * SPB;
            if constexpr (SH) {
                const uint2 n = narrow8(v);
                word_visit(i0, n.x);
                word_visit(i0 + 4, n.y);
            } else {
                word_visit(i0, v.x);
                word_visit(i0 + 4, v.y);
                word_visit(i0 + 8, v.z);
                word_visit(i0 + 12, v.w);
            }
        };
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (k0 + (int64_t)u * NT < nblk) block(v[u], k0 + (int64_t)u * NT);
    }
    for (int64_t i = t0 + tid; i < hi; i += NT) sym_visit(i, sym(i));
}

// Per byte of a word of symbols, 0x80 where: not a digit; the digit '0'; a
// decimal point; an exponent mark (e or E). Exact per byte.
__device__ inline uint32_t nondigit_bytes(uint32_t w) { return above9_bytes(w ^ 0x30303030u); }
__device__ inline uint32_t zerodigit_bytes(uint32_t w) { return zero_bytes(w ^ 0x30303030u); }
__device__ inline uint32_t point_bytes(uint32_t w) { return zero_bytes(w ^ 0x2e2e2e2eu); }
__device__ inline uint32_t expmark_bytes(uint32_t w) { return zero_bytes((w | 0x20202020u) ^ 0x65656565u); }
__device__ inline int64_t first_byte(uint32_t f) { return __builtin_ctz(f) >> 3; }
__device__ inline int64_t last_byte(uint32_t f) { return (31 - __builtin_clz(f)) >> 3; }

// Converts the queued long numeric fields, one at a time, with the whole
// workgroup (every thread calls this): the field's symbols are classified
// in parallel and the facts the sequential conversions depend on are reduced
// -- for INT64 the grammar and the first nonzero digit; for FLOAT64 the
// exponent mark, the decimal point, the grammar, the first and last nonzero
// mantissa digits and the first nonzero exponent digit -- and the first
// kDigCap significant digits gathered in LDS. One thread then finishes with
// the same arithmetic as conv_int64 / conv_float64 (Clinger's exact case, or
// the Decimal of the slow path built from the gathered digits), so every
// result equals the sequential conversion's. Stores the value and validity
// of records within the capacity and adds the conversion errors to the
// tile's count.
template <int NT, int B, int SH>
__device__ __noinline__ void long_pass(TileSmem<NT, B>& sm)
{
    const uint8_t* const in = sm.lin;
    const int64_t cap_records = sm.lcap;
    const ColDesc* const cols = sm.lcols;
    constexpr u64 NONE = ~0ull;
    const int tid = threadIdx.x, lane = tid & 63;
    const uint32_t nl = sm.nlong < (uint32_t)TileSmem<NT, B>::LCAP ? sm.nlong : (uint32_t)TileSmem<NT, B>::LCAP;
    uint8_t* const dig = reinterpret_cast<uint8_t*>(sm.pos);  // free once the tile's conversion is done
    static_assert(TileSmem<NT, B>::FCAP * 2 >= kDigCap, "digit buffer");
    auto sym = [&](int64_t i) -> uint32_t {
        if constexpr (SH) return narrow_unit(gptr(reinterpret_cast<const uint16_t*>(in))[i]);
        else return gptr(in)[i];
    };
    auto rmin = [&](int k, u64 v) {
        v = wave_min_u64(v);
        if (lane == 0 && v != NONE) atomicMin((unsigned long long*)&sm.red[k], (unsigned long long)v);
    };
    auto rmax = [&](int k, u64 v) {
        v = wave_max_u64(v);
        if (lane == 0 && v) atomicMax((unsigned long long*)&sm.red[k], (unsigned long long)v);
    };
    auto rsum = [&](int k, u64 v) {
        v = wave_sum_u64(v);
        if (lane == 0 && v) atomicAdd((unsigned long long*)&sm.red[k], (unsigned long long)v);
    };
    u64 errs = 0;
    for (uint32_t q = 0; q < nl; ++q) {
        const LongEntry en = sm.longq[q];
        const uint32_t ty = en.meta >> 16, col = en.meta & 0xffffu;
        const int64_t b = en.b, e = en.e;
        const uint32_t c0 = sym(b);
        const bool neg = c0 == '-', sg = neg || c0 == '+';
        const int64_t s0 = b + (sg ? 1 : 0);
        if (tid < 12) sm.red[tid] = (tid == 0 || tid == 7 || tid == 8) ? NONE : 0ull;
        __syncthreads();
        int ok = 0;
        u64 bits = 0;
        if (ty == PP_INT64) {
            // [+-]?[0-9]+: any other symbol (red[1]), the first nonzero digit (red[0])
            u64 bad = 0, fnz = NONE;
            scan_symbols<NT, SH>(
                in, s0, e,
                [&](int64_t i, uint32_t c) {
                    bad |= (u64)(c - '0' > 9u);
                    if (c - '1' < 9u && (u64)i < fnz) fnz = (u64)i;
                },
                [&](int64_t i, uint32_t w) {
                    const uint32_t nd = nondigit_bytes(w), nz = ~nd & ~zerodigit_bytes(w) & 0x80808080u;
                    bad |= (u64)(nd != 0u);
                    if (nz && (u64)(i + first_byte(nz)) < fnz) fnz = (u64)(i + first_byte(nz));
                });
            rsum(1, bad);
            rmin(0, fnz);
            __syncthreads();
            if (tid == 0) {
                const u64 f = sm.red[0];
                if (s0 < e && sm.red[1] == 0) {
                    if (f == NONE) {
                        ok = 1;  // all zeros
                    } else if (e - (int64_t)f <= 19) {  // more significant digits overflow
                        const uint64_t limit = neg ? (1ull << 63) : (1ull << 63) - 1;
                        uint64_t mag = 0;
                        ok = 1;
                        for (int64_t i = (int64_t)f; i < e; ++i) {
                            const uint32_t d = sym(i) - '0';
                            if (mag > (limit - d) / 10u) { ok = 0; break; }
                            mag = mag * 10u + d;
                        }
                        if (ok) bits = neg ? 0ull - mag : mag;
                    }
                }
            }
        } else {
            // One pass over [s0, e) classifies every symbol: exponent marks
            // (first red[0], count red[1]), points (count red[2], last
            // red[3] + 1), other symbols (red[4]), signs (count red[5], last
            // red[6] + 1), nonzero digits (first red[8], last red[9] + 1).
            // A valid field has at most one mark E, signs only right after
            // it, no point after it; then the nonzero digits before E are
            // the mantissa's and only the exponent's digits (usually few)
            // and, when they hold a nonzero digit, the mantissa's last
            // nonzero digit need another pass.
            u64 em = NONE, ne = 0, ndot = 0, dpos = 0, nbad = 0, nsg = 0, spos = 0, fnz = NONE, lnz = 0;
            scan_symbols<NT, SH>(
                in, s0, e,
                [&](int64_t i, uint32_t c) {
                    const bool d = c - '0' < 10u, dot = c == '.', mk = (c | 0x20u) == 'e', sgn = c == '+' || c == '-';
                    ne += mk;
                    if (mk && (u64)i < em) em = (u64)i;
                    ndot += dot;
                    if (dot && (u64)i + 1 > dpos) dpos = (u64)i + 1;
                    nsg += sgn;
                    if (sgn && (u64)i + 1 > spos) spos = (u64)i + 1;
                    nbad += !d && !dot && !mk && !sgn;
                    if (c - '1' < 9u) {
                        fnz = (u64)i < fnz ? (u64)i : fnz;
                        lnz = (u64)i + 1 > lnz ? (u64)i + 1 : lnz;
                    }
                },
                [&](int64_t i, uint32_t w) {
                    const uint32_t nd = nondigit_bytes(w), nz = ~nd & ~zerodigit_bytes(w) & 0x80808080u;
                    if (nz) {  // positions increase: the first is the least, the latest the greatest
                        if (fnz == NONE) fnz = (u64)(i + first_byte(nz));
                        lnz = (u64)(i + last_byte(nz)) + 1;
                    }
                    if (nd == 0u) return;  // four digits (the common word)
                    const uint32_t pt = point_bytes(w), mk = expmark_bytes(w);
                    const uint32_t sg = zero_bytes(w ^ 0x2b2b2b2bu) | zero_bytes(w ^ 0x2d2d2d2du);
                    if (mk) {
                        ne += (u64)__popc(mk);
                        const u64 f = (u64)(i + first_byte(mk));
                        em = f < em ? f : em;
                    }
                    if (pt) {
                        ndot += (u64)__popc(pt);
                        const u64 l = (u64)(i + last_byte(pt)) + 1;
                        dpos = l > dpos ? l : dpos;
                    }
                    if (sg) {
                        nsg += (u64)__popc(sg);
                        const u64 l = (u64)(i + last_byte(sg)) + 1;
                        spos = l > spos ? l : spos;
                    }
                    nbad += (u64)__popc(nd & ~pt & ~mk & ~sg);
                });
            rmin(0, em);
            rsum(1, ne);
            rsum(2, ndot);
            rmax(3, dpos);
            rsum(4, nbad);
            rsum(5, nsg);
            rmax(6, spos);
            rmin(8, fnz);
            rmax(9, lnz);
            __syncthreads();
            const u64 nmark = sm.red[1], ndots = sm.red[2], nsigns = sm.red[5];
            const int64_t E = nmark ? (int64_t)sm.red[0] : e;
            const bool esg = nsigns == 1 && (int64_t)sm.red[6] - 1 == E + 1;  // the exponent's sign
            const int64_t x0 = E + 1 + (esg ? 1 : 0);                        // its first digit
            const int64_t dotpos = ndots ? (int64_t)sm.red[3] - 1 : E;        // the point, or E without one
            const bool valid = nmark <= 1 && sm.red[4] == 0 && ndots <= 1 && dotpos <= E &&
                               (E - s0 - (int64_t)ndots) >= 1 &&
                               (nmark ? (nsigns == 0 || esg) && x0 < e : nsigns == 0);
            const u64 F = sm.red[8] != NONE && (int64_t)sm.red[8] < E ? sm.red[8] : NONE;  // first nonzero mantissa digit
            const bool exp_nz = valid && nmark && sm.red[9] != 0 && (int64_t)sm.red[9] - 1 > E;
            if (exp_nz) {
                // the exponent's first nonzero digit (red[7]), and the
                // mantissa's last nonzero digit (red[10] + 1) without the
                // exponent's digits
                u64 efnz = NONE, mlnz = 0;
                scan_symbols<NT, SH>(
                    in, x0, e,
                    [&](int64_t i, uint32_t c) {
                        if (c - '1' < 9u && (u64)i < efnz) efnz = (u64)i;
                    },
                    [&](int64_t i, uint32_t w) {
                        const uint32_t nz = ~nondigit_bytes(w) & ~zerodigit_bytes(w) & 0x80808080u;
                        if (nz && (u64)(i + first_byte(nz)) < efnz) efnz = (u64)(i + first_byte(nz));
                    });
                if (F != NONE)
                    scan_symbols<NT, SH>(
                        in, (int64_t)F, E,
                        [&](int64_t i, uint32_t c) {
                            if (c - '1' < 9u && (u64)i + 1 > mlnz) mlnz = (u64)i + 1;
                        },
                        [&](int64_t i, uint32_t w) {
                            const uint32_t nz = ~nondigit_bytes(w) & ~zerodigit_bytes(w) & 0x80808080u;
                            if (nz && (u64)(i + last_byte(nz)) + 1 > mlnz) mlnz = (u64)(i + last_byte(nz)) + 1;
                        });
                rmin(7, efnz);
                rmax(10, mlnz);
                __syncthreads();
            }
            const int64_t L = (exp_nz ? (int64_t)sm.red[10] : (int64_t)sm.red[9]) - 1;  // the last nonzero mantissa digit
            // significant digits from the first nonzero one, the point skipped
            auto sigidx = [&](int64_t i) -> int64_t { return (i - (int64_t)F) - (ndots && dotpos > (int64_t)F && dotpos < i ? 1 : 0); };
            if (valid && F != NONE) {
                for (int64_t i = (int64_t)F + tid; i < E && i < (int64_t)F + kDigCap + 1; i += NT) {
                    const uint32_t c = sym(i);
                    if (c != '.') {
                        const int64_t k = sigidx(i);
                        if (k < kDigCap) dig[k] = (uint8_t)(c - '0');
                    }
                }
            }
            __syncthreads();
            if (tid == 0 && valid) {
                ok = 1;
                if (F == NONE) {
                    bits = neg ? (1ull << 63) : 0ull;  // a signed zero
                } else {
                    // the exponent as the sequential loops read it: digits
                    // accumulate while the value is below 10^8, so the first
                    // (at most nine) significant ones count
                    int64_t ex = 0;
                    if (E < e && sm.red[7] != NONE)
                        for (int64_t i = (int64_t)sm.red[7]; i < e && ex < 100000000; ++i) ex = ex * 10 + (sym(i) - '0');
                    if (esg && sym(E + 1) == '-') ex = -ex;
                    const int64_t nS = (E - (int64_t)F) - (ndots && dotpos > (int64_t)F ? 1 : 0);
                    const int64_t nint = (int64_t)F < dotpos ? dotpos - (int64_t)F : 0;  // significant integer digits
                    const int64_t nfrac = ndots ? E - dotpos - 1 : 0;
                    const int64_t last = sigidx(L);
                    uint64_t w = 0;
                    for (int64_t k = 0; k < nS && k < 19; ++k) w = w * 10 + dig[k];
                    const int64_t dropped = nint > 19 ? nint - 19 : 0;
                    int64_t kept = 0;
                    if (ndots && nint < 19) {
                        if ((int64_t)F > dotpos) {
                            const int64_t lz = (int64_t)F - dotpos - 1;
                            kept = lz + (nfrac - lz < 19 ? nfrac - lz : 19);
                        } else {
                            kept = nfrac < 19 - nint ? nfrac : 19 - nint;
                        }
                    }
                    const int64_t e10 = ex + dropped - kept;
                    if (last < 19 && w <= (1ull << 53) && e10 >= -22 && e10 <= 22) {
                        double v = (double)w;
                        v = e10 < 0 ? v / exact_pow10((int)-e10) : v * exact_pow10((int)e10);
                        bits = __builtin_bit_cast(u64, neg ? -v : v);
                    } else {
                        Decimal a;
                        a.nd = (int)(nS < kDecCap ? nS : kDecCap);
                        for (int k = 0; k < a.nd; ++k) a.d[k] = dig[k];
                        a.trunc = last >= kDecCap;
                        a.dp = (int)((int64_t)F < dotpos ? nint : -((int64_t)F - dotpos - 1));
                        a.dp += (int)ex;
                        bits = __builtin_bit_cast(u64, dec_to_double(a, neg));
                    }
                }
            }
        }
        if (tid == 0) {
            if (en.rec < cap_records) {
                const ColDesc cd = cols[col];
                gptr((u64*)cd.values)[en.rec] = ok ? bits : 0ull;
                gptr(cd.valid)[en.rec] = (uint8_t)ok;
            }
            errs += !ok;
        }
        __syncthreads();  // red and the digits are reused by the next field
    }
    if (tid == 0 && errs) atomicAdd((u64*)&sm.lres->num_conversion_errors, errs);
}

// The whole pipeline for tile `tile` of one buffer (steps 1-7 above).
// SETUP: load the buffer's constants here (else the caller has, before a
// barrier that precedes this call). SH: symbols are bytes (0) or UTF-16
// code units (1); p.n counts symbols.
template <int NT, int B, bool NS8, bool SETUP = true, int SH = 0>
__device__ __forceinline__ void parse_tile(const TileArgs& p, const uint32_t tile, TileSmem<NT, B>& sm)
{
    static_assert(B == 16 || B == 32 || B == 64, "chunk bitmaps are one or two dwords");
    using M = std::conditional_t<(B > 32), u64, uint32_t>;
    constexpr int TILE = NT * B;
    constexpr int NW = NT / 64;
    constexpr int FCAP = TileSmem<NT, B>::FCAP;
    constexpr int RCAP = TileSmem<NT, B>::RCAP;
    static_assert(TILE <= 32768, "u16 positions");
    uint32_t* const s_tnext = sm.tnext;
    uint32_t* const s_tcomb = sm.tcomb;
    uint8_t* const s_bytes = sm.bytes + TileSmem<NT, B>::PRE;  // the tile; s_bytes[-PRE, 0) precede it
    uint16_t* const s_pos = sm.pos;
    uint8_t* const s_colid = sm.colid;
    uint16_t* const s_recend = sm.recend;
    uint32_t* const s_ctl = sm.ctl;
    const ColDesc* const s_cols = p.cols;  // column descriptors in global memory
    SV<NS8>* const s_wsv = reinterpret_cast<SV<NS8>*>(&sm.wsv[0][0]);
    Cnt* const s_wcnt = sm.wcnt;
    uint32_t& s_anyctl = sm.anyctl;
    uint32_t& s_s0 = sm.s0;
    uint32_t& s_final = sm.fin;
    uint32_t& s_last_sa = sm.last_sa;
    u64* const s_pref = sm.pref;
    u64& s_err = sm.err;
    u64& s_ragged = sm.ragged;
    u64& s_fmin = sm.fmin;
    u64& s_fmax = sm.fmax;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;

    // No barrier first: a workgroup parses one tile, and its kernel's own
    // barrier (after the ticket) precedes this; nothing written below is
    // read before the staging barrier.
    if (tid == 0) {
        sm.colovf = 0;
        sm.nlong = 0;
        sm.lin = p.in;
        sm.lcap = p.cap_records;
        sm.lcols = p.cols;
        sm.lres = p.result;
        s_anyctl = 0;
        s_err = 0;
        s_ragged = 0;
        s_fmin = ~0ull;
        s_fmax = 0;
    }
    if constexpr (SETUP) tile_setup<NT, B, NS8>(p, sm);  // first read after the staging barrier

    const int64_t n = p.n;
    const int64_t tile_start = (int64_t)tile * TILE;
    const int tile_len = (int)(n - tile_start < TILE ? n - tile_start : TILE);
    u64* const tw = p.words + (size_t)tile * kWordsPerTile;

    // ---- 1. stage the tile --------------------------------------------------------
    if constexpr (SH) {  // code units, narrowed on the way into LDS
        constexpr int PRE = TileSmem<NT, B>::PRE;
        const uint16_t* src = reinterpret_cast<const uint16_t*>(p.in) + tile_start;
        if (tile_len == TILE && (((uintptr_t)src) & 15) == 0) {
            const u32x4* s4 = reinterpret_cast<const u32x4*>(src);
            uint2* d2 = reinterpret_cast<uint2*>(s_bytes);
#pragma unroll
            for (int k = tid; k < TILE / 8; k += NT) d2[k] = narrow8(__builtin_nontemporal_load(gptr(s4) + k));
        } else {
            for (int k = tid; k < TILE; k += NT) s_bytes[k] = k < tile_len ? narrow_unit(gptr(src)[k]) : 0;
        }
        if (tile_start >= PRE) {  // the symbols just before the tile
            const uint16_t* pre = src - PRE;
            if ((((uintptr_t)pre) & 15) == 0) {
                if (tid < PRE / 8)
                    reinterpret_cast<uint2*>(s_bytes - PRE)[tid] =
                        narrow8(__builtin_nontemporal_load(gptr(reinterpret_cast<const u32x4*>(pre)) + tid));
            } else if (tid < PRE) {
                s_bytes[tid - PRE] = narrow_unit(gptr(pre)[tid]);
            }
        }
    } else {
        const uint8_t* src = p.in + tile_start;
        if (tile_len == TILE && (((uintptr_t)src) & 15) == 0) {
            const u32x4* s4 = reinterpret_cast<const u32x4*>(src);
            u32x4* d4 = reinterpret_cast<u32x4*>(s_bytes);
#pragma unroll
            for (int k = tid; k < TILE / 16; k += NT) d4[k] = __builtin_nontemporal_load(gptr(s4) + k);
        } else {
            for (int k = tid; k < TILE; k += NT) s_bytes[k] = k < tile_len ? gptr(src)[k] : 0;
        }
        constexpr int PRE = TileSmem<NT, B>::PRE;
        if (tile_start >= PRE) {  // the bytes just before the tile
            const uint8_t* pre = src - PRE;
            if ((((uintptr_t)pre) & 15) == 0) {
                if (tid < PRE / 16)
                    reinterpret_cast<u32x4*>(s_bytes - PRE)[tid] =
                        __builtin_nontemporal_load(gptr(reinterpret_cast<const u32x4*>(pre)) + tid);
            } else if (tid < PRE) {
                s_bytes[tid - PRE] = gptr(pre)[tid];
            }
        }
    }
    __syncthreads();

    const int c0 = tid * B;  // tile-relative chunk start
    const int len = tile_len - c0 <= 0 ? 0 : (tile_len - c0 < B ? tile_len - c0 : B);
    uint32_t wd[B / 4];
    {
        const uint4* q = reinterpret_cast<const uint4*>(s_bytes + c0);
#pragma unroll
        for (int k = 0; k < B / 16; ++k) {
            uint4 v = q[k];
            wd[4 * k] = v.x; wd[4 * k + 1] = v.y; wd[4 * k + 2] = v.z; wd[4 * k + 3] = v.w;
        }
    }
    auto byte_at = [&](int i) -> uint32_t { return (wd[i >> 2] >> ((i & 3) * 8)) & 0xffu; };
    // Cold paths (a chunk shorter than B, the state searches below) walk the
    // chunk in rolled loops over its LDS copy: the unrolled forms would add
    // kilobytes of code that every tile's hot path shares the instruction
    // cache with.
    const uint8_t* const cb_lds = s_bytes + c0;

    // ---- 2. multi-state pass ----------------------------------------------------------
    SV<NS8> vec = sv_identity<NS8>();
    auto mstep = [&](int i) {
        const uint32_t b = byte_at(i);
        SV<NS8> t;
        if constexpr (NS8) { t.lo = s_tnext[2 * b]; t.hi = s_tnext[2 * b + 1]; }
        else { t.lo = s_tnext[b]; t.hi = 0; }
        vec = compose(vec, t);
    };
    if (len == B) {
#pragma unroll
        for (int i = 0; i < B; ++i) mstep(i);
    } else {
        for (int i = 0; i < len; ++i) {
            const uint32_t b = cb_lds[i];
            SV<NS8> t;
            if constexpr (NS8) { t.lo = s_tnext[2 * b]; t.hi = s_tnext[2 * b + 1]; }
            else { t.lo = s_tnext[b]; t.hi = 0; }
            vec = compose(vec, t);
        }
    }

    // ---- 3. composition scan ------------------------------------------------------------
    const SV<NS8> incl = wave_scan_sv<NS8>(vec);
    if (lane == 63) s_wsv[wave] = incl;
    // A guess of the tile's start state for the speculative tag pass: the
    // DFA run from its start state over the 64 bytes before the tile (one
    // byte per lane, composed by a wavefront scan), when those bytes hold no
    // control symbol. It tracks the field structure up to the tile start
    // (typically the middle of a field), so the tile's first chunk is
    // usually spared its second tag pass; the lookback still decides.
    // Otherwise the guess is the DFA's start state.
    if (wave == 0) {
        uint32_t tile_guess = (uint32_t)p.start_state;
        if (tile_start >= kLdsBefore) {
            const uint32_t b = s_bytes[lane - kLdsBefore];
            SV<NS8> t;
            if constexpr (NS8) { t.lo = s_tnext[2 * b]; t.hi = s_tnext[2 * b + 1]; }
            else { t.lo = s_tnext[b]; t.hi = 0; }
            const SV<NS8> all = wave_scan_sv<NS8>(t);
            SV<NS8> v;
            v.lo = (uint32_t)__builtin_amdgcn_readlane((int)all.lo, 63);
            v.hi = NS8 ? (uint32_t)__builtin_amdgcn_readlane((int)all.hi, 63) : 0u;
            // trusted only when no byte there can be a control symbol (a quote
            // could flip the quoting of everything after it)
            if (ballot(sm.ctl_any[b] != 0) == 0) tile_guess = sv_get(v, (uint32_t)p.start_state);
        }
        if (lane == 0) sm.guess = tile_guess;
    }
    __syncthreads();
    // the wavefront aggregates in one unrolled pass (their reads go out
    // together): the prefix of the wavefronts before this one, and the tile's
    SV<NS8> wpre = sv_identity<NS8>(), agg = sv_identity<NS8>();
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const SV<NS8> v = s_wsv[w];
        if (w < wave) wpre = compose(wpre, v);
        agg = compose(agg, v);
    }
    const SV<NS8> ex = compose(wpre, wave_prev_sv<NS8>(incl));  // exclusive prefix of this chunk within the tile

    // the tile's aggregate goes out first; successors wait on it
    if (wave == 0 && lane == 0) publish(tw + W_STATE, (tile == 0 ? kIncl : kAgg) | sv_to_nib(agg));

    // ---- 4. tag pass ----------------------------------------------------------------------
    // x = tcomb[b] >> (8*state): bits 3-5 next state * 8, bit 6 tag bit 0, bit 7 tag bit 1.
    // It runs first under a guess of the tile's start state (above), while
    // the state lookback is still to come; chunks whose start state the
    // lookback then changes run it again.
    M p0 = 0, p1 = 0;
    uint32_t s8 = 0;
    auto tag_pass = [&](const uint32_t s_init, const bool hot) {
        p0 = 0;
        p1 = 0;
        s8 = s_init * 8u;
        auto tstep = [&](int i, uint32_t b) {
            uint32_t x;
            if constexpr (NS8) {
                const uint32_t e = s_tcomb[2 * b + (s8 >> 5)];
                x = __builtin_amdgcn_ubfe(e, s8 & 31u, 8);
            } else {
                x = __builtin_amdgcn_ubfe(s_tcomb[b], s8, 8);
            }
            // <= 4 states: the next state * 8 sits in bits 3-4 and the bit-field
            // offset reads bits 0-4 only, so x serves as the offset unmasked
            s8 = NS8 ? (x & 0x38u) : x;
            p0 |= (M)((x >> 6) & 1u) << i;
            p1 |= (M)(x >> 7) << i;
        };
        if (hot && len == B) {
            // Unrolled: the two tag bits of byte i go to bits 2(i%16) and
            // 2(i%16)+1 of word i/16 (one shift-or per byte), separated into
            // the two bitmaps once at the end.
            uint32_t il[B / 16];
#pragma unroll
            for (int k = 0; k < B / 16; ++k) il[k] = 0u;
            if constexpr (NS8) {
                // the table as bytes: byte 8b + s is state s's entry for byte b
                const uint8_t* const tb = reinterpret_cast<const uint8_t*>(s_tcomb);
                uint32_t st = s8 >> 3;
#pragma unroll
                for (int i = 0; i < B; ++i) {
                    const uint32_t x = tb[(byte_at(i) << 3) | st];
                    st = (x >> 3) & 7u;
                    il[i >> 4] |= (x >> 6) << (2 * (i & 15));
                }
                s8 = st << 3;
            } else {
#pragma unroll
                for (int i = 0; i < B; ++i) {
                    const uint32_t x = __builtin_amdgcn_ubfe(s_tcomb[byte_at(i)], s8, 8);
                    s8 = x;
                    il[i >> 4] |= (x >> 6) << (2 * (i & 15));
                }
            }
#pragma unroll
            for (int k = 0; k < B / 16; ++k) {
                const uint32_t w = unzip_bits(il[k]);
                p0 |= (M)(w & 0xffffu) << (16 * k);
                p1 |= (M)(w >> 16) << (16 * k);
            }
        } else {
            for (int i = 0; i < len; ++i) tstep(i, cb_lds[i]);
        }
    };
    const uint32_t s_guess = sv_get(ex, sm.guess);
    tag_pass(s_guess, true);

    if (wave == 0) {
        SV<NS8> pre = sv_identity<NS8>();
        if (tile > 0) {
            // one wavefront polls 64 predecessors per step
            SV<NS8> acc = sv_identity<NS8>();
            for (int64_t base = (int64_t)tile - 1;; base -= 64) {
                const int64_t j = base - lane;
                u64 v = j >= 0 ? peek(p.words + (size_t)j * kWordsPerTile + W_STATE) : kIncl;
                int first;
                for (;;) {
                    const u64 inc = ballot((v >> 62) == 2);
                    const u64 rdy = ballot((v >> 62) != 0);
                    first = inc ? __ffsll((long long)inc) - 1 : 64;
                    const u64 need = first >= 63 ? ~0ull : ((2ull << first) - 1);
                    if ((rdy & need) == need) break;
                    __builtin_amdgcn_s_sleep(1);
                    if ((v >> 62) == 0) v = peek(p.words + (size_t)j * kWordsPerTile + W_STATE);
                }
                // ordered reduction, earlier tiles (higher lanes) on the left
                const SV<NS8> x = lane <= first ? sv_from_nib<NS8>((uint32_t)v) : sv_identity<NS8>();
                const SV<NS8> w = wave_reduce_desc_sv<NS8>(x);
                acc = compose(w, acc);
                if (first < 64) break;
            }
            pre = acc;
            if (lane == 0) publish(tw + W_STATE, kIncl | sv_to_nib(compose(acc, agg)));
        }
        if (lane == 0) {
            s_s0 = sv_get(pre, (uint32_t)p.start_state);
            s_final = sv_get(compose(pre, agg), (uint32_t)p.start_state);
        }
    }
    __syncthreads();
    const uint32_t s_start = sv_get(ex, s_s0);
    if (s_start != s_guess) tag_pass(s_start, true);  // typically the tile's first chunk
    const uint32_t s_end = (s8 & 0x38u) >> 3;
    const M dmask = p1, rmask = p1 & p0, cmask = p0 & ~p1;
    const int64_t cstart = tile_start + c0;
    const bool holds_last = len > 0 && cstart + len == n;
    const uint32_t vend = holds_last && !((rmask >> (len - 1)) & 1u);  // end of input closes a record

    // first transition into the (absorbing) invalid state
    if (p.invalid_state >= 0 && s_start != (uint32_t)p.invalid_state && s_end == (uint32_t)p.invalid_state) {
        const uint32_t inv8 = (uint32_t)p.invalid_state * 8u;
        uint32_t r8 = s_start * 8u;
        int at = -1;
        for (int i = 0; i < len && at < 0; ++i) {
            r8 = step_state<NS8>(s_tcomb, cb_lds[i], r8);
            if (r8 == inv8) at = i;
        }
        gptr(p.result)->first_invalid_offset = (cstart + at) << SH;
    }

    auto popc = [](M m) -> uint32_t {
        if constexpr (B > 32) return (uint32_t)__popcll(m);
        else return (uint32_t)__popc(m);
    };
    auto msb = [](M m) -> int {
        if constexpr (B > 32) return 63 - __clzll((long long)m);
        else return 31 - __clz((int)m);
    };
    Cnt mine;
    mine.nr = popc(rmask) + vend;
    mine.nf = popc(dmask) + vend;
    if (rmask | vend) {
        uint32_t after = 0;
        if (!vend) {
            const int hb = msb(rmask);
            after = hb == B - 1 ? 0u : popc(dmask & ~rmask & (~(M)0 << (hb + 1)));
        }
        mine.col = kCAbs | after;
    } else {
        mine.col = popc(dmask);
    }
    mine.last = vend ? (uint32_t)(tile_len + 1) : (dmask ? (uint32_t)(c0 + msb(dmask) + 1) : 0u);
    {
        const bool wave_ctl = ballot(cmask != 0) != 0;  // every lane takes part in the ballot
        if (lane == 0 && wave_ctl) s_anyctl = 1u;       // one store per wavefront
    }
    {
        // this chunk's words of the tile's control bitmap (and of the whole
        // input's, when requested: words of bytes below n only)
        uint32_t* const g = p.ctl_out ? p.ctl_out + (size_t)tile * (TILE / 32) : nullptr;
        if constexpr (B == 64) {
            s_ctl[2 * tid] = (uint32_t)cmask;
            s_ctl[2 * tid + 1] = (uint32_t)(cmask >> 32);
            if (g && c0 < tile_len) put(g, 2u * tid, (uint32_t)cmask);
            if (g && c0 + 32 < tile_len) put(g, 2u * tid + 1u, (uint32_t)(cmask >> 32));
        } else if constexpr (B == 32) {
            s_ctl[tid] = cmask;
            if (g && c0 < tile_len) put(g, (uint32_t)tid, (uint32_t)cmask);
        } else {  // two 16-byte chunks per bitmap word
            const uint32_t part = cmask << ((tid & 1) * 16);
            const uint32_t other = (uint32_t)__shfl_xor((int)part, 1);
            if ((tid & 1) == 0) s_ctl[tid >> 1] = part | other;
            if (g && (tid & 1) == 0 && c0 < tile_len) put(g, (uint32_t)(tid >> 1), part | other);
        }
    }

    // ---- 5. count scans ------------------------------------------------------------------
    const Cnt cin = wave_scan_cnt(mine);
    if (lane == 63) s_wcnt[wave] = cin;
    __syncthreads();
    Cnt cpre = {0u, 0u, 0u, 0u}, tagg = {0u, 0u, 0u, 0u};  // wavefronts before this one; the whole tile
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const Cnt v = s_wcnt[w];
        if (w < wave) cpre = cnt_combine(cpre, v);
        tagg = cnt_combine(tagg, v);
    }
    const Cnt cex = cnt_combine(cpre, dpp_cnt<0x138, 0xF>(cin));  // previous lane's (zero in lane 0)

    // The tile's aggregate needs the DFA state after its last delimiter and
    // the control bit of its last byte. Every thread reads both from LDS (the
    // delimiter byte's entry in the after-delimiter table; the control
    // bitmap, complete since the barrier above), so no further barrier is
    // needed, except where the state after that byte depends on the state
    // before it: then the chunk holding the delimiter (the one whose own last
    // delimiter is the tile's: positions are unique) walks to it.
    const uint32_t lastrel = tagg.last;                      // position + 1, 0 = none
    const bool virt_end = lastrel == (uint32_t)tile_len + 1u;  // the end of input closes the last record
    uint32_t my_last_sa = 0;
    if (lastrel && !virt_end) my_last_sa = sm.after_delim[s_bytes[lastrel - 1u]];
    if (my_last_sa == 0xffu) {  // the same for every thread: one byte of LDS decides
        if (mine.nf && mine.last == tagg.last) {
            const int hb = msb(dmask);
            uint32_t r8 = s_start * 8u;
            for (int i = 0; i <= hb; ++i) r8 = step_state<NS8>(s_tcomb, cb_lds[i], r8);
            s_last_sa = r8 >> 3;
        }
        __syncthreads();
        my_last_sa = s_last_sa;
    }
    const uint32_t my_ctl_last =
        tile_len > 0 ? (s_ctl[(tile_len - 1) >> 5] >> ((tile_len - 1) & 31)) & 1u : 0u;

    const int Ft = (int)tagg.nf, Rt = (int)tagg.nr;
    const bool staged = Ft <= FCAP && Rt <= RCAP;

    // this tile's count aggregate in the device representation, published
    // before any further work so that successors waiting on it see it early
    const u64 a0 = ((u64)tagg.nr << 31) | tagg.nf;
    u64 a1;
    {
        const u64 colw = (tagg.col & kCAbs) ? ((1ull << 30) | (tagg.col & ~kCAbs)) : tagg.col;
        u64 lastw = my_ctl_last ? (1ull << 29) : 0ull;
        if (lastrel) lastw |= (1ull << 30) | ((u64)my_last_sa << 25) | (u64)(lastrel - 1);
        a1 = (colw << 31) | lastw;
    }
    if (tid == 0 && tile > 0) {
        publish(tw + W_AGG0, kAgg | a0);
        publish(tw + W_AGG1, kAgg | a1);
    }
    if (staged) {
        // ---- 6a. stage the tile's structure in LDS (tile-local; done before the
        // count lookback so that predecessors have time to publish): delimiter
        // positions, column ids and record ends. Fields of the record open at
        // the tile start carry column ids relative to the carried column C0,
        // which the lookback supplies.
        uint32_t L = cex.nf, lr = cex.nr;
        uint32_t col = cex.col & ~kCAbs;
#pragma unroll
        for (int h = 0; h < (B > 32 ? 2 : 1); ++h) {
            uint32_t m = (uint32_t)(dmask >> (32 * h));
            const uint32_t rm = (uint32_t)(rmask >> (32 * h));
            const uint32_t base = (uint32_t)c0 + 32u * h;
            while (m) {
                const uint32_t i = (uint32_t)__builtin_ctz(m);
                m &= m - 1;
                const bool isr = (rm >> i) & 1u;
                s_pos[L] = (uint16_t)(base + i);
                s_colid[L] = (uint8_t)col;
                if (col > 254u) sm.colovf = 1u;
                if (isr) s_recend[lr++] = (uint16_t)L;
                col = isr ? 0u : col + 1u;
                ++L;
            }
        }
        if (vend) {
            s_pos[L] = (uint16_t)tile_len;
            s_colid[L] = (uint8_t)col;
            if (col > 254u) sm.colovf = 1u;
            s_recend[lr] = (uint16_t)L;
        }
    }

    if (wave == 0) {
        const Tot mineT = tot_from_agg(a0, a1, tile_start);
        Tot pre = {0ull, 0ull, kColAbs, 0ull};  // seed: record 0, field 0, column (abs, 0)
        if (tile > 0) {
            bool have = false;
            Tot acc;
            for (int64_t base = (int64_t)tile - 1;; base -= 64) {
                const int64_t j = base - lane;
                u64* pw = p.words + (size_t)(j >= 0 ? j : 0) * kWordsPerTile;
                u64 ir = 0, iF = 0, ic = 0, il = 0, g0 = 0, g1 = 0;
                bool incl_ok = false, agg_ok = false;
                int first;
                for (;;) {
                    if (j >= 0 && !incl_ok) {  // all words of the tile in one round trip
                        ir = peek(pw + W_IREC); iF = peek(pw + W_IFLD);
                        ic = peek(pw + W_ICOL); il = peek(pw + W_ILAST);
                        if (!agg_ok) {
                            g0 = peek(pw + W_AGG0); g1 = peek(pw + W_AGG1);
                        }
                        incl_ok = (ir >> 62) && (iF >> 62) && (ic >> 62) && (il >> 62);
                        agg_ok = agg_ok || ((g0 >> 62) && (g1 >> 62));
                    }
                    if (j < 0) incl_ok = true;  // before tile 0: the seed (never reached)
                    const u64 inc = ballot(incl_ok);
                    const u64 rdy = ballot(incl_ok || agg_ok);
                    first = inc ? __ffsll((long long)inc) - 1 : 64;
                    const u64 need = first >= 63 ? ~0ull : ((2ull << first) - 1);
                    if ((rdy & need) == need) break;
                    __builtin_amdgcn_s_sleep(1);
                }
                Tot x;
                if (lane > first) x = {0ull, 0ull, 0ull, 0ull};
                else if (incl_ok) x = {ir & kPayload, iF & kPayload, ic & kPayload, il & kPayload};
                else x = tot_from_agg(g0, g1, (int64_t)j * TILE);
                if (j < 0) x = {0ull, 0ull, kColAbs, 0ull};
                const Tot w = wave_reduce_desc_tot(x);
                acc = have ? tot_combine(w, acc) : w;
                have = true;
                if (first < 64) break;
            }
            pre = acc;
        }
        const Tot inc = tot_combine(pre, mineT);
        if (lane == 0) {
            publish(tw + W_IREC, kIncl | inc.rec);
            publish(tw + W_IFLD, kIncl | inc.fld);
            publish(tw + W_ICOL, kIncl | inc.col);
            publish(tw + W_ILAST, kIncl | inc.last);
            s_pref[0] = pre.rec;
            s_pref[1] = pre.fld;
            s_pref[2] = pre.col;
            s_pref[3] = pre.last;
        }
    }
    __syncthreads();

    const bool staged2 = staged && sm.colovf == 0u;
    // the tile's prefixes as scalars (every lane is active here)
    const int64_t R0 = (int64_t)readlane0_64(s_pref[0]);
    const int64_t F0 = (int64_t)readlane0_64(s_pref[1]);
    const int64_t C0 = (int64_t)(readlane0_64(s_pref[2]) & kColVal);  // always absolute: seeded with (abs, 0)
    const u64 lastw = readlane0_64(s_pref[3]);
    const int ncols = p.ncols;
    const ByteSrc<SH> src{s_bytes, p.in, tile_start};
    const bool last_has = (lastw & kLastHas) != 0;
    const int64_t last_pos = (int64_t)(lastw & kLastPos);
    const uint32_t last_sa = (uint32_t)((lastw >> 56) & 0xf);
    const bool prev_ctl = (lastw & kLastCtl) != 0;

    // control bit of byte b (b may precede the tile only for the tile's first field)
    auto ctl_at_begin = [&](int64_t b) -> bool {
        if (b >= tile_start) {
            const int r = (int)(b - tile_start);
            return (s_ctl[r >> 5] >> (r & 31)) & 1u;
        }
        const uint32_t by = src(b);
        // b follows the last delimiter before the tile, or is the buffer's
        // first byte (no delimiter before the tile), read in the start state
        const uint32_t s8 = (last_has ? last_sa : (uint32_t)p.start_state) * 8u;
        uint32_t x;
        if constexpr (NS8) x = __builtin_amdgcn_ubfe(s_tcomb[2 * by + (s8 >> 5)], s8 & 31u, 8);
        else x = __builtin_amdgcn_ubfe(s_tcomb[by], s8, 8);
        return (x >> 6) == kTagControl;
    };
    auto ctl_at_end = [&](int64_t e) -> bool {  // control bit of byte e-1
        if (e - 1 >= tile_start) {
            const int r = (int)(e - 1 - tile_start);
            return (s_ctl[r >> 5] >> (r & 31)) & 1u;
        }
        return prev_ctl;
    };

    int64_t nerr = 0, nragged = 0;
    u64 fmin = ~0ull, fmax = 0;  // over the records this thread closes
    if (staged2) {
        {
            const int64_t roomf = p.cap_fields - F0;
            const int kf = roomf < Ft ? (int)(roomf < 0 ? 0 : roomf) : Ft;
            int64_t* const fo = p.field_offsets + F0 + 1;
            int32_t* const ci = p.column_ids + F0;
            const int open_end = Rt ? (int)s_recend[0] + 1 : Ft;  // fields of the record open at the tile start
            for (int k = tid; k < kf; k += NT) {
                put(fo, (uint32_t)k, (tile_start + 1 + s_pos[k]) << SH);
                put(ci, (uint32_t)k, (int32_t)s_colid[k] + (k < open_end ? (int32_t)C0 : 0));
            }
            const int64_t roomr = p.cap_records - R0;
            const int kr = roomr < Rt ? (int)(roomr < 0 ? 0 : roomr) : Rt;
            int64_t* const ro = p.record_offsets + R0 + 1;
            for (int k = tid; k < kr; k += NT) put(ro, (uint32_t)k, F0 + 1 + s_recend[k]);
        }

        // ---- 7. typed columns ---------------------------------------------------------------
        // The records of the tile (those it closes, plus the open one) are cut
        // into blocks of 64 and the columns into contiguous groups; a
        // wavefront takes one (group, record block) pair at a time, a lane
        // one record of the block, and walks the group's columns in order.
        // The column is thus the same for every lane by construction: its
        // type and output bases are wavefront-uniform (scalar branches, no
        // divergence on the type), and the stores into a typed column are
        // contiguous. Walking a group's fields in order reads one delimiter
        // position per field.
        const uint32_t nrec = (uint32_t)Rt + 1u;  // records closed here plus the open one
        const int64_t roomr = p.cap_records - R0;
        const uint32_t lr_cap = roomr <= 0 ? 0u : (roomr > (int64_t)nrec ? nrec : (uint32_t)roomr);
        const bool anyctl = s_anyctl != 0;
        const uint32_t* const words = reinterpret_cast<const uint32_t*>(s_bytes);
        const uint32_t nrb = (nrec + 63u) >> 6;  // record blocks
        uint32_t groups = (uint32_t)NW / nrb;
        groups = groups < 1u ? 1u : (groups > (uint32_t)ncols ? (uint32_t)ncols : groups);
        const uint32_t per = ncols ? ((uint32_t)ncols + groups - 1u) / groups : 0u;  // columns per group
        groups = per ? ((uint32_t)ncols + per - 1u) / per : 0u;
        const uint32_t witems = nrb * groups;
        using KCol = const __attribute__((address_space(4))) ColDesc;
        KCol* const kcols = (KCol*)p.cols;
        // the wavefront's index as a scalar (every lane is active here)
        const uint32_t wv = __builtin_amdgcn_readfirstlane((uint32_t)wave);
        for (uint32_t wi = wv; wi < witems; wi += (uint32_t)NW) {
            const uint32_t g = wi / nrb, rb = wi - g * nrb;
            const uint32_t lr = rb * 64u + (uint32_t)lane;
            if (lr >= nrec) continue;  // idle lanes of the group's last record block
            const uint32_t first = lr ? s_recend[lr - 1] + 1u : 0u;
            const uint32_t end1 = lr < (uint32_t)Rt ? s_recend[lr] + 1u : (uint32_t)Ft;  // one past the last field
            // the open record from the previous tile continues at column C0 (any
            // C0 >= 65535 is beyond every schema column)
            const uint32_t cf = lr ? 0u : (C0 < 65535 ? (uint32_t)C0 : 65535u);
            if (g == 0 && lr < (uint32_t)Rt) {  // the record's field count (exact C0)
                const u64 nf = (lr ? 0ull : (u64)C0) + (end1 - first);
                nragged += nf != (u64)ncols;
                fmin = nf < fmin ? nf : fmin;
                fmax = nf > fmax ? nf : fmax;
            }
            const uint32_t cb = g * per;
            const uint32_t ce = cb + per < (uint32_t)ncols ? cb + per : (uint32_t)ncols;
            const bool st = lr < lr_cap;
            int pend = -1;  // position of the delimiter before the next field, once known
            for (uint32_t c = cb; c < ce; ++c) {
                // Column c's type and output bases through the scalar cache (c
                // is wavefront-uniform; the descriptors stay fixed during the
                // launch), offset to the tile's first record.
                const KCol& kc = kcols[c];
                const uint32_t ty = (uint32_t)kc.type;
                u64* const vals = (u64*)kc.values + R0;
                uint8_t* const valid = (uint8_t*)kc.valid + R0;
                int64_t* const ends = (int64_t*)kc.str_end + R0;
                if (c < cf) continue;
                const uint32_t L = first + c - cf;
                if (__builtin_expect(L >= end1, 0)) {
                    if (lr < (uint32_t)Rt && st && ty != PP_SKIP) {  // missing column of a short record
                        put(vals, lr, (u64)0);
                        put(valid, lr, (uint8_t)0);
                        if (ty == PP_STRING) put(ends, lr, (int64_t)0);
                    }
                    continue;
                }
                int bb, ee;  // tile-relative span; the first field's may begin before the tile
                if (__builtin_expect(L == 0, 0)) {
                    const int64_t e = tile_start + s_pos[0];
                    pend = s_pos[0];
                    if (ty == PP_SKIP) continue;
                    const int64_t hb = last_has ? last_pos + 1 : 0;
                    if (hb < tile_start - kLdsBefore) {  // begins further back than LDS holds: general path
                        const bool cfst = e > hb && ctl_at_begin(hb);
                        const bool clst = e > hb && ctl_at_end(e);
                        if ((ty == PP_INT64 || ty == PP_FLOAT64) && e - hb >= kLongField) {
                            // a long number (it began tiles back): the workgroup
                            // pass converts and stores it (one such field per tile)
                            sm.longq[0] = LongEntry{hb + (int64_t)cfst, e - (int64_t)clst, R0 + lr,
                                                    c | (ty << 16), 0u};
                            sm.nlong = 1u;
                            continue;
                        }
                        nerr += store_field(p, s_cols, src, (int)c, (int)ty, R0 + lr, hb, e, cfst, clst);
                        continue;
                    }
                    bb = (int)(hb - tile_start);
                    ee = s_pos[0];
                    if (ee > bb) {  // strip enclosing control symbols
                        const bool cfst = ctl_at_begin(hb), clst = ctl_at_end(e);
                        if (cfst) ++bb;
                        if (ee - 1 >= bb && clst) --ee;
                    }
                } else {
                    bb = (pend >= 0 ? pend : (int)s_pos[L - 1]) + 1;
                    ee = s_pos[L];
                    pend = ee;
                    if (ty == PP_SKIP) continue;
                    if (anyctl && ee > bb) {  // strip enclosing control symbols
                        if ((s_ctl[bb >> 5] >> (bb & 31)) & 1u) ++bb;
                        if (ee - 1 >= bb && ((s_ctl[(ee - 1) >> 5] >> ((ee - 1) & 31)) & 1u)) --ee;
                    }
                }
                if (ty == PP_STRING) {
                    if (st) {
                        put((int64_t*)vals, lr, (tile_start + bb) << SH);
                        put(ends, lr, (tile_start + ee) << SH);
                        put(valid, lr, (uint8_t)1);
                    }
                } else if (ee == bb) {  // empty: the column default, not an error
                    if (st) {
                        put(vals, lr, (u64)0);
                        put(valid, lr, (uint8_t)0);
                    }
                } else {
                    const int len = ee - bb;
                    int r = -1;
                    u64 bits = 0;
                    if (len <= kWin) {
                        const Win x = load_win_lazy(words, bb, len);
                        if (ty == PP_FLOAT64) {
                            double dv = 0.0;
                            r = wave_any(len > 8) ? ser_float64(x, len, &dv, sm.pow10)
                                                  : ser_float64_8(x, len, &dv, sm.pow10);
                            bits = __builtin_bit_cast(u64, dv);
                        } else {
                            int64_t iv = 0;
                            if (ty == PP_INT64) r = ser_int64(x, len, &iv);
                            else if (ty == PP_TIMESTAMP_S) r = win_timestamp(x, len, &iv);
                            else r = win_date(x, len, &iv);
                            bits = (u64)iv;
                        }
                    }
                    if (__builtin_expect(r < 0, 0)) r = convert_general((int)ty, src, tile_start + bb, tile_start + ee, &bits);
                    nerr += r == 0;
                    if (st) {
                        put(vals, lr, r ? bits : 0ull);
                        put(valid, lr, (uint8_t)r);
                    }
                }
            }
        }
        if (ncols == 0) {  // no column groups above: count the records here
            for (int k = tid; k < Rt; k += NT) {
                const u64 nf = k ? (u64)(s_recend[k] - s_recend[k - 1]) : (u64)C0 + s_recend[0] + 1u;
                nragged += nf != (u64)ncols;
                fmin = nf < fmin ? nf : fmin;
                fmax = nf > fmax ? nf : fmax;
            }
        }
    } else {
        // ---- 6'/7'. per-thread path: each thread closes the fields whose delimiter it holds
        uint32_t L = cex.nf;
        int64_t lr = cex.nr;
        int64_t col = (cex.col & kCAbs) ? (int64_t)(cex.col & ~kCAbs) : C0 + (int64_t)cex.col;
        int64_t prev = cex.last ? tile_start + (int64_t)cex.last - 1 : (last_has ? last_pos : -1);
        M m = dmask;
        const int cnt = (int)popc(dmask) + (int)vend;
        for (int k = 0; k < cnt; ++k) {
            int64_t pos;
            bool isrec;
            if (m) {
                const int i = B > 32 ? __ffsll((long long)m) - 1 : __ffs((int)m) - 1;
                m &= m - 1;
                pos = cstart + i;
                isrec = (rmask >> i) & 1u;
            } else {  // the virtual delimiter at the end of input
                pos = n;
                isrec = true;
            }
            const int64_t f = F0 + L;
            if (f + 1 <= p.cap_fields) gptr(p.field_offsets)[f + 1] = (pos + 1) << SH;
            if (f < p.cap_fields) gptr(p.column_ids)[f] = (int32_t)col;
            const int64_t rec = R0 + lr;
            if (col < ncols) {
                const int ty = s_cols[col].type;
                if (ty != PP_SKIP) {
                    const int64_t b = prev + 1;
                    const bool cfst = pos > b && ctl_at_begin(b);
                    const bool clst = pos > b && ctl_at_end(pos);
                    nerr += store_field(p, s_cols, src, (int)col, ty, rec, b, pos, cfst, clst);
                }
            }
            if (isrec) {
                if (col + 1 != ncols) ++nragged;
                fmin = (u64)(col + 1) < fmin ? (u64)(col + 1) : fmin;
                fmax = (u64)(col + 1) > fmax ? (u64)(col + 1) : fmax;
                for (int64_t c = col + 1; c < ncols; ++c) store_missing(p, s_cols, (int)c, s_cols[c].type, rec);
                if (rec + 1 <= p.cap_records) gptr(p.record_offsets)[rec + 1] = f + 1;
                ++lr;
                col = 0;
            } else {
                ++col;
            }
            prev = pos;
            ++L;
        }
    }

    if (nerr) atomicAdd(&s_err, (u64)nerr);
    if (nragged) atomicAdd(&s_ragged, (u64)nragged);
    // Wavefront reduction of the field counts; the common case, every lane
    // with records holding the same counts, takes no shuffles.
    const u64 hasf = ballot(fmax != 0);
    if (hasf) {
        const int l0 = __ffsll((long long)hasf) - 1;
        const u64 mn0 = readlane64(fmin, l0), mx0 = readlane64(fmax, l0);
        if (ballot(fmax != 0 && (fmin != mn0 || fmax != mx0))) {
#pragma unroll
            for (int d = 32; d; d >>= 1) {
                const u64 a = shfl_xor64(fmin, d), b = shfl_xor64(fmax, d);
                fmin = a < fmin ? a : fmin;
                fmax = b > fmax ? b : fmax;
            }
        } else {
            fmin = mn0;
            fmax = mx0;
        }
        if (lane == 0) {
            atomicMin(&s_fmin, fmin);
            atomicMax(&s_fmax, fmax);
        }
    }
    __syncthreads();
    if (tid == 0) {
        if (s_err) atomicAdd((u64*)&p.result->num_conversion_errors, s_err);  // rare: generic is fine
        if (s_ragged) atomicAdd((u64*)&p.result->num_ragged_records, s_ragged);
        if (s_fmax) {  // results unused: no wait for the atomics before the workgroup ends
            atomicMin((u64*)&p.result->min_record_fields, s_fmin);
            atomicMax((u64*)&p.result->max_record_fields, s_fmax);
        }
        if (tile == (uint32_t)p.num_tiles - 1) {
            const int64_t R = R0 + Rt, F = F0 + Ft;
            const uint32_t fin = s_final;
            int64_t st;
            if (!p.count_only && (R > p.cap_records || F > p.cap_fields)) st = PP_RESULT_CAPACITY;
            else if (p.invalid_state >= 0 && fin == (uint32_t)p.invalid_state) st = PP_RESULT_INVALID_INPUT;
            else if (!((p.accept_mask >> fin) & 1u)) st = PP_RESULT_NON_ACCEPTING_END;
            else st = PP_RESULT_OK;
            PP_GLOBAL pp_result_t* res = gptr(p.result);
            res->num_records = R;
            res->num_fields = F;
            res->final_state = fin;
            res->status = st;
        }
    }
    // Last, so that nothing of the tile stays live across the call:
    // workgroup-uniform (LDS written before the barrier above).
    if (sm.nlong) long_pass<NT, B, SH>(sm);
}

}  // namespace pp
