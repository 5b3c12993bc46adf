// Single-pass parallel parse of delimiter-separated text on gfx950.
//
// One workgroup of NT threads owns a tile of NT*B input bytes; each thread
// owns a chunk of B bytes (Sec. 3.1 chunks). Per tile, in one kernel:
//   1. stage the tile in LDS with 16-byte loads;
//   2. multi-state pass (Sec. 3.1): per chunk, one DFA instance per state,
//      packed one byte per state in a register; a step is one v_perm_b32
//      (<= 4 states) or two (<= 8 states) that looks every instance up in
//      the byte's transition row: the state-transition vector;
//   3. exclusive composition scan (Sec. 3.1, (a o b)_i = b[a_i]): wave scan
//      by shuffles, block scan through LDS, device scan by decoupled
//      lookback over per-tile words (single-pass scan, Sec. 2);
//   4. tag pass from the chunk's start state: register bitmaps of record
//      delimiters, field delimiters and control symbols (Sec. 3.1);
//   5. record counts (+), field counts (+) and column carries (the abs/rel
//      operator of Sec. 3.2) scanned the same way, one lookback word each;
//   6. delimiter positions staged in LDS, then written coalesced as
//      field_offsets / record_offsets; column ids written per delimiter;
//   7. conversion (Sec. 3.3): the tile's fields are visited column-major,
//      (column, record) pairs, so a wavefront converts one column's type and
//      its stores to that typed column are contiguous. This replaces the
//      paper's radix-sort partition by column: the pair addresses the slot.
// The input is read from HBM once; per-symbol metadata never leaves the chip.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>

#include "convert.h"
#include "parparaw.h"

namespace pp {

constexpr int kTagControl = 1;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

struct ColDesc {
    void* values;
    uint8_t* valid;
    int64_t* str_end;
};

struct Params {
    const uint8_t* in;
    int64_t n;
    int64_t cap_records;
    int64_t cap_fields;
    int64_t* record_offsets;
    int64_t* field_offsets;
    int32_t* column_ids;
    pp_result_t* result;
    unsigned long long* words;  // kWordsPerTile per tile
    unsigned int* counter;      // tile ticket
    int32_t num_tiles;
    int32_t ncols;
    int32_t num_states;
    int32_t start_state;
    int32_t invalid_state;
    uint32_t accept_mask;
    uint8_t group_of[256];
    uint8_t next[PP_MAX_GROUPS][PP_MAX_STATES];
    uint8_t tag[PP_MAX_GROUPS][PP_MAX_STATES];
    uint8_t types[PP_MAX_COLUMNS];
    ColDesc cols[PP_MAX_COLUMNS];
};

// ---- lookback words ----------------------------------------------------------
// Each word is self-contained: [status:2 | payload:62], published and polled
// with relaxed agent-scope atomics (no ordering with other memory is needed).
constexpr int kWordsPerTile = 5;
enum { W_STATE = 0, W_REC = 1, W_FLD = 2, W_COL = 3, W_LAST = 4 };
constexpr unsigned long long kAgg = 1ull << 62, kIncl = 2ull << 62;
constexpr unsigned long long kPayload = (1ull << 62) - 1;
constexpr unsigned long long kColAbs = 1ull << 61;
constexpr unsigned long long kColVal = kColAbs - 1;
// W_LAST payload: has:1 @61 | ctl_last:1 @60 | state_after:4 @56 | pos:56
constexpr unsigned long long kLastHas = 1ull << 61, kLastCtl = 1ull << 60;
constexpr unsigned long long kLastPos = (1ull << 56) - 1;

__device__ inline void publish(unsigned long long* w, unsigned long long v)
{
    __hip_atomic_store(w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline unsigned long long poll(unsigned long long* w)
{
    unsigned long long v;
    while (((v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >> 62) == 0)
        __builtin_amdgcn_s_sleep(1);
    return v;
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
// from src1, 4-7 from src0.
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

template <bool NS8>
__device__ inline SV<NS8> shfl_up_sv(SV<NS8> v, int d)
{
    SV<NS8> r;
    r.lo = (uint32_t)__shfl_up((int)v.lo, d);
    r.hi = NS8 ? (uint32_t)__shfl_up((int)v.hi, d) : 0u;
    return r;
}

// ---- count scan element (Sec. 3.2) ----------------------------------------------
// records, delimiters (fields closed), column carry (bit 31 = abs).
struct Cnt {
    uint32_t nr, nf, col;
};
constexpr uint32_t kCAbs = 1u << 31;

__device__ inline Cnt cnt_combine(Cnt a, Cnt b)
{
    Cnt r;
    r.nr = a.nr + b.nr;
    r.nf = a.nf + b.nf;
    r.col = (b.col & kCAbs) ? b.col : a.col + b.col;  // Sec. 3.2 abs/rel operator
    return r;
}

__device__ inline Cnt shfl_up_cnt(Cnt c, int d)
{
    return {(uint32_t)__shfl_up((int)c.nr, d), (uint32_t)__shfl_up((int)c.nf, d),
            (uint32_t)__shfl_up((int)c.col, d)};
}

// Reads input bytes for conversion: from the LDS tile when inside it, from
// HBM for the head of a field that began in an earlier tile.
struct ByteSrc {
    const uint8_t* lds;
    const uint8_t* g;
    int64_t tile_start;
    __device__ uint32_t operator()(int64_t pos) const
    {
        int64_t r = pos - tile_start;
        return r >= 0 ? lds[r] : g[pos];
    }
};

__device__ inline int64_t wave_sum(int64_t v)
{
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

// ---- the kernel ---------------------------------------------------------------
template <int NT, int B, bool NS8>
__global__ __launch_bounds__(NT) void parse_tiles(Params p)
{
    static_assert(B == 16 || B == 32, "chunk bitmaps are one dword");
    constexpr int TILE = NT * B;
    constexpr int NW = NT / 64;
    static_assert(TILE <= 32768, "u16 positions");

    __shared__ uint32_t s_tnext[NS8 ? 512 : 256];  // byte -> next state of every state
    __shared__ uint32_t s_tcomb[NS8 ? 512 : 256];  // byte -> per state (next*8 | tag<<6)
    __shared__ __align__(16) uint8_t s_bytes[TILE];
    __shared__ uint16_t s_pos[TILE + 2];     // tile-relative delimiter positions
    __shared__ uint16_t s_recend[TILE + 2];  // local field index of each record delimiter
    __shared__ uint32_t s_ctl[TILE / 32];    // control-symbol bitmap of the tile
    __shared__ uint8_t s_types[PP_MAX_COLUMNS];
    __shared__ SV<NS8> s_wsv[NW];
    __shared__ Cnt s_wcnt[NW];
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_s0;
    __shared__ unsigned long long s_pref[4];
    __shared__ int s_lasttid;
    __shared__ uint32_t s_last_sa;
    __shared__ unsigned long long s_last_pos;
    __shared__ uint32_t s_ctl_last;
    __shared__ uint32_t s_final;
    __shared__ unsigned long long s_err, s_ragged;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;

    if (tid == 0) {
        s_tile = atomicAdd(p.counter, 1u);
        s_lasttid = -1;
        s_err = 0;
        s_ragged = 0;
    }
    // per-byte transition rows from the DFA's group table (Table 1 layout)
    for (int b = tid; b < 256; b += NT) {
        const uint32_t g = p.group_of[b];
        uint32_t lo = 0, hi = 0, clo = 0, chi = 0;
        for (int s = 0; s < (NS8 ? 8 : 4); ++s) {
            const bool real = s < p.num_states;
            const uint32_t nx = real ? p.next[g][s] : (uint32_t)s;
            const uint32_t tg = real ? p.tag[g][s] : 0u;
            const uint32_t cb = (nx * 8u) | (tg << 6);
            if (s < 4) { lo |= nx << (8 * s); clo |= cb << (8 * s); }
            else { hi |= nx << (8 * (s - 4)); chi |= cb << (8 * (s - 4)); }
        }
        if constexpr (NS8) {
            s_tnext[2 * b] = lo; s_tnext[2 * b + 1] = hi;
            s_tcomb[2 * b] = clo; s_tcomb[2 * b + 1] = chi;
        } else {
            s_tnext[b] = lo;
            s_tcomb[b] = clo;
        }
    }
    for (int c = tid; c < p.ncols; c += NT) s_types[c] = p.types[c];
    __syncthreads();

    const uint32_t tile = s_tile;
    const int64_t n = p.n;
    const int64_t tile_start = (int64_t)tile * TILE;
    const int tile_len = (int)(n - tile_start < TILE ? n - tile_start : TILE);

    // ---- 1. stage the tile --------------------------------------------------------
    {
        const uint8_t* src = p.in + tile_start;
        if (tile_len == TILE && (((uintptr_t)src) & 15) == 0) {
            const u32x4* s4 = reinterpret_cast<const u32x4*>(src);
            u32x4* d4 = reinterpret_cast<u32x4*>(s_bytes);
#pragma unroll
            for (int k = tid; k < TILE / 16; k += NT) d4[k] = __builtin_nontemporal_load(s4 + k);
        } else {
            for (int k = tid; k < TILE; k += NT) s_bytes[k] = k < tile_len ? src[k] : 0;
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

    // ---- 2. multi-state pass ----------------------------------------------------------
    SV<NS8> vec = sv_identity<NS8>();
    if (len == B) {
#pragma unroll
        for (int i = 0; i < B; ++i) {
            const uint32_t b = byte_at(i);
            SV<NS8> t;
            if constexpr (NS8) { t.lo = s_tnext[2 * b]; t.hi = s_tnext[2 * b + 1]; }
            else { t.lo = s_tnext[b]; t.hi = 0; }
            vec = compose(vec, t);
        }
    } else {
#pragma unroll
        for (int i = 0; i < B; ++i) {
            if (i < len) {
                const uint32_t b = byte_at(i);
                SV<NS8> t;
                if constexpr (NS8) { t.lo = s_tnext[2 * b]; t.hi = s_tnext[2 * b + 1]; }
                else { t.lo = s_tnext[b]; t.hi = 0; }
                vec = compose(vec, t);
            }
        }
    }

    // ---- 3. composition scan ------------------------------------------------------------
    SV<NS8> incl = vec;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        SV<NS8> y = shfl_up_sv(incl, d);
        if (lane >= d) incl = compose(y, incl);
    }
    if (lane == 63) s_wsv[wave] = incl;
    __syncthreads();
    SV<NS8> wpre = sv_identity<NS8>();
    for (int w = 0; w < wave; ++w) wpre = compose(wpre, s_wsv[w]);
    SV<NS8> ex = shfl_up_sv(incl, 1);
    if (lane == 0) ex = sv_identity<NS8>();
    ex = compose(wpre, ex);  // exclusive prefix of this chunk within the tile

    unsigned long long* tw = p.words + (size_t)tile * kWordsPerTile;
    if (tid == 0) {
        SV<NS8> agg = sv_identity<NS8>();
        for (int w = 0; w < NW; ++w) agg = compose(agg, s_wsv[w]);
        SV<NS8> pre = sv_identity<NS8>();
        if (tile == 0) {
            publish(tw + W_STATE, kIncl | sv_to_nib(agg));
        } else {
            publish(tw + W_STATE, kAgg | sv_to_nib(agg));
            SV<NS8> acc = sv_identity<NS8>();
            for (int64_t j = (int64_t)tile - 1;; --j) {
                unsigned long long v = poll(p.words + (size_t)j * kWordsPerTile + W_STATE);
                acc = compose(sv_from_nib<NS8>((uint32_t)v), acc);
                if ((v >> 62) == 2) break;
            }
            pre = acc;
            publish(tw + W_STATE, kIncl | sv_to_nib(compose(acc, agg)));
        }
        s_s0 = sv_get(pre, (uint32_t)p.start_state);
        s_final = sv_get(compose(pre, agg), (uint32_t)p.start_state);
    }
    __syncthreads();
    const uint32_t s_start = sv_get(ex, s_s0);

    // ---- 4. tag pass ----------------------------------------------------------------------
    // x = tcomb[b] >> (8*state): bits 3-5 next state * 8, bit 6 tag bit 0, bit 7 tag bit 1.
    uint32_t p0 = 0, p1 = 0, s8 = s_start * 8u;
    auto step = [&](int i) {
        const uint32_t b = byte_at(i);
        uint32_t x;
        if constexpr (NS8) {
            const uint32_t e = s_tcomb[2 * b + (s8 >> 5)];
            x = __builtin_amdgcn_ubfe(e, s8 & 31u, 8);
        } else {
            x = __builtin_amdgcn_ubfe(s_tcomb[b], s8, 8);
        }
        s8 = x & 0x38u;
        p0 |= ((x >> 6) & 1u) << i;
        p1 |= (x >> 7) << i;
    };
    if (len == B) {
#pragma unroll
        for (int i = 0; i < B; ++i) step(i);
    } else {
#pragma unroll
        for (int i = 0; i < B; ++i)
            if (i < len) step(i);
    }
    const uint32_t s_end = s8 >> 3;
    const uint32_t dmask = p1, rmask = p1 & p0, cmask = p0 & ~p1;
    const int64_t cstart = tile_start + c0;
    const bool holds_last = len > 0 && cstart + len == n;
    const uint32_t vend = holds_last && !((rmask >> (len - 1)) & 1u);  // end of input closes a record

    // first transition into the (absorbing) invalid state
    if (p.invalid_state >= 0 && s_start != (uint32_t)p.invalid_state && s_end == (uint32_t)p.invalid_state) {
        uint32_t s = s_start;
        for (int i = 0; i < len; ++i) {
            const uint32_t g = p.group_of[s_bytes[c0 + i]];
            const uint32_t nx = p.next[g][s];
            if (nx == (uint32_t)p.invalid_state) {
                p.result->first_invalid_offset = cstart + i;
                break;
            }
            s = nx;
        }
    }

    Cnt mine;
    mine.nr = __popc(rmask) + vend;
    mine.nf = __popc(dmask) + vend;
    if (rmask | vend) {
        uint32_t after = 0;
        if (!vend) {
            const int hb = 31 - __clz(rmask);
            after = hb == 31 ? 0u : __popc(dmask & ~rmask & (~0u << (hb + 1)));
        }
        mine.col = kCAbs | after;
    } else {
        mine.col = __popc(dmask);
    }
    if constexpr (B == 32) {
        s_ctl[tid] = cmask;
    } else {  // two 16-byte chunks per bitmap word
        const uint32_t part = cmask << ((tid & 1) * 16);
        const uint32_t other = (uint32_t)__shfl_xor((int)part, 1);
        if ((tid & 1) == 0) s_ctl[tid >> 1] = part | other;
    }

    // ---- 5. count scans ------------------------------------------------------------------
    Cnt cin = mine;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        Cnt y = shfl_up_cnt(cin, d);
        if (lane >= d) cin = cnt_combine(y, cin);
    }
    if (lane == 63) s_wcnt[wave] = cin;
    if (mine.nf) atomicMax(&s_lasttid, tid);
    __syncthreads();
    Cnt cpre = {0u, 0u, 0u};
    for (int w = 0; w < wave; ++w) cpre = cnt_combine(cpre, s_wcnt[w]);
    Cnt cex = shfl_up_cnt(cin, 1);
    if (lane == 0) cex = {0u, 0u, 0u};
    cex = cnt_combine(cpre, cex);

    // position of the tile's last delimiter and the state after it, found by
    // the chunk that holds it (a virtual end-of-input delimiter sits at n)
    if (tid == s_lasttid) {
        uint32_t sa = 0;
        int64_t pos = n;
        if (!vend) {
            const int hb = 31 - __clz(dmask);
            uint32_t s = s_start;
            for (int i = 0; i <= hb; ++i) s = p.next[p.group_of[s_bytes[c0 + i]]][s];
            sa = s;
            pos = cstart + hb;
        }
        s_last_sa = sa;
        s_last_pos = (unsigned long long)pos;
    }
    if (len > 0 && c0 + len == tile_len) s_ctl_last = (cmask >> (len - 1)) & 1u;
    __syncthreads();

    if (tid < 4) {
        Cnt agg = {0u, 0u, 0u};
        for (int w = 0; w < NW; ++w) agg = cnt_combine(agg, s_wcnt[w]);
        unsigned long long a;
        if (tid == 0) a = agg.nr;
        else if (tid == 1) a = agg.nf;
        else if (tid == 2) a = (agg.col & kCAbs) ? (kColAbs | (agg.col & ~kCAbs)) : agg.col;
        else {
            a = s_ctl_last ? kLastCtl : 0ull;
            if (s_lasttid >= 0)
                a |= kLastHas | ((unsigned long long)s_last_sa << 56) | (s_last_pos & kLastPos);
        }
        auto comb = [&](unsigned long long x, unsigned long long y) -> unsigned long long {
            if (tid <= 1) return (x + y) & kPayload;
            if (tid == 2) return (y & kColAbs) ? y : ((x + y) & kPayload);
            // last delimiter: the later one wins; control bit of the last byte from y
            unsigned long long r = (y & kLastHas) ? (y & ~kLastCtl) : (x & ~kLastCtl);
            return r | (y & kLastCtl);
        };
        unsigned long long seed = tid == 2 ? kColAbs : 0ull;
        unsigned long long* wp = tw + W_REC + tid;
        unsigned long long pre;
        if (tile == 0) {
            pre = seed;
            publish(wp, kIncl | comb(seed, a));
        } else {
            publish(wp, kAgg | a);
            unsigned long long acc = 0;  // identity of every operator: rel 0, no delimiter
            bool first = true;
            for (int64_t j = (int64_t)tile - 1;; --j) {
                unsigned long long v = poll(p.words + (size_t)j * kWordsPerTile + W_REC + tid);
                unsigned long long val = v & kPayload;
                acc = first ? val : comb(val, acc);
                first = false;
                if ((v >> 62) == 2) break;
            }
            pre = acc;
            publish(wp, kIncl | comb(acc, a));
        }
        s_pref[tid] = pre;
    }
    __syncthreads();

    const int64_t R0 = (int64_t)s_pref[0];
    const int64_t F0 = (int64_t)s_pref[1];
    const int64_t C0 = (int64_t)(s_pref[2] & kColVal);
    const unsigned long long lastw = s_pref[3];
    Cnt tagg = {0u, 0u, 0u};
    for (int w = 0; w < NW; ++w) tagg = cnt_combine(tagg, s_wcnt[w]);
    const int Ft = (int)tagg.nf, Rt = (int)tagg.nr;

    // ---- 6. emit structure ------------------------------------------------------------------
    {
        uint32_t L = cex.nf, lr = cex.nr;
        int64_t col = (cex.col & kCAbs) ? (int64_t)(cex.col & ~kCAbs) : C0 + (int64_t)cex.col;
        uint32_t m = dmask;
        while (m) {
            const int i = __ffs(m) - 1;
            m &= m - 1;
            s_pos[L] = (uint16_t)(c0 + i);
            if (F0 + L < p.cap_fields) p.column_ids[F0 + L] = (int32_t)col;
            if ((rmask >> i) & 1u) { s_recend[lr++] = (uint16_t)L; col = 0; }
            else ++col;
            ++L;
        }
        if (vend) {
            s_pos[L] = (uint16_t)tile_len;
            if (F0 + L < p.cap_fields) p.column_ids[F0 + L] = (int32_t)col;
            s_recend[lr++] = (uint16_t)L;
        }
    }
    __syncthreads();
    for (int k = tid; k < Ft; k += NT) {
        const int64_t f = F0 + 1 + k;
        if (f <= p.cap_fields) p.field_offsets[f] = tile_start + s_pos[k] + 1;
    }
    for (int k = tid; k < Rt; k += NT) {
        const int64_t r = R0 + 1 + k;
        if (r <= p.cap_records) p.record_offsets[r] = F0 + s_recend[k] + 1;
    }

    // ---- 7. typed columns, column-major over (column, local record) ------------------------
    const int ncols = p.ncols;
    const int nrec = Rt + 1;  // records closed here plus the open one
    const int items = nrec * ncols;
    const float rcp = 1.0f / (float)nrec;
    const ByteSrc src{s_bytes, p.in, tile_start};
    const bool last_has = (lastw & kLastHas) != 0;
    const int64_t last_pos = (int64_t)(lastw & kLastPos);
    const uint32_t last_sa = (uint32_t)((lastw >> 56) & 0xf);
    const bool prev_ctl = (lastw & kLastCtl) != 0;
    int64_t nerr = 0, nragged = 0;
    for (int q = tid; q < items; q += NT) {
        int c = (int)((float)q * rcp);
        if (c * nrec > q) --c;
        else if ((c + 1) * nrec <= q) ++c;
        const int lr = q - c * nrec;
        const int first = lr == 0 ? 0 : s_recend[lr - 1] + 1;
        const int64_t cf = lr == 0 ? C0 : 0;
        const int last = lr < Rt ? (int)s_recend[lr] : Ft - 1;
        const int64_t rec = R0 + lr;
        if (c == 0 && lr < Rt && cf + (last - first + 1) != ncols) ++nragged;
        if (c < cf) continue;
        const int64_t Lz = first + (c - cf);
        const int ty = s_types[c];
        if (ty == PP_SKIP) continue;
        ColDesc cd = p.cols[c];
        if (Lz > last) {
            if (lr < Rt && rec < p.cap_records) {  // missing column of a short record
                ((int64_t*)cd.values)[rec] = 0;  // 0 and 0.0 share the bit pattern
                cd.valid[rec] = 0;
                if (ty == PP_STRING) cd.str_end[rec] = 0;
            }
            continue;
        }
        const int L = (int)Lz;
        const int64_t e = tile_start + s_pos[L];
        const int64_t b = L == 0 ? (last_has ? last_pos + 1 : 0) : tile_start + s_pos[L - 1] + 1;
        // strip one leading and one trailing control symbol (enclosing quotes)
        int64_t begin = b, end = e;
        if (end > begin) {
            bool ctl;
            if (b >= tile_start) {
                const int r = (int)(b - tile_start);
                ctl = (s_ctl[r >> 5] >> (r & 31)) & 1u;
            } else {
                uint32_t x;
                const uint32_t by = p.in[b];
                if constexpr (NS8) x = __builtin_amdgcn_ubfe(s_tcomb[2 * by + (last_sa >> 2)], (last_sa & 3) * 8, 8);
                else x = __builtin_amdgcn_ubfe(s_tcomb[by], last_sa * 8, 8);
                ctl = (x >> 6) == (uint32_t)kTagControl;
            }
            if (ctl) ++begin;
        }
        if (end - 1 >= begin) {
            bool ctl;
            if (e - 1 >= tile_start) {
                const int r = (int)(e - 1 - tile_start);
                ctl = (s_ctl[r >> 5] >> (r & 31)) & 1u;
            } else {
                ctl = prev_ctl;
            }
            if (ctl) --end;
        }
        if (rec >= p.cap_records) {
            // still count conversion errors so the result does not depend on capacity
            if (ty != PP_STRING && end > begin) {
                bool ok;
                int64_t iv;
                double dv;
                if (ty == PP_INT64) ok = conv_int64(src, begin, end, &iv);
                else if (ty == PP_FLOAT64) ok = conv_float64(src, begin, end, &dv);
                else if (ty == PP_TIMESTAMP_S) ok = conv_timestamp(src, begin, end, &iv);
                else ok = conv_date(src, begin, end, &iv);
                nerr += !ok;
            }
            continue;
        }
        if (ty == PP_STRING) {
            ((int64_t*)cd.values)[rec] = begin;
            cd.str_end[rec] = end;
            cd.valid[rec] = 1;
        } else if (end == begin) {
            ((int64_t*)cd.values)[rec] = 0;
            cd.valid[rec] = 0;
        } else if (ty == PP_FLOAT64) {
            double dv = 0.0;
            const bool ok = conv_float64(src, begin, end, &dv);
            ((double*)cd.values)[rec] = ok ? dv : 0.0;
            cd.valid[rec] = ok;
            nerr += !ok;
        } else {
            int64_t iv = 0;
            bool ok;
            if (ty == PP_INT64) ok = conv_int64(src, begin, end, &iv);
            else if (ty == PP_TIMESTAMP_S) ok = conv_timestamp(src, begin, end, &iv);
            else ok = conv_date(src, begin, end, &iv);
            ((int64_t*)cd.values)[rec] = ok ? iv : 0;
            cd.valid[rec] = ok;
            nerr += !ok;
        }
    }
    if (ncols == 0 && tid == 0) nragged = Rt;
    nerr = wave_sum(nerr);
    nragged = wave_sum(nragged);
    if (lane == 0 && (nerr | nragged)) {
        atomicAdd(&s_err, (unsigned long long)nerr);
        atomicAdd(&s_ragged, (unsigned long long)nragged);
    }
    __syncthreads();
    if (tid == 0) {
        if (s_err) atomicAdd((unsigned long long*)&p.result->num_conversion_errors, s_err);
        if (s_ragged) atomicAdd((unsigned long long*)&p.result->num_ragged_records, s_ragged);
        if (tile == (uint32_t)p.num_tiles - 1) {
            const int64_t R = R0 + Rt, F = F0 + Ft;
            const uint32_t fin = s_final;
            int64_t st;
            if (R > p.cap_records || F > p.cap_fields) st = PP_RESULT_CAPACITY;
            else if (p.invalid_state >= 0 && fin == (uint32_t)p.invalid_state) st = PP_RESULT_INVALID_INPUT;
            else if (!((p.accept_mask >> fin) & 1u)) st = PP_RESULT_NON_ACCEPTING_END;
            else st = PP_RESULT_OK;
            p.result->num_records = R;
            p.result->num_fields = F;
            p.result->final_state = fin;
            p.result->status = st;
        }
    }
}

// Resets the workspace and the result before a parse; writes the outputs of
// an empty input. Plain stores only, so the pair of launches can be captured.
__global__ void parse_init(Params p, size_t nwords)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (size_t k = i; k < nwords; k += (size_t)gridDim.x * blockDim.x) p.words[k] = 0ull;
    if (i == 0) {
        *p.counter = 0u;
        pp_result_t* r = p.result;
        r->first_invalid_offset = -1;
        r->num_conversion_errors = 0;
        r->num_ragged_records = 0;
        r->num_records = 0;
        r->num_fields = 0;
        r->final_state = p.start_state;
        r->status = ((p.accept_mask >> p.start_state) & 1u) ? PP_RESULT_OK : PP_RESULT_NON_ACCEPTING_END;
        if (p.record_offsets && p.cap_records >= 0) p.record_offsets[0] = 0;
        if (p.field_offsets && p.cap_fields >= 0) p.field_offsets[0] = 0;
    }
}

// ---- host side ------------------------------------------------------------------------

constexpr int kDefaultNT = 256;
constexpr int kDefaultB = 32;

static int tile_bytes(const pp_options_t* o)
{
    int nt = (o && o->block_threads) ? o->block_threads : kDefaultNT;
    int b = (o && o->bytes_per_thread) ? o->bytes_per_thread : kDefaultB;
    return nt * b;
}

static bool options_ok(const pp_options_t* o)
{
    if (!o) return true;
    int nt = o->block_threads ? o->block_threads : kDefaultNT;
    int b = o->bytes_per_thread ? o->bytes_per_thread : kDefaultB;
    return nt == 256 && (b == 16 || b == 32);
}

static pp_status_t check_dfa(const pp_dfa_t* d)
{
    if (!d) return PP_ERR_ARG;
    if (d->num_states < 1 || d->num_states > PP_MAX_STATES) return PP_ERR_DFA;
    if (d->num_groups < 1 || d->num_groups > PP_MAX_GROUPS) return PP_ERR_DFA;
    if (d->start_state < 0 || d->start_state >= d->num_states) return PP_ERR_DFA;
    if (d->invalid_state < -1 || d->invalid_state >= d->num_states) return PP_ERR_DFA;
    for (int b = 0; b < 256; ++b)
        if (d->group_of[b] >= d->num_groups) return PP_ERR_DFA;
    for (int g = 0; g < d->num_groups; ++g)
        for (int s = 0; s < d->num_states; ++s) {
            if (d->next[g][s] >= d->num_states || d->tag[g][s] > PP_TAG_RECORD) return PP_ERR_DFA;
            if (s == d->invalid_state && d->next[g][s] != s) return PP_ERR_DFA;  // must absorb
        }
    return PP_OK;
}

}  // namespace pp

using namespace pp;

extern "C" size_t pp_workspace_size(int64_t n, const pp_options_t* opts)
{
    if (n < 0 || !options_ok(opts)) return 0;
    const int64_t tb = tile_bytes(opts);
    const int64_t tiles = (n + tb - 1) / tb;
    return 256 + (size_t)tiles * kWordsPerTile * sizeof(unsigned long long);
}

extern "C" pp_status_t pp_parse(const uint8_t* d_in, int64_t n, const pp_dfa_t* dfa,
                                const pp_schema_t* schema, const pp_outputs_t* out, void* d_ws,
                                size_t ws_bytes, const pp_options_t* opts, void* stream)
{
    if (n < 0 || (n > 0 && !d_in) || !schema || !out || !d_ws || !out->d_result) return PP_ERR_ARG;
    if (!options_ok(opts)) return PP_ERR_ARG;
    if (out->cap_records < 0 || out->cap_fields < 0) return PP_ERR_ARG;
    if (!out->d_record_offsets || !out->d_field_offsets) return PP_ERR_ARG;
    if (out->cap_fields > 0 && !out->d_column_ids) return PP_ERR_ARG;
    if (n >= (1ll << 55)) return PP_ERR_UNSUPPORTED;
    pp_status_t st = check_dfa(dfa);
    if (st != PP_OK) return st;
    if (schema->ncols < 0 || schema->ncols > PP_MAX_COLUMNS) return PP_ERR_SCHEMA;
    if (schema->ncols > 0 && !schema->types) return PP_ERR_SCHEMA;
    if (ws_bytes < pp_workspace_size(n, opts)) return PP_ERR_WORKSPACE;

    Params p;
    memset(&p, 0, sizeof p);
    p.in = d_in;
    p.n = n;
    p.cap_records = out->cap_records;
    p.cap_fields = out->cap_fields;
    p.record_offsets = out->d_record_offsets;
    p.field_offsets = out->d_field_offsets;
    p.column_ids = out->d_column_ids;
    p.result = out->d_result;
    p.counter = (unsigned int*)d_ws;
    p.words = (unsigned long long*)((char*)d_ws + 256);
    const int tb = tile_bytes(opts);
    const int64_t tiles = (n + tb - 1) / tb;
    if (tiles > 0x7fffffff) return PP_ERR_UNSUPPORTED;
    p.num_tiles = (int32_t)tiles;
    p.ncols = schema->ncols;
    p.num_states = dfa->num_states;
    p.start_state = dfa->start_state;
    p.invalid_state = dfa->invalid_state;
    p.accept_mask = dfa->accept_mask;
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
        p.types[c] = (uint8_t)ty;
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
    const int init_blocks = (int)std::min<size_t>(1024, (nwords + 255) / 256 + 1);
    hipLaunchKernelGGL(parse_init, dim3(init_blocks), dim3(256), 0, s, p, nwords);
    if (hipGetLastError() != hipSuccess) return PP_ERR_HIP;
    if (tiles == 0) return PP_OK;
    const int b = (opts && opts->bytes_per_thread) ? opts->bytes_per_thread : kDefaultB;
    const bool ns8 = dfa->num_states > 4;
    if (b == 32) {
        if (ns8) hipLaunchKernelGGL((parse_tiles<256, 32, true>), dim3((unsigned)tiles), dim3(256), 0, s, p);
        else hipLaunchKernelGGL((parse_tiles<256, 32, false>), dim3((unsigned)tiles), dim3(256), 0, s, p);
    } else {
        if (ns8) hipLaunchKernelGGL((parse_tiles<256, 16, true>), dim3((unsigned)tiles), dim3(256), 0, s, p);
        else hipLaunchKernelGGL((parse_tiles<256, 16, false>), dim3((unsigned)tiles), dim3(256), 0, s, p);
    }
    if (hipGetLastError() != hipSuccess) return PP_ERR_HIP;
    return PP_OK;
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
    }
    return "unknown status";
}
