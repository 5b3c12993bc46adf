// Materialised string columns (Sec. 3.3: a column's symbol string holds its
// fields' symbols without the control symbols). After a parse that wrote the
// control-symbol bitmap, a string column's values -- every byte of the
// field's span that is not a control symbol, so the enclosing quotes, the
// first quote of a doubled pair and escape characters go -- are written back
// to back in the Arrow large-string layout: int64 offsets[R + 1] and chars.
//
// Steps (all on the device, one stream, sizes read from the parse's result):
//   1. control symbols per 256-byte block of the input, scanned: the number
//      of control symbols before any byte is a block prefix plus at most
//      eight bitmap words;
//   2. per record, the value's length (span length minus its control
//      symbols) and its number of 4 KiB pieces; both scanned: the offsets,
//      and a piece index that spreads a long field over many wavefronts;
//   3. one wavefront per piece: finds its record by binary search over the
//      piece index, then copies the piece's data bytes, 64 at a time, to
//      their place (a ballot gives each byte's rank among the data bytes).
// A field of any length (tens of MiB) is thus copied by many wavefronts in
// parallel.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "dfa_check.h"
#include "parparaw.h"
#include "scan.h"

namespace {

using pp::kScanItems;
using pp::count_of;
using pp::scan_i64;

constexpr int kBlockBytes = 256;    // bytes per control-count block (8 bitmap words)
constexpr int64_t kPiece = 4096;    // input bytes per gather work item

// ---- control-symbol counts ------------------------------------------------------

__global__ void block_counts(const uint32_t* bitmap, int64_t nwords, int64_t nblocks, int64_t* cb)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nblocks; k += stride) {
        int64_t c = 0;
        for (int w = 0; w < kBlockBytes / 32; ++w) {
            const int64_t i = k * (kBlockBytes / 32) + w;
            if (i < nwords) c += __popc(bitmap[i]);
        }
        cb[k] = c;
    }
}

// control symbols before byte i (i <= n)
__device__ inline int64_t ctl_before(const uint32_t* bitmap, const int64_t* cp, int64_t i)
{
    const int64_t blk = i / kBlockBytes;
    int64_t c = cp[blk];
    const int64_t w0 = blk * (kBlockBytes / 32), w1 = i >> 5;
    for (int64_t w = w0; w < w1; ++w) c += __popc(bitmap[w]);
    const uint32_t part = (uint32_t)(i & 31);
    if (part) c += __popc(bitmap[w1] & ((1u << part) - 1u));
    return c;
}

// SH: log2 of the bytes per symbol (0: bytes; 1: UTF-16 code units, whose
// spans the parse gives in bytes)
template <int SH>
__global__ void value_lengths(const int64_t* begin, const int64_t* end, const uint8_t* valid, int64_t cap,
                              const pp_result_t* res, const uint32_t* bitmap, const int64_t* cp, int64_t* len,
                              int64_t* pieces, int64_t extra)
{
    const int64_t R = count_of(cap, res);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R; r += stride) {
        int64_t l = 0, p = 0;
        if (valid[r]) {
            const int64_t b = begin[r] >> SH, e = end[r] >> SH;
            if (e > b) {
                l = (e - b) - (ctl_before(bitmap, cp, e) - ctl_before(bitmap, cp, b));
                p = (e - b + kPiece - 1) / kPiece;
            }
        }
        len[r] = l + extra;  // extra: the terminator of the inline-terminated form
        pieces[r] = p;
    }
}

// one wavefront per piece of a value; U: the symbol type (byte or code unit)
template <typename U, int SH>
__global__ __launch_bounds__(256) void gather_pieces(const U* in, const int64_t* begin, const int64_t* end,
                                                     int64_t cap, const pp_result_t* res, const uint32_t* bitmap,
                                                     const int64_t* cp, const int64_t* offsets,
                                                     const int64_t* piece_off, U* chars, int64_t cap_chars)
{
    const int64_t R = count_of(cap, res);
    const int64_t total = piece_off[R];
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t q = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); q < total; q += waves) {
        // the record whose pieces hold q: the last r with piece_off[r] <= q
        int64_t lo = 0, hi = R - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (piece_off[mid] <= q) lo = mid;
            else hi = mid - 1;
        }
        const int64_t r = lo;
        const int64_t b = begin[r] >> SH, e = end[r] >> SH;
        const int64_t s0 = b + (q - piece_off[r]) * kPiece;
        const int64_t s1 = s0 + kPiece < e ? s0 + kPiece : e;
        int64_t out = offsets[r] + (s0 - b) - (ctl_before(bitmap, cp, s0) - ctl_before(bitmap, cp, b));
        for (int64_t i0 = s0; i0 < s1; i0 += 64) {
            const int64_t i = i0 + lane;
            bool data = false;
            U sym = 0;
            if (i < s1) {
                data = !((bitmap[i >> 5] >> (i & 31)) & 1u);
                sym = in[i];
            }
            const uint64_t m = __ballot(data);
            const int64_t pos = out + __popcll(m & ((1ull << lane) - 1ull));
            if (data && pos < cap_chars) chars[pos] = sym;
            out += __popcll(m);
        }
    }
}

// the inline-terminated form: the terminator after every value
template <typename U>
__global__ void terminate_values(const int64_t* offsets, int64_t cap, const pp_result_t* res, U* chars,
                                 int64_t cap_chars, U term)
{
    const int64_t R = count_of(cap, res);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R; r += stride) {
        const int64_t at = offsets[r + 1] - 1;
        if (at < cap_chars) chars[at] = term;
    }
}

constexpr size_t align256(size_t x) { return (x + 255) / 256 * 256; }

struct WsLayout {
    size_t cp, pieces, partial, total;
};

WsLayout ws_layout(int64_t n, int64_t cap_records)
{
    const int64_t nblocks = (n + kBlockBytes - 1) / kBlockBytes;
    const int64_t biggest = std::max<int64_t>(nblocks, cap_records) + 1;
    WsLayout w;
    w.cp = 0;
    w.pieces = align256((size_t)(nblocks + 1) * 8);
    w.partial = w.pieces + align256((size_t)(cap_records + 1) * 8);
    w.total = w.partial + align256((size_t)((biggest + kScanItems - 1) / kScanItems + 1) * 8);
    return w;
}

}  // namespace

extern "C" size_t pp_materialize_workspace_size(int64_t n, int64_t cap_records)
{
    if (n < 0 || cap_records < 0) return 0;
    return ws_layout(n, cap_records).total;
}

namespace {

// n: symbols (bytes, or code units); the offsets count symbols
template <typename U, int SH>
pp_status_t materialize(const U* d_in, int64_t n, const pp_outputs_t* parsed, int32_t column, int32_t terminator,
                        int64_t* d_offsets, U* d_chars, int64_t cap_chars, void* d_ws, size_t ws_bytes, void* stream)
{
    if (terminator < -1 || terminator > (SH ? 0xffff : 0xff)) return PP_ERR_ARG;
    if (n < 0 || (n > 0 && !d_in) || !parsed || !parsed->d_result || !d_offsets || cap_chars < 0 ||
        (cap_chars > 0 && !d_chars) || !d_ws || !pp::ws_aligned(d_ws) || column < 0 || column >= PP_MAX_COLUMNS)
        return PP_ERR_ARG;
    const int64_t cap = parsed->cap_records;
    if (cap < 0) return PP_ERR_ARG;
    if (n > 0 && !parsed->d_control_bitmap) return PP_ERR_ARG;  // the parse must have written it
    if (cap > 0 && (!parsed->d_values || !parsed->d_valid || !parsed->d_str_end || !parsed->d_values[column] ||
                    !parsed->d_valid[column] || !parsed->d_str_end[column]))
        return PP_ERR_ARG;  // not a string column of that parse
    const WsLayout w = ws_layout(n, cap);
    if (ws_bytes < w.total) return PP_ERR_WORKSPACE;
    if ((int64_t)(cap / kScanItems + 1) > ((int64_t)1 << 31)) return PP_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)d_ws;
    int64_t* cp = (int64_t*)(ws + w.cp);
    int64_t* pieces = (int64_t*)(ws + w.pieces);
    int64_t* partial = (int64_t*)(ws + w.partial);
    const int64_t nwords = (n + 31) / 32;
    const int64_t nblocks = (n + kBlockBytes - 1) / kBlockBytes;
    const uint32_t* bm = parsed->d_control_bitmap;
    const pp_result_t* res = parsed->d_result;
    auto grid = [](int64_t items) {
        return dim3((unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, (items + 255) / 256)));
    };
    if (nblocks > 0) {
        hipLaunchKernelGGL(block_counts, grid(nblocks), dim3(256), 0, s, bm, nwords, nblocks, cp);
        scan_i64(cp, cp, nblocks, nullptr, partial, s);
    }
    if (cap > 0) {
        const int64_t* begin = (const int64_t*)parsed->d_values[column];
        const int64_t* end = parsed->d_str_end[column];
        const uint8_t* valid = parsed->d_valid[column];
        hipLaunchKernelGGL((value_lengths<SH>), grid(cap), dim3(256), 0, s, begin, end, valid, cap, res, bm, cp,
                           d_offsets, pieces, (int64_t)(terminator >= 0));
        scan_i64(d_offsets, d_offsets, cap, res, partial, s);
        scan_i64(pieces, pieces, cap, res, partial, s);
        hipLaunchKernelGGL((gather_pieces<U, SH>), dim3(2048), dim3(256), 0, s, d_in, begin, end, cap, res, bm, cp,
                           d_offsets, pieces, d_chars, cap_chars);
        if (terminator >= 0)
            hipLaunchKernelGGL((terminate_values<U>), grid(cap), dim3(256), 0, s, d_offsets, cap, res, d_chars,
                               cap_chars, (U)terminator);
    } else {
        scan_i64(d_offsets, d_offsets, 0, res, partial, s);  // offsets[0] = 0
    }
    return hipGetLastError() == hipSuccess ? PP_OK : PP_ERR_HIP;
}

}  // namespace

extern "C" pp_status_t pp_materialize_strings(const uint8_t* d_in, int64_t n, const pp_outputs_t* parsed,
                                              int32_t column, int32_t terminator, int64_t* d_offsets,
                                              uint8_t* d_chars, int64_t cap_chars, void* d_ws, size_t ws_bytes,
                                              void* stream)
{
    return materialize<uint8_t, 0>(d_in, n, parsed, column, terminator, d_offsets, d_chars, cap_chars, d_ws, ws_bytes,
                                   stream);
}

extern "C" pp_status_t pp_materialize_strings_utf16(const uint16_t* d_in, int64_t n_units, const pp_outputs_t* parsed,
                                                    int32_t column, int32_t terminator, int64_t* d_offsets,
                                                    uint16_t* d_chars, int64_t cap_chars, void* d_ws, size_t ws_bytes,
                                                    void* stream)
{
    return materialize<uint16_t, 1>(d_in, n_units, parsed, column, terminator, d_offsets, d_chars, cap_chars, d_ws,
                                    ws_bytes, stream);
}
