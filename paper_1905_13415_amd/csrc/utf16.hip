// UTF-16 input (Sec. 4.2, multi-byte symbols): text of 16-bit code units.
//
// The structural symbols of the DFAs are ASCII, and a UTF-16 code unit below
// 0x80 is exactly that ASCII symbol while every other unit (including both
// halves of a surrogate pair) can only be data. So the parse runs over a
// narrowed copy with one byte per code unit: the unit itself below 0x80, byte
// 0x80 for any other (the catch-all group's data). Chunk and tile boundaries
// then fall between code units by construction, which is what Sec. 4.2 asks
// of multi-byte symbols; numbers, dates and times convert from the same
// bytes (a numeral with a non-ASCII digit is not one of the grammar's). The
// outputs' positions are then doubled into byte offsets of the UTF-16 input.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dfa_check.h"
#include "parparaw.h"

namespace {

constexpr size_t kNarrowAlign = 256;
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

size_t narrowed_bytes(int64_t n_units) { return ((size_t)n_units + kNarrowAlign - 1) / kNarrowAlign * kNarrowAlign; }

__device__ __forceinline__ uint8_t narrow1(uint32_t u) { return u < 0x80u ? (uint8_t)u : (uint8_t)0x80u; }

// One byte per code unit; eight units per thread and step through 16-byte
// loads when the input is 16-byte aligned, else one unit at a time.
__global__ void narrow_units(const uint16_t* __restrict__ in, int64_t n, uint8_t* __restrict__ out)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if ((((uintptr_t)in) & 15) == 0) {
        const int64_t groups = n / 8;
        const v4u* in4 = reinterpret_cast<const v4u*>(in);
        for (int64_t g = tid; g < groups; g += stride) {
            const v4u v = __builtin_nontemporal_load(in4 + g);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
            uint32_t lo = 0, hi = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t b = (uint32_t)narrow1(w[k] & 0xffffu) | ((uint32_t)narrow1(w[k] >> 16) << 8);
                if (k < 2) lo |= b << (16 * k);
                else hi |= b << (16 * (k - 2));
            }
            reinterpret_cast<uint2*>(out)[g] = make_uint2(lo, hi);
        }
        for (int64_t i = groups * 8 + tid; i < n; i += stride) out[i] = narrow1(in[i]);
    } else {
        for (int64_t i = tid; i < n; i += stride) out[i] = narrow1(in[i]);
    }
}

struct Widen {
    int64_t* field_offsets;
    const pp_result_t* result;
    int64_t cap_records, cap_fields;
    int32_t nspans;
    int64_t* span[2 * PP_MAX_COLUMNS];  // begin and end arrays of the string columns
};

// Positions in code units -> byte offsets: the field offsets (F + 1 entries
// written), the string spans of the records written, and the first invalid
// offset. blockIdx.y = 0: field offsets; y > 0: span array y - 1.
__global__ void widen_positions(Widen w)
{
    const pp_result_t* r = w.result;
    const int64_t R = r->num_records < w.cap_records ? r->num_records : w.cap_records;
    const int64_t F = r->num_fields < w.cap_fields ? r->num_fields : w.cap_fields;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (blockIdx.y == 0) {
        for (int64_t i = tid; i <= F; i += stride) w.field_offsets[i] *= 2;
    } else {
        int64_t* a = w.span[blockIdx.y - 1];
        for (int64_t i = tid; i < R; i += stride) a[i] *= 2;
    }
}

__global__ void widen_result(pp_result_t* r)
{
    if (threadIdx.x == 0 && r->first_invalid_offset >= 0) r->first_invalid_offset *= 2;
}

}  // namespace

extern "C" size_t pp_workspace_size_utf16(int64_t n_units, const pp_options_t* opts)
{
    if (n_units < 0) return 0;
    const size_t inner = pp_workspace_size(n_units, opts);
    return inner ? narrowed_bytes(n_units) + inner : 0;
}

extern "C" pp_status_t pp_parse_utf16(const uint16_t* d_in, int64_t n_units, const pp_dfa_t* dfa,
                                      const pp_schema_t* schema, const pp_outputs_t* out, void* d_ws,
                                      size_t ws_bytes, const pp_options_t* opts, void* stream)
{
    if (n_units < 0 || (n_units > 0 && !d_in) || !schema || !out || !d_ws || !out->d_result) return PP_ERR_ARG;
    if (!pp::ws_aligned(d_ws)) return PP_ERR_ARG;
    // everything pp_parse would reject is rejected before the narrowing runs
    const pp_status_t dst = pp::check_dfa_tables(dfa);
    if (dst != PP_OK) return dst;
    if (schema->ncols < 0 || schema->ncols > PP_MAX_COLUMNS || (schema->ncols > 0 && !schema->types) ||
        (schema->flags & ~PP_SCHEMA_REJECT_RAGGED))
        return PP_ERR_SCHEMA;
    for (int c = 0; c < schema->ncols; ++c)
        if (schema->types[c] < PP_INT64 || schema->types[c] > PP_SKIP) return PP_ERR_SCHEMA;
    if (opts && opts->tile_order < 0) return PP_ERR_ARG;
    const size_t need = pp_workspace_size_utf16(n_units, opts);
    if (!need) return PP_ERR_ARG;  // no such launch shape
    if (ws_bytes < need) return PP_ERR_WORKSPACE;
    if (out->cap_records < 0 || out->cap_fields < 0 || !out->d_record_offsets || !out->d_field_offsets ||
        (out->cap_fields > 0 && !out->d_column_ids))
        return PP_ERR_ARG;
    if (out->cap_records > 0)
        for (int c = 0; c < schema->ncols; ++c)
            if (schema->types[c] != PP_SKIP &&
                (!out->d_values || !out->d_valid || !out->d_values[c] || !out->d_valid[c]))
                return PP_ERR_ARG;
    // the string columns' span arrays
    Widen w = {};
    w.field_offsets = out->d_field_offsets;
    w.result = out->d_result;
    w.cap_records = out->cap_records;
    w.cap_fields = out->cap_fields;
    if (out->cap_records > 0)
        for (int c = 0; c < schema->ncols; ++c) {
            if (schema->types[c] != PP_STRING) continue;
            if (!out->d_values || !out->d_str_end || !out->d_values[c] || !out->d_str_end[c]) return PP_ERR_ARG;
            w.span[w.nspans++] = (int64_t*)out->d_values[c];
            w.span[w.nspans++] = out->d_str_end[c];
        }
    hipStream_t s = (hipStream_t)stream;
    uint8_t* narrowed = (uint8_t*)d_ws;
    if (n_units > 0) {
        const int64_t work = (n_units + 7) / 8;
        const int blocks = (int)(work / 256 + 1 < 4096 ? work / 256 + 1 : 4096);
        hipLaunchKernelGGL(narrow_units, dim3(blocks), dim3(256), 0, s, d_in, n_units, narrowed);
        if (hipGetLastError() != hipSuccess) return PP_ERR_HIP;
    }
    const size_t off = narrowed_bytes(n_units);
    const pp_status_t st = pp_parse(n_units > 0 ? narrowed : nullptr, n_units, dfa, schema, out,
                                    (char*)d_ws + off, ws_bytes - off, opts, stream);
    if (st != PP_OK) return st;
    const int64_t most = (out->cap_fields > out->cap_records ? out->cap_fields : out->cap_records) + 1;
    const int blocks = (int)(most / 256 + 1 < 2048 ? most / 256 + 1 : 2048);
    hipLaunchKernelGGL(widen_positions, dim3(blocks, 1 + w.nspans), dim3(256), 0, s, w);
    if (hipGetLastError() != hipSuccess) return PP_ERR_HIP;
    hipLaunchKernelGGL(widen_result, dim3(1), dim3(64), 0, s, out->d_result);
    return hipGetLastError() == hipSuccess ? PP_OK : PP_ERR_HIP;
}
