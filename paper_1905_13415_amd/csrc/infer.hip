// Type inference (Sec. 4.3): after a parse whose columns are string spans,
// every non-empty field is checked against each type's grammar -- INT64
// (converts without overflow), FLOAT64 (the float grammar), DATE_DAYS and
// TIMESTAMP_S (valid calendar values) -- and a column keeps the types all of
// its fields admit (an AND over the fields, reduced per wavefront and
// workgroup, then one atomic per workgroup). The inferred type is the first
// kept type in the order INT64, FLOAT64, DATE_DAYS, TIMESTAMP_S, else STRING
// (also for a column without non-empty fields). A field's checks stop at its
// first byte that no candidate type accepts, so long text costs little; a
// field of kInferLong bytes or more (it can only be a number or text) is
// queued and checked by a whole workgroup afterwards (Sec. 3.3's block
// level), the symbols classified a word at a time in parallel.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>

#include "convert.h"
#include "dfa_check.h"
#include "parparaw.h"
#include "tile.h"

namespace {

enum : uint32_t { OK_INT = 1, OK_FLOAT = 2, OK_DATE = 4, OK_TS = 8, OK_ALL = 15 };

struct ColSpans {
    const int64_t* begin[PP_MAX_COLUMNS];
    const int64_t* end[PP_MAX_COLUMNS];
    const uint8_t* valid[PP_MAX_COLUMNS];
};

// Fields this long are checked by a workgroup (kInferLongCap of them per
// call; any more by their own thread).
constexpr int64_t kInferLong = 4096;
constexpr int kInferLongCap = 1024;
struct LongSpan {
    int64_t b, e;
    int32_t col, pad;
};
// workspace: [admitted-type masks, ncols words, padded to 16 B] [queue count, 16 B] [queue]
size_t mask_bytes(int32_t ncols) { return ((size_t)std::max(ncols, 1) * sizeof(uint32_t) + 15) / 16 * 16; }

struct GlobalBytes {
    const uint8_t* p;
    __device__ uint32_t operator()(int64_t i) const { return p[i]; }
};

__global__ void infer_init(uint32_t* mask, int64_t* nonempty, int32_t ncols, uint32_t* qcount)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncols) {
        mask[c] = OK_ALL;
        nonempty[c] = 0;
    }
    if (c == 0) *qcount = 0u;
}

__device__ uint32_t field_admits(const GlobalBytes& src, int64_t b, int64_t e)
{
    uint32_t m = 0;
    int64_t v = 0;
    if (pp::conv_int64(src, b, e, &v)) m |= OK_INT;
    if (pp::float_grammar(src, b, e)) m |= OK_FLOAT;
    if (pp::conv_date(src, b, e, &v)) m |= OK_DATE;
    if (pp::conv_timestamp(src, b, e, &v)) m |= OK_TS;
    return m;
}

// grid: (x: record blocks, y: column)
__global__ __launch_bounds__(256) void infer_fields(const uint8_t* in, ColSpans cs, int64_t cap,
                                                    const pp_result_t* res, uint32_t* mask, int64_t* nonempty,
                                                    uint32_t* qcount, LongSpan* queue)
{
    __shared__ uint32_t s_and[4];
    __shared__ unsigned long long s_cnt[4];
    const int c = blockIdx.y;
    const int64_t R0 = res->num_records;
    const int64_t R = R0 < cap ? R0 : cap;
    const GlobalBytes src{in};
    uint32_t acc = OK_ALL;
    unsigned long long cnt = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R; r += stride) {
        if (!cs.valid[c][r]) continue;
        const int64_t b = cs.begin[c][r], e = cs.end[c][r];
        if (e <= b) continue;  // empty: no constraint
        ++cnt;
        if (e - b >= kInferLong) {  // to the workgroup pass, while the queue has room
            const uint32_t k = atomicAdd(qcount, 1u);
            if (k < (uint32_t)kInferLongCap) {
                queue[k] = LongSpan{b, e, c, 0};
                continue;
            }
        }
        acc &= field_admits(src, b, e);
    }
    for (int d = 32; d; d >>= 1) {
        acc &= (uint32_t)__shfl_xor((int)acc, d);
        cnt += __shfl_xor(cnt, d);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_and[w] = acc;
        s_cnt[w] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = OK_ALL;
        unsigned long long n = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
            a &= s_and[k];
            n += s_cnt[k];
        }
        if (n) {
            atomicAnd(mask + c, a);
            atomicAdd((unsigned long long*)(nonempty + c), n);
        }
    }
}

// The queued long fields, a workgroup each: the types the field admits.
// INT64: [+-]?[0-9]+ with at most 19 significant digits that fit; FLOAT64:
// the float grammar (at most one exponent mark, a sign only right after it,
// at most one point and none after the mark, at least one mantissa digit and
// one exponent digit); DATE_DAYS and TIMESTAMP_S have fixed lengths far
// below kInferLong. Same answers as field_admits.
__global__ __launch_bounds__(256) void infer_long(const uint8_t* in, const uint32_t* qcount, const LongSpan* queue,
                                                 uint32_t* mask)
{
    constexpr int NT = 256;
    constexpr unsigned long long NONE = ~0ull;
    __shared__ unsigned long long red[8];
    const int tid = threadIdx.x, lane = tid & 63;
    const uint32_t nq = *qcount < (uint32_t)kInferLongCap ? *qcount : (uint32_t)kInferLongCap;
    auto rmin = [&](int k, unsigned long long v) {
        v = pp::wave_min_u64(v);
        if (lane == 0 && v != NONE) atomicMin(&red[k], v);
    };
    auto rmax = [&](int k, unsigned long long v) {
        v = pp::wave_max_u64(v);
        if (lane == 0 && v) atomicMax(&red[k], v);
    };
    auto rsum = [&](int k, unsigned long long v) {
        v = pp::wave_sum_u64(v);
        if (lane == 0 && v) atomicAdd(&red[k], v);
    };
    for (uint32_t q = blockIdx.x; q < nq; q += gridDim.x) {
        const LongSpan f = queue[q];
        const int64_t b = f.b, e = f.e;
        const uint32_t c0 = in[b];
        const bool neg = c0 == '-', sg = neg || c0 == '+';
        const int64_t s0 = b + (sg ? 1 : 0);
        if (tid < 8) red[tid] = (tid == 0 || tid == 7) ? NONE : 0ull;
        __syncthreads();
        // marks (first red[0], count red[1]), points (count red[2], last
        // red[3] + 1), other symbols (red[4]), signs (count red[5], last
        // red[6] + 1), first nonzero digit (red[7])
        unsigned long long em = NONE, ne = 0, ndot = 0, dpos = 0, nbad = 0, nsg = 0, spos = 0, fnz = NONE;
        pp::scan_symbols<NT, 0>(
            in, s0, e,
            [&](int64_t i, uint32_t c) {
                const bool d = c - '0' < 10u, dot = c == '.', mk = (c | 0x20u) == 'e', sgn = c == '+' || c == '-';
                ne += mk;
                if (mk && (unsigned long long)i < em) em = (unsigned long long)i;
                ndot += dot;
                if (dot && (unsigned long long)i + 1 > dpos) dpos = (unsigned long long)i + 1;
                nsg += sgn;
                if (sgn && (unsigned long long)i + 1 > spos) spos = (unsigned long long)i + 1;
                nbad += !d && !dot && !mk && !sgn;
                if (c - '1' < 9u && (unsigned long long)i < fnz) fnz = (unsigned long long)i;
            },
            [&](int64_t i, uint32_t w) {
                const uint32_t nd = pp::nondigit_bytes(w), nz = ~nd & ~pp::zerodigit_bytes(w) & 0x80808080u;
                if (nz && fnz == NONE) fnz = (unsigned long long)(i + pp::first_byte(nz));
                if (nd == 0u) return;
                const uint32_t pt = pp::point_bytes(w), mk = pp::expmark_bytes(w);
                const uint32_t sgb = pp::zero_bytes(w ^ 0x2b2b2b2bu) | pp::zero_bytes(w ^ 0x2d2d2d2du);
                if (mk) {
                    ne += (unsigned long long)__popc(mk);
                    const unsigned long long x = (unsigned long long)(i + pp::first_byte(mk));
                    em = x < em ? x : em;
                }
                if (pt) {
                    ndot += (unsigned long long)__popc(pt);
                    const unsigned long long x = (unsigned long long)(i + pp::last_byte(pt)) + 1;
                    dpos = x > dpos ? x : dpos;
                }
                if (sgb) {
                    nsg += (unsigned long long)__popc(sgb);
                    const unsigned long long x = (unsigned long long)(i + pp::last_byte(sgb)) + 1;
                    spos = x > spos ? x : spos;
                }
                nbad += (unsigned long long)__popc(nd & ~pt & ~mk & ~sgb);
            });
        rmin(0, em);
        rsum(1, ne);
        rsum(2, ndot);
        rmax(3, dpos);
        rsum(4, nbad);
        rsum(5, nsg);
        rmax(6, spos);
        rmin(7, fnz);
        __syncthreads();
        if (tid == 0) {
            const unsigned long long nmark = red[1], ndots = red[2], nsigns = red[5];
            uint32_t m = 0;
            // INT64: digits only after the sign, at most 19 significant, within range
            if (s0 < e && nmark == 0 && ndots == 0 && nsigns == 0 && red[4] == 0) {
                if (red[7] == NONE) {
                    m |= OK_INT;  // all zeros
                } else if (e - (int64_t)red[7] <= 19) {
                    const uint64_t limit = neg ? (1ull << 63) : (1ull << 63) - 1;
                    uint64_t mag = 0;
                    bool fits = true;
                    for (int64_t i = (int64_t)red[7]; i < e && fits; ++i) {
                        const uint32_t d = in[i] - '0';
                        if (mag > (limit - d) / 10u) fits = false;
                        else mag = mag * 10u + d;
                    }
                    if (fits) m |= OK_INT;
                }
            }
            // FLOAT64 grammar
            const int64_t E = nmark ? (int64_t)red[0] : e;
            const bool esg = nsigns == 1 && (int64_t)red[6] - 1 == E + 1;
            const int64_t x0 = E + 1 + (esg ? 1 : 0);
            const int64_t dotpos = ndots ? (int64_t)red[3] - 1 : E;
            if (nmark <= 1 && red[4] == 0 && ndots <= 1 && dotpos <= E && (E - s0 - (int64_t)ndots) >= 1 &&
                (nmark ? (nsigns == 0 || esg) && x0 < e : nsigns == 0))
                m |= OK_FLOAT;
            atomicAnd(mask + f.col, m);
        }
        __syncthreads();  // red is reused by the next field
    }
}

__global__ void infer_finish(const uint32_t* mask, const int64_t* nonempty, int32_t ncols, int32_t* types)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncols) return;
    const uint32_t m = nonempty[c] ? mask[c] : 0u;
    types[c] = (m & OK_INT) ? PP_INT64 : (m & OK_FLOAT) ? PP_FLOAT64 : (m & OK_DATE) ? PP_DATE_DAYS
             : (m & OK_TS) ? PP_TIMESTAMP_S : PP_STRING;
}

}  // namespace

extern "C" size_t pp_infer_types_workspace_size(int32_t ncols)
{
    return ncols < 0 ? 0 : mask_bytes(ncols) + 16 + (size_t)kInferLongCap * sizeof(LongSpan);
}

extern "C" pp_status_t pp_infer_types(const uint8_t* d_in, int64_t n, const pp_outputs_t* parsed, int32_t ncols,
                                      int32_t* d_types, int64_t* d_nonempty, void* d_ws, size_t ws_bytes,
                                      void* stream)
{
    if (n < 0 || (n > 0 && !d_in) || !parsed || !parsed->d_result || !d_types || !d_nonempty || !d_ws ||
        !pp::ws_aligned(d_ws) || ncols < 0 || ncols > PP_MAX_COLUMNS || parsed->cap_records < 0)
        return PP_ERR_ARG;
    if (ws_bytes < pp_infer_types_workspace_size(ncols)) return PP_ERR_WORKSPACE;
    if (ncols == 0) return PP_OK;
    ColSpans cs;
    memset(&cs, 0, sizeof cs);
    if (parsed->cap_records > 0) {
        if (!parsed->d_values || !parsed->d_valid || !parsed->d_str_end) return PP_ERR_ARG;
        for (int c = 0; c < ncols; ++c) {
            // every column a string span column of the parse
            if (!parsed->d_values[c] || !parsed->d_valid[c] || !parsed->d_str_end[c]) return PP_ERR_ARG;
            cs.begin[c] = (const int64_t*)parsed->d_values[c];
            cs.end[c] = parsed->d_str_end[c];
            cs.valid[c] = parsed->d_valid[c];
        }
    }
    hipStream_t s = (hipStream_t)stream;
    uint32_t* mask = (uint32_t*)d_ws;
    uint32_t* qcount = (uint32_t*)((char*)d_ws + mask_bytes(ncols));
    LongSpan* queue = (LongSpan*)((char*)d_ws + mask_bytes(ncols) + 16);
    hipLaunchKernelGGL(infer_init, dim3(1), dim3(64), 0, s, mask, d_nonempty, ncols, qcount);
    if (parsed->cap_records > 0) {
        const int64_t cap = parsed->cap_records;
        const unsigned bx = (unsigned)std::min<int64_t>(512, std::max<int64_t>(1, (cap + 255) / 256));
        hipLaunchKernelGGL(infer_fields, dim3(bx, (unsigned)ncols), dim3(256), 0, s, d_in, cs, cap, parsed->d_result,
                           mask, d_nonempty, qcount, queue);
        // long fields: few, often none (then every workgroup exits at once)
        if (n >= kInferLong)
            hipLaunchKernelGGL(infer_long, dim3(64), dim3(256), 0, s, d_in, qcount, queue, mask);
    }
    hipLaunchKernelGGL(infer_finish, dim3(1), dim3(64), 0, s, mask, d_nonempty, ncols, d_types);
    return hipGetLastError() == hipSuccess ? PP_OK : PP_ERR_HIP;
}
