// Type inference (Sec. 4.3): after a parse whose columns are string spans,
// every non-empty field is checked against each type's grammar -- INT64
// (converts without overflow), FLOAT64 (the float grammar), DATE_DAYS and
// TIMESTAMP_S (valid calendar values) -- and a column keeps the types all of
// its fields admit (an AND over the fields, reduced per wavefront and
// workgroup, then one atomic per workgroup). The inferred type is the first
// kept type in the order INT64, FLOAT64, DATE_DAYS, TIMESTAMP_S, else STRING
// (also for a column without non-empty fields). A field's checks stop at its
// first byte that no candidate type accepts, so long text costs little.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>

#include "convert.h"
#include "dfa_check.h"
#include "parparaw.h"

namespace {

enum : uint32_t { OK_INT = 1, OK_FLOAT = 2, OK_DATE = 4, OK_TS = 8, OK_ALL = 15 };

struct ColSpans {
    const int64_t* begin[PP_MAX_COLUMNS];
    const int64_t* end[PP_MAX_COLUMNS];
    const uint8_t* valid[PP_MAX_COLUMNS];
};

struct GlobalBytes {
    const uint8_t* p;
    __device__ uint32_t operator()(int64_t i) const { return p[i]; }
};

__global__ void infer_init(uint32_t* mask, int64_t* nonempty, int32_t ncols)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncols) {
        mask[c] = OK_ALL;
        nonempty[c] = 0;
    }
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
                                                    const pp_result_t* res, uint32_t* mask, int64_t* nonempty)
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
        acc &= field_admits(src, b, e);
        ++cnt;
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
    return ncols < 0 ? 0 : (size_t)std::max(ncols, 1) * sizeof(uint32_t);
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
    hipLaunchKernelGGL(infer_init, dim3(1), dim3(64), 0, s, mask, d_nonempty, ncols);
    if (parsed->cap_records > 0) {
        const int64_t cap = parsed->cap_records;
        const unsigned bx = (unsigned)std::min<int64_t>(512, std::max<int64_t>(1, (cap + 255) / 256));
        hipLaunchKernelGGL(infer_fields, dim3(bx, (unsigned)ncols), dim3(256), 0, s, d_in, cs, cap, parsed->d_result,
                           mask, d_nonempty);
    }
    hipLaunchKernelGGL(infer_finish, dim3(1), dim3(64), 0, s, mask, d_nonempty, ncols, d_types);
    return hipGetLastError() == hipSuccess ? PP_OK : PP_ERR_HIP;
}
