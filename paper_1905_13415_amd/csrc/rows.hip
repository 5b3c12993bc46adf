// Skipping rows (Sec. 4.3): rows are line-feed separated lines of the raw
// input (a quoted record may span several), so they are dropped before the
// parse by a parallel stream compaction of the input bytes:
//   1. line feeds per 4 KiB block, scanned: the row of each block's first byte;
//   2. per block, each thread's 16 bytes get their rows (a workgroup scan of
//      the line-feed counts) and keep flags (binary search of the row in the
//      sorted skip ranges); kept bytes per block, scanned: the output base;
//   3. the same flags again, and every kept byte written to its place.
// Skipping records (Sec. 4.3, after the parse, where records are known):
// the typed values of the records in the given ranges are cleared to the
// column defaults (value 0, valid 0, empty span), so they read as ignored;
// their fields stay in the offsets.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "dfa_check.h"
#include "parparaw.h"
#include "scan.h"

namespace {

constexpr int kRowBlock = 4096;  // bytes per workgroup: 256 threads x 16
constexpr int kMaxRanges = PP_MAX_SKIP_RANGES;

struct Ranges {
    int64_t first[kMaxRanges], last[kMaxRanges];
    int32_t count;
};

__device__ inline bool skipped(const Ranges& rg, int64_t row)
{
    // the last range whose first <= row (ranges sorted, disjoint)
    int lo = 0, hi = rg.count - 1, k = -1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        if (rg.first[mid] <= row) { k = mid; lo = mid + 1; }
        else hi = mid - 1;
    }
    return k >= 0 && row < rg.last[k];
}

// exclusive workgroup scan of one value per thread (256 threads)
__device__ inline int64_t block_exclusive(int64_t v, int64_t* sh, int64_t* total)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        const int64_t t = threadIdx.x >= (unsigned)d ? sh[threadIdx.x - d] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    const int64_t incl = sh[threadIdx.x];
    *total = sh[255];
    __syncthreads();
    return incl - v;
}

// this thread's 16 bytes (zero past n), as bytes in registers
__device__ inline int load16(const uint8_t* in, int64_t n, int64_t at, uint8_t* b)
{
    int m = 0;
    for (int k = 0; k < 16; ++k) {
        const int64_t i = at + k;
        b[k] = i < n ? in[i] : 0;
        m += i < n;
    }
    return m;
}

__global__ __launch_bounds__(256) void lf_counts(const uint8_t* in, int64_t n, int64_t* cnt)
{
    __shared__ int64_t sh[4];
    const int64_t at = (int64_t)blockIdx.x * kRowBlock + (int64_t)threadIdx.x * 16;
    uint8_t b[16];
    const int m = load16(in, n, at, b);
    int64_t c = 0;
    for (int k = 0; k < m; ++k) c += b[k] == '\n';
    c = pp::block_reduce(c, sh);
    if (threadIdx.x == 0) cnt[blockIdx.x] = c;
}

// WRITE = false: kept bytes per block into cnt; WRITE = true: the kept bytes
// to out at the scanned block bases.
template <bool WRITE>
__global__ __launch_bounds__(256) void keep_pass(const uint8_t* in, int64_t n, Ranges rg, const int64_t* row_base,
                                                 int64_t* cnt, const int64_t* out_base, uint8_t* out)
{
    __shared__ int64_t sh[256];
    const int64_t at = (int64_t)blockIdx.x * kRowBlock + (int64_t)threadIdx.x * 16;
    uint8_t b[16];
    const int m = load16(in, n, at, b);
    int64_t lf = 0;
    for (int k = 0; k < m; ++k) lf += b[k] == '\n';
    int64_t tot;
    int64_t row = row_base[blockIdx.x] + block_exclusive(lf, sh, &tot);
    uint32_t keepmask = 0;
    bool skip = skipped(rg, row);
    for (int k = 0; k < m; ++k) {
        if (!skip) keepmask |= 1u << k;
        if (b[k] == '\n') skip = skipped(rg, ++row);
    }
    const int64_t kept = __popc(keepmask);
    int64_t ktot;
    const int64_t before = block_exclusive(kept, sh, &ktot);
    if (!WRITE) {
        if (threadIdx.x == 0) cnt[blockIdx.x] = ktot;
        return;
    }
    int64_t o = out_base[blockIdx.x] + before;
    for (int k = 0; k < m; ++k)
        if ((keepmask >> k) & 1u) out[o++] = b[k];
}

__global__ void store_len(const int64_t* base, int64_t nblocks, int64_t* out_len)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *out_len = base[nblocks];
}

}  // namespace

struct ColOut {
    void* values[PP_MAX_COLUMNS];
    uint8_t* valid[PP_MAX_COLUMNS];
    int64_t* str_end[PP_MAX_COLUMNS];
};

// grid-stride over records r < min(R, cap) in a skipped range, then columns
__global__ void clear_records(ColOut co, int32_t ncols, int64_t cap, const pp_result_t* res, Ranges rg)
{
    const int64_t R0 = res->num_records;
    const int64_t R = R0 < cap ? R0 : cap;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R; r += stride) {
        if (!skipped(rg, r)) continue;
        for (int c = 0; c < ncols; ++c) {
            if (!co.values[c]) continue;
            ((int64_t*)co.values[c])[r] = 0;  // 0 and 0.0 share the bit pattern
            co.valid[c][r] = 0;
            if (co.str_end[c]) co.str_end[c][r] = 0;
        }
    }
}

extern "C" size_t pp_skip_rows_workspace_size(int64_t n)
{
    if (n < 0) return 0;
    const int64_t nb = (n + kRowBlock - 1) / kRowBlock;
    return (size_t)(2 * (nb + 1) + (nb / pp::kScanItems + 2)) * sizeof(int64_t);
}

extern "C" pp_status_t pp_skip_rows(const uint8_t* d_in, int64_t n, const int64_t* ranges, int32_t nranges,
                                    uint8_t* d_out, int64_t* d_out_len, void* d_ws, size_t ws_bytes, void* stream)
{
    if (n < 0 || (n > 0 && (!d_in || !d_out)) || !d_out_len || !d_ws || !pp::ws_aligned(d_ws) || nranges < 0 ||
        nranges > kMaxRanges || (nranges > 0 && !ranges))
        return PP_ERR_ARG;
    Ranges rg;
    rg.count = nranges;
    for (int k = 0; k < nranges; ++k) {
        rg.first[k] = ranges[2 * k];
        rg.last[k] = ranges[2 * k + 1];
        if (rg.first[k] < 0 || rg.last[k] <= rg.first[k] || (k && rg.first[k] < rg.last[k - 1]))
            return PP_ERR_ARG;  // each range non-empty, sorted and disjoint
    }
    if (ws_bytes < pp_skip_rows_workspace_size(n)) return PP_ERR_WORKSPACE;
    const int64_t nb = (n + kRowBlock - 1) / kRowBlock;
    if (nb > 0x7fffffff) return PP_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    int64_t* rows = (int64_t*)d_ws;       // [nb + 1]
    int64_t* kept = rows + (nb + 1);      // [nb + 1]
    int64_t* partial = kept + (nb + 1);
    if (nb > 0) {
        hipLaunchKernelGGL(lf_counts, dim3((unsigned)nb), dim3(256), 0, s, d_in, n, rows);
        pp::scan_i64(rows, rows, nb, nullptr, partial, s);
        hipLaunchKernelGGL(keep_pass<false>, dim3((unsigned)nb), dim3(256), 0, s, d_in, n, rg, rows, kept, nullptr,
                           nullptr);
        pp::scan_i64(kept, kept, nb, nullptr, partial, s);
        hipLaunchKernelGGL(keep_pass<true>, dim3((unsigned)nb), dim3(256), 0, s, d_in, n, rg, rows, nullptr, kept,
                           d_out);
    } else {
        pp::scan_i64(kept, kept, 0, nullptr, partial, s);  // kept[0] = 0
    }
    hipLaunchKernelGGL(store_len, dim3(1), dim3(64), 0, s, kept, nb, d_out_len);
    return hipGetLastError() == hipSuccess ? PP_OK : PP_ERR_HIP;
}

extern "C" pp_status_t pp_skip_records(const pp_outputs_t* parsed, int32_t ncols, const int32_t* types,
                                       const int64_t* ranges, int32_t nranges, void* stream)
{
    if (!parsed || !parsed->d_result || ncols < 0 || ncols > PP_MAX_COLUMNS || (ncols > 0 && !types) ||
        nranges < 0 || nranges > kMaxRanges || (nranges > 0 && !ranges) || parsed->cap_records < 0)
        return PP_ERR_ARG;
    Ranges rg;
    rg.count = nranges;
    for (int k = 0; k < nranges; ++k) {
        rg.first[k] = ranges[2 * k];
        rg.last[k] = ranges[2 * k + 1];
        if (rg.first[k] < 0 || rg.last[k] <= rg.first[k] || (k && rg.first[k] < rg.last[k - 1])) return PP_ERR_ARG;
    }
    ColOut co;
    for (int c = 0; c < PP_MAX_COLUMNS; ++c) {
        co.values[c] = nullptr;
        co.valid[c] = nullptr;
        co.str_end[c] = nullptr;
    }
    const int64_t cap = parsed->cap_records;
    for (int c = 0; c < ncols && cap > 0; ++c) {
        if (types[c] < PP_INT64 || types[c] > PP_SKIP) return PP_ERR_SCHEMA;
        if (types[c] == PP_SKIP) continue;
        if (!parsed->d_values || !parsed->d_valid || !parsed->d_values[c] || !parsed->d_valid[c]) return PP_ERR_ARG;
        if (types[c] == PP_STRING && (!parsed->d_str_end || !parsed->d_str_end[c])) return PP_ERR_ARG;
        co.values[c] = parsed->d_values[c];
        co.valid[c] = parsed->d_valid[c];
        co.str_end[c] = types[c] == PP_STRING ? parsed->d_str_end[c] : nullptr;
    }
    if (cap == 0 || nranges == 0 || ncols == 0) return PP_OK;
    const unsigned grid = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, (cap + 255) / 256));
    hipLaunchKernelGGL(clear_records, dim3(grid), dim3(256), 0, (hipStream_t)stream, co, ncols, cap, parsed->d_result,
                       rg);
    return hipGetLastError() == hipSuccess ? PP_OK : PP_ERR_HIP;
}
