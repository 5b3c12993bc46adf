// Exclusive scan of int64 values on the device (three launches: block
// sums, one workgroup over the block sums, block scans plus their prefix),
// shared by the materialisation and the row compaction.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "parparaw.h"

namespace pp {

constexpr int kScanItems = 2048;  // elements per scan block (256 threads x 8)

// ---- exclusive scan of int64 values -----------------------------------------
// out[i] = sum of in[j] for j < i, i <= N; out[N] = total. N is the parse's
// record count capped at nmax when res is set, else nmax. in and out may
// alias (a block reads its elements before it writes them).

static __device__ inline int64_t count_of(int64_t nmax, const pp_result_t* res)
{
    if (res) {
        const int64_t r = res->num_records;
        return r < nmax ? r : nmax;
    }
    return nmax;
}

static __device__ inline int64_t block_reduce(int64_t v, int64_t* sh)
{
    for (int d = 32; d; d >>= 1) v += __shfl_xor(v, d);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) sh[w] = v;
    __syncthreads();
    int64_t t = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sh[k];
    __syncthreads();
    return t;
}

static __global__ __launch_bounds__(256) void scan_partials(const int64_t* in, int64_t nmax, const pp_result_t* res,
                                                     int64_t* partial)
{
    __shared__ int64_t sh[4];
    const int64_t N = count_of(nmax, res);
    const int64_t base = (int64_t)blockIdx.x * kScanItems;
    int64_t s = 0;
    for (int k = 0; k < kScanItems / 256; ++k) {
        const int64_t i = base + k * 256 + threadIdx.x;
        if (i < N) s += in[i];
    }
    s = block_reduce(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// one workgroup: exclusive scan of the partials (few thousand at most)
static __global__ __launch_bounds__(1024) void scan_top(int64_t* partial, int64_t nparts)
{
    __shared__ int64_t sh[1024];
    int64_t carry = 0;
    for (int64_t base = 0; base < nparts; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const int64_t v = i < nparts ? partial[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {  // Hillis-Steele inclusive scan
            const int64_t t = threadIdx.x >= (unsigned)d ? sh[threadIdx.x - d] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nparts) partial[i] = carry + sh[threadIdx.x] - v;
        carry += sh[1023];
        __syncthreads();
    }
}

static __global__ __launch_bounds__(256) void scan_apply(const int64_t* in, int64_t* out, int64_t nmax,
                                                  const pp_result_t* res, const int64_t* partial)
{
    __shared__ int64_t sh[256];
    const int64_t N = count_of(nmax, res);
    const int64_t base = (int64_t)blockIdx.x * kScanItems;
    if (base > N) return;
    // each thread owns 8 consecutive elements
    const int64_t my = base + (int64_t)threadIdx.x * (kScanItems / 256);
    int64_t v[kScanItems / 256];
    int64_t sum = 0;
    for (int k = 0; k < kScanItems / 256; ++k) {
        v[k] = my + k < N ? in[my + k] : 0;
        sum += v[k];
    }
    sh[threadIdx.x] = sum;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        const int64_t t = threadIdx.x >= (unsigned)d ? sh[threadIdx.x - d] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    int64_t run = partial[blockIdx.x] + sh[threadIdx.x] - sum;
    for (int k = 0; k < kScanItems / 256; ++k) {
        const int64_t i = my + k;
        if (i <= N) out[i] = run;  // out[N]: the total
        run += v[k];
    }
}

// Exclusive scan of in[0, N) into out[0, N], N <= nmax (the parse's record
// count when res is set); out[N] = the total. partial: nmax / kScanItems + 2
// int64 of scratch.
static inline void scan_i64(const int64_t* in, int64_t* out, int64_t nmax, const pp_result_t* res, int64_t* partial,
                            hipStream_t s)
{
    const int64_t nb = nmax / kScanItems + 1;  // covers index nmax (the total)
    hipLaunchKernelGGL(scan_partials, dim3((unsigned)nb), dim3(256), 0, s, in, nmax, res, partial);
    hipLaunchKernelGGL(scan_top, dim3(1), dim3(1024), 0, s, partial, nb);
    hipLaunchKernelGGL(scan_apply, dim3((unsigned)nb), dim3(256), 0, s, in, out, nmax, res, partial);
}

}  // namespace pp
