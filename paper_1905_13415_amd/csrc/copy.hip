// Streaming device copy: the practical HBM ceiling that the parse kernels
// are measured against (the fastest a kernel can read n bytes and write n
// bytes on this device), and the device-to-device copy that the streaming
// form uses to move a partition's unfinished record to the front of the
// next one.
//
// Every lane moves 16-byte vectors with nontemporal loads and stores (the
// data is touched once); consecutive lanes take consecutive vectors, so a
// wavefront reads and writes 1 KiB contiguously per step. The grid is sized
// to a few workgroups per CU and strides over the buffer.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "parparaw.h"

namespace pp {

typedef unsigned int cp_u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void copy_stream16(const cp_u32x4* __restrict__ src, cp_u32x4* __restrict__ dst,
                                                     size_t n16)
{
    constexpr int U = 4;  // vectors in flight per lane per step
    const size_t lanes = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (U - 1) * lanes < n16; i += U * lanes) {
        cp_u32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(src + i + u * lanes);
#pragma unroll
        for (int u = 0; u < U; ++u) __builtin_nontemporal_store(v[u], dst + i + u * lanes);
    }
    for (; i < n16; i += lanes) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

__global__ void copy_bytes(const uint8_t* __restrict__ src, uint8_t* __restrict__ dst, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace pp

using namespace pp;

extern "C" pp_status_t pp_copy(void* d_dst, const void* d_src, size_t n, void* stream)
{
    if (n == 0) return PP_OK;
    if (!d_dst || !d_src) return PP_ERR_ARG;
    const uintptr_t s = (uintptr_t)d_src, d = (uintptr_t)d_dst;
    if ((s < d && s + n > d) || (d < s && d + n > s)) return PP_ERR_ARG;  // overlapping ranges
    hipStream_t st = (hipStream_t)stream;
    size_t head = 0;
    if ((s & 15) == (d & 15)) head = (16 - (s & 15)) & 15;  // align both to 16 bytes
    else head = n;                                          // no common alignment: bytes only
    if (head > n) head = n;
    const size_t n16 = (n - head) / 16, tail = n - head - n16 * 16;
    if (head) hipLaunchKernelGGL(copy_bytes, dim3(1), dim3(64), 0, st, (const uint8_t*)d_src, (uint8_t*)d_dst, head);
    if (n16) {
        // about eight workgroups of 256 lanes per CU (256 CUs), fewer for small copies
        const size_t want = (n16 + 4 * 256 - 1) / (4 * 256);
        const unsigned grid = (unsigned)(want < 2048 ? (want ? want : 1) : 2048);
        hipLaunchKernelGGL(copy_stream16, dim3(grid), dim3(256), 0, st, (const cp_u32x4*)((const uint8_t*)d_src + head),
                           (cp_u32x4*)((uint8_t*)d_dst + head), n16);
    }
    if (tail) {
        const size_t off = head + n16 * 16;
        hipLaunchKernelGGL(copy_bytes, dim3(1), dim3(64), 0, st, (const uint8_t*)d_src + off, (uint8_t*)d_dst + off,
                           tail);
    }
    return hipGetLastError() == hipSuccess ? PP_OK : PP_ERR_HIP;
}
