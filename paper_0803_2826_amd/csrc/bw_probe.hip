// Bandwidth reference for the benchmark (not part of the LB library): a
// plain streaming copy, 16 bytes per thread, one vector per thread, with
// non-temporal stores.  Its rate over a buffer of the size the step kernel
// streams is the practical HBM ceiling that kernel is compared with.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__global__ void k_copy16(const float4 *__restrict__ src, float4 *__restrict__ dst, size_t n16)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n16) return;
    const float4 v = src[i];
    __builtin_nontemporal_store(v.x, &dst[i].x);
    __builtin_nontemporal_store(v.y, &dst[i].y);
    __builtin_nontemporal_store(v.z, &dst[i].z);
    __builtin_nontemporal_store(v.w, &dst[i].w);
}

}  // namespace

extern "C" {

// Copy nbytes (a multiple of 16; both pointers 16-byte aligned device
// memory) from src to dst on `stream` with `block` threads per block
// (64..1024).  Returns 0, or -1 for bad arguments, or the HIP error code of
// the launch.
int bw_copy(const void *src, void *dst, uint64_t nbytes, int32_t block, void *stream)
{
    if (!src || !dst || (nbytes & 15u) || block < 64 || block > 1024 || (block & 63)) return -1;
    if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15u) return -1;
    const size_t n16 = nbytes / 16;
    if (n16 == 0) return 0;
    const size_t grid = (n16 + block - 1) / block;
    if (grid > 0x7fffffffu) return -1;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)grid), dim3(block), 0, static_cast<hipStream_t>(stream),
                       static_cast<const float4 *>(src), static_cast<float4 *>(dst), n16);
    return (int)hipGetLastError();
}

}  // extern "C"
