// Bandwidth references for the benchmark (not part of the LB library):
//   bw_copy    a plain streaming copy, 16 bytes per thread, one vector per
//              thread, non-temporal stores: the practical HBM ceiling;
//   bw_pull19  the memory pattern of the LB step alone (19 planes, each
//              pulled from the neighbour r - c_i, 4 bytes per lane): the
//              ceiling of that access pattern without arithmetic.
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

// The memory pattern of the LB step without its arithmetic, in the step's
// z-major layout ([z][i][y][x], 19 values per site, N = 2^(3 lg) sites):
// each site pulls population i from its periodic neighbour r - c_i (D3Q19
// velocity set) and stores it non-temporally at r.
__constant__ int kPX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__constant__ int kPY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__constant__ int kPZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

__global__ void __launch_bounds__(1024) k_pull19(const float *__restrict__ src, float *__restrict__ dst, uint32_t lg)
{
    const uint32_t m = (1u << lg) - 1u;
    const size_t layer = (size_t)1 << (2 * lg);
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t x = s & m, y = (s >> lg) & m, z = s >> (2 * lg);
    float v[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const uint32_t xs = (x - kPX[i]) & m, ys = (y - kPY[i]) & m, zs = (z - kPZ[i]) & m;
        v[i] = src[((size_t)zs * 19 + i) * layer + (xs + (ys << lg))];
    }
#pragma unroll
    for (int i = 0; i < 19; ++i)
        __builtin_nontemporal_store(v[i], &dst[((size_t)z * 19 + i) * layer + (x + (y << lg))]);
}

}  // namespace

extern "C" {

// The pull pattern of one LB step (z-major layout) over a cube of edge 2^lg (4 <= lg <= 10):
// src and dst are device arrays of 19 * 2^(3 lg) floats; `block` threads per
// block (64..1024, dividing 2^(3 lg)).  Returns 0, -1 for bad arguments, or
// the HIP error code of the launch.
int bw_pull19(const float *src, float *dst, int32_t lg, int32_t block, void *stream)
{
    if (!src || !dst || lg < 4 || lg > 10 || block < 64 || block > 1024 || (block & 63)) return -1;
    const size_t N = (size_t)1 << (3 * lg);
    if (N % (size_t)block) return -1;
    hipLaunchKernelGGL(k_pull19, dim3((unsigned)(N / block)), dim3(block), 0, static_cast<hipStream_t>(stream), src, dst,
                       (uint32_t)lg);
    return (int)hipGetLastError();
}


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
