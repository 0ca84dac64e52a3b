// Bandwidth references for the benchmark (not part of the LB library): the
// memory patterns of the LB step and of plain streaming kernels, without the
// collision's arithmetic, to show what an HBM-bound kernel of this shape can
// reach on the device.
//   bw_copy      plain streaming copy, 16 bytes per thread, non-temporal
//                stores (the reference the benchmark reports);
//   bw_copy_v    copy variants: V vectors of 16 B per thread (consecutive
//                block-wide chunks), optional non-temporal loads, optional
//                persistent grid (grid-stride loop over a fixed block count);
//   bw_read      read-only stream (16 B per thread), bw_write write-only
//                stream, bw_inplace read-modify-write of the same 16 B;
//   bw_pull      the step's access pattern in its z-major layout with P
//                planes per layer: populations 0..18 pulled from the D3Q19
//                neighbours r - c_i, plane 19 (P = 20, the rest
//                population's rounding residual) read at r, all stored at r
//                in a second buffer;
//   bw_aa        the in-place alternative ("AA" pattern, one buffer):
//                parity 0 reads the 19 slots of its own site and writes them
//                back swapped to the opposite slots; parity 1 reads slot
//                opp(i) at r - c_i and writes slot i at r + c_i (each site
//                reads and writes the same 19 addresses, so sites never
//                collide); plane 19 is read and written at r.
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

__device__ __forceinline__ float4 ld16(const float4 *p, bool nt)
{
    if (nt) {
        float4 v;
        v.x = __builtin_nontemporal_load(&p->x);
        v.y = __builtin_nontemporal_load(&p->y);
        v.z = __builtin_nontemporal_load(&p->z);
        v.w = __builtin_nontemporal_load(&p->w);
        return v;
    }
    return *p;
}

__device__ __forceinline__ void st16(float4 *p, float4 v, bool nt)
{
    if (nt) {
        __builtin_nontemporal_store(v.x, &p->x);
        __builtin_nontemporal_store(v.y, &p->y);
        __builtin_nontemporal_store(v.z, &p->z);
        __builtin_nontemporal_store(v.w, &p->w);
    } else {
        *p = v;
    }
}

// V vectors per thread: thread t of block b copies elements
// b * V * blockDim + v * blockDim + t, v = 0..V-1 (every access of a wave is
// 1 KiB contiguous); with a persistent grid the block index strides by
// gridDim.  All loads of a thread are issued before its stores.
template <int V>
__global__ void __launch_bounds__(1024) k_copy_v(const float4 *__restrict__ src, float4 *__restrict__ dst, size_t n16,
                                                 int nt_load, int nt_store)
{
    const size_t chunk = (size_t)V * blockDim.x;
    for (size_t base = (size_t)blockIdx.x * chunk; base < n16; base += (size_t)gridDim.x * chunk) {
        float4 v[V];
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const size_t i = base + (size_t)k * blockDim.x + threadIdx.x;
            if (i < n16) v[k] = ld16(src + i, nt_load != 0);
        }
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const size_t i = base + (size_t)k * blockDim.x + threadIdx.x;
            if (i < n16) st16(dst + i, v[k], nt_store != 0);
        }
    }
}

// Read-only stream: the loaded values feed a store that never happens
// (the buffer holds finite values), so the loads cannot be dropped.
__global__ void __launch_bounds__(1024) k_read16(const float4 *__restrict__ src, size_t n16, float *__restrict__ sink)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n16) return;
    const float4 v = src[i];
    const float s = v.x + v.y + v.z + v.w;
    if (s == __builtin_inff()) sink[0] = s;
}

__global__ void __launch_bounds__(1024) k_write16(float4 *__restrict__ dst, size_t n16)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n16) return;
    st16(dst + i, make_float4(1.f, 2.f, 3.f, 4.f), true);
}

// Read-modify-write of the same 16 bytes (the value changes, so the store
// is not a no-op the compiler could drop).
__global__ void __launch_bounds__(1024) k_inplace16(float4 *__restrict__ buf, size_t n16)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n16) return;
    float4 v = buf[i];
    v.x += 1.f;
    st16(buf + i, v, true);
}

__constant__ int kPX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__constant__ int kPY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__constant__ int kPZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

__device__ __forceinline__ int opp_dir(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// The step's memory pattern (z-major, P planes per layer, cube of edge 2^lg).
template <int P>
__global__ void __launch_bounds__(1024) k_pull(const float *__restrict__ src, float *__restrict__ dst, uint32_t lg)
{
    const uint32_t m = (1u << lg) - 1u;
    const size_t layer = (size_t)1 << (2 * lg);
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t x = s & m, y = (s >> lg) & m, z = s >> (2 * lg);
    float v[P];
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const uint32_t xs = (x - kPX[i]) & m, ys = (y - kPY[i]) & m, zs = (z - kPZ[i]) & m;
        v[i] = src[((size_t)zs * P + i) * layer + (xs + (ys << lg))];
    }
    if (P == 20) v[P - 1] = src[((size_t)z * P + 19) * layer + (x + (y << lg))];
#pragma unroll
    for (int i = 0; i < P; ++i)
        __builtin_nontemporal_store(v[i], &dst[((size_t)z * P + i) * layer + (x + (y << lg))]);
}

// In-place AA pattern, P = 20 planes (see the header).
template <int PAR>
__global__ void __launch_bounds__(1024) k_aa(float *__restrict__ buf, uint32_t lg)
{
    constexpr int P = 20;
    const uint32_t m = (1u << lg) - 1u;
    const size_t layer = (size_t)1 << (2 * lg);
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t x = s & m, y = (s >> lg) & m, z = s >> (2 * lg);
    float v[P];
    size_t at[P];
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        if (PAR == 0) {
            at[i] = ((size_t)z * P + i) * layer + (x + (y << lg));
        } else {
            const int j = opp_dir(i);  // slot opp(i) of r - c_i = slot j of r + c_j
            const uint32_t xs = (x + kPX[j]) & m, ys = (y + kPY[j]) & m, zs = (z + kPZ[j]) & m;
            at[i] = ((size_t)zs * P + j) * layer + (xs + (ys << lg));
        }
        v[i] = buf[at[i]];
    }
    at[19] = ((size_t)z * P + 19) * layer + (x + (y << lg));
    v[19] = buf[at[19]];
    // parity 0 writes value i to the slot of opp(i); parity 1 writes value i
    // to slot i of r + c_i, which is where it read opp(i)'s value: in both
    // cases site r writes exactly the addresses it read
#pragma unroll
    for (int i = 0; i < 19; ++i) __builtin_nontemporal_store(v[opp_dir(i)] + 1.f, &buf[at[i]]);
    __builtin_nontemporal_store(v[19], &buf[at[19]]);
}

bool bad_block(int32_t block) { return block < 64 || block > 1024 || (block & 63); }

}  // namespace

extern "C" {

// The pull pattern of one LB step (z-major layout, 19 planes) over a cube of
// edge 2^lg (4 <= lg <= 10): src and dst are device arrays of 19 * 2^(3 lg)
// floats; `block` threads per block (64..1024, dividing 2^(3 lg)).  Returns
// 0, -1 for bad arguments, or the HIP error code of the launch.
int bw_pull19(const float *src, float *dst, int32_t lg, int32_t block, void *stream)
{
    if (!src || !dst || lg < 4 || lg > 10 || bad_block(block)) return -1;
    const size_t N = (size_t)1 << (3 * lg);
    if (N % (size_t)block) return -1;
    hipLaunchKernelGGL(k_pull<19>, dim3((unsigned)(N / block)), dim3(block), 0, static_cast<hipStream_t>(stream), src,
                       dst, (uint32_t)lg);
    return (int)hipGetLastError();
}

// As bw_pull19 with P = 20 planes per layer (src, dst: 20 * 2^(3 lg) floats).
int bw_pull20(const float *src, float *dst, int32_t lg, int32_t block, void *stream)
{
    if (!src || !dst || lg < 4 || lg > 10 || bad_block(block)) return -1;
    const size_t N = (size_t)1 << (3 * lg);
    if (N % (size_t)block) return -1;
    hipLaunchKernelGGL(k_pull<20>, dim3((unsigned)(N / block)), dim3(block), 0, static_cast<hipStream_t>(stream), src,
                       dst, (uint32_t)lg);
    return (int)hipGetLastError();
}

// One in-place AA step of parity 0 or 1 over buf (20 * 2^(3 lg) floats).
int bw_aa(float *buf, int32_t lg, int32_t parity, int32_t block, void *stream)
{
    if (!buf || lg < 4 || lg > 10 || bad_block(block) || (parity != 0 && parity != 1)) return -1;
    const size_t N = (size_t)1 << (3 * lg);
    if (N % (size_t)block) return -1;
    if (parity == 0)
        hipLaunchKernelGGL(k_aa<0>, dim3((unsigned)(N / block)), dim3(block), 0, static_cast<hipStream_t>(stream), buf,
                           (uint32_t)lg);
    else
        hipLaunchKernelGGL(k_aa<1>, dim3((unsigned)(N / block)), dim3(block), 0, static_cast<hipStream_t>(stream), buf,
                           (uint32_t)lg);
    return (int)hipGetLastError();
}

// Copy nbytes (a multiple of 16; both pointers 16-byte aligned device
// memory) from src to dst on `stream` with `block` threads per block
// (64..1024).  Returns 0, or -1 for bad arguments, or the HIP error code of
// the launch.
int bw_copy(const void *src, void *dst, uint64_t nbytes, int32_t block, void *stream)
{
    if (!src || !dst || (nbytes & 15u) || bad_block(block)) return -1;
    if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15u) return -1;
    const size_t n16 = nbytes / 16;
    if (n16 == 0) return 0;
    const size_t grid = (n16 + block - 1) / block;
    if (grid > 0x7fffffffu) return -1;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)grid), dim3(block), 0, static_cast<hipStream_t>(stream),
                       static_cast<const float4 *>(src), static_cast<float4 *>(dst), n16);
    return (int)hipGetLastError();
}

// Copy variant: vec = 1, 2, 4 or 8 vectors of 16 B per thread; nt_load /
// nt_store: non-temporal loads / stores; grid = 0: one chunk per block,
// else that many blocks looping over the chunks.  Same pointer rules as
// bw_copy.
int bw_copy_v(const void *src, void *dst, uint64_t nbytes, int32_t block, int32_t vec, int32_t nt_load,
              int32_t nt_store, int32_t grid, void *stream)
{
    if (!src || !dst || (nbytes & 15u) || bad_block(block) || grid < 0) return -1;
    if (vec != 1 && vec != 2 && vec != 4 && vec != 8) return -1;
    if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15u) return -1;
    const size_t n16 = nbytes / 16;
    if (n16 == 0) return 0;
    const size_t chunks = (n16 + (size_t)vec * block - 1) / ((size_t)vec * block);
    const size_t g = grid > 0 ? (size_t)grid : chunks;
    if (g > 0x7fffffffu) return -1;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const float4 *a = static_cast<const float4 *>(src);
    float4 *b = static_cast<float4 *>(dst);
    switch (vec) {
    case 1: hipLaunchKernelGGL(k_copy_v<1>, dim3((unsigned)g), dim3(block), 0, s, a, b, n16, nt_load, nt_store); break;
    case 2: hipLaunchKernelGGL(k_copy_v<2>, dim3((unsigned)g), dim3(block), 0, s, a, b, n16, nt_load, nt_store); break;
    case 4: hipLaunchKernelGGL(k_copy_v<4>, dim3((unsigned)g), dim3(block), 0, s, a, b, n16, nt_load, nt_store); break;
    default: hipLaunchKernelGGL(k_copy_v<8>, dim3((unsigned)g), dim3(block), 0, s, a, b, n16, nt_load, nt_store); break;
    }
    return (int)hipGetLastError();
}

// Read-only (sink: one float of device memory, never written for finite
// data), write-only and in-place streams over nbytes (multiple of 16,
// 16-byte aligned), 16 B per thread.
int bw_read(const void *src, uint64_t nbytes, int32_t block, float *sink, void *stream)
{
    if (!src || !sink || (nbytes & 15u) || bad_block(block) || (reinterpret_cast<uintptr_t>(src) & 15u)) return -1;
    const size_t n16 = nbytes / 16, grid = (n16 + block - 1) / block;
    if (n16 == 0) return 0;
    if (grid > 0x7fffffffu) return -1;
    hipLaunchKernelGGL(k_read16, dim3((unsigned)grid), dim3(block), 0, static_cast<hipStream_t>(stream),
                       static_cast<const float4 *>(src), n16, sink);
    return (int)hipGetLastError();
}

int bw_write(void *dst, uint64_t nbytes, int32_t block, void *stream)
{
    if (!dst || (nbytes & 15u) || bad_block(block) || (reinterpret_cast<uintptr_t>(dst) & 15u)) return -1;
    const size_t n16 = nbytes / 16, grid = (n16 + block - 1) / block;
    if (n16 == 0) return 0;
    if (grid > 0x7fffffffu) return -1;
    hipLaunchKernelGGL(k_write16, dim3((unsigned)grid), dim3(block), 0, static_cast<hipStream_t>(stream),
                       static_cast<float4 *>(dst), n16);
    return (int)hipGetLastError();
}

int bw_inplace(void *buf, uint64_t nbytes, int32_t block, void *stream)
{
    if (!buf || (nbytes & 15u) || bad_block(block) || (reinterpret_cast<uintptr_t>(buf) & 15u)) return -1;
    const size_t n16 = nbytes / 16, grid = (n16 + block - 1) / block;
    if (n16 == 0) return 0;
    if (grid > 0x7fffffffu) return -1;
    hipLaunchKernelGGL(k_inplace16, dim3((unsigned)grid), dim3(block), 0, static_cast<hipStream_t>(stream),
                       static_cast<float4 *>(buf), n16);
    return (int)hipGetLastError();
}

}  // extern "C"
