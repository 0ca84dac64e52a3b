// Device kernels of liblbmi (gfx950): fused pull-stream + collide, state
// conversions, diagnostics and the point-particle coupling.
//
// Memory layout: two population buffers A (read) and B (written) of
// [19][N] storage elements.  The buffer the next step reads holds the
// post-collision populations of the previous step at their pre-streaming
// site, so the pre-collision state is n_i(r,t) = A_i(r - c_i) (pull).  One
// step reads A at r - c_i, collides at r and writes B at r; then A and B swap.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "collide.h"

namespace lbmi {

constexpr int Q = 19;

// Velocity components of the 19 directions (order fixed by the C ABI).
__device__ __constant__ static const int8_t kCX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__device__ __constant__ static const int8_t kCY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__device__ __constant__ static const int8_t kCZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

// Exact division by a runtime constant for n, d < 2^31: q = (n * M) >> P with
// P = 31 + ceil(log2 d), M = ceil(2^P / d).
struct FastDiv {
    uint32_t d;
    uint32_t M;
    uint32_t P;
};

__host__ __device__ inline FastDiv make_fastdiv(uint32_t d)
{
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    const uint32_t P = 31 + l;
    const uint64_t M = ((1ull << P) + d - 1) / d;
    return FastDiv{d, (uint32_t)M, P};
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv &f)
{
    return (uint32_t)(((uint64_t)n * (uint64_t)f.M) >> f.P);
}

// Storage traits: populations are stored as shifted deviations, optionally
// scaled (FP16) before rounding.
template <int ST> struct Storage;
template <> struct Storage<1> {  // LB_F32
    using T = float;
    static __device__ __forceinline__ float ld(T v, float) { return v; }
    static __device__ __forceinline__ T st(float f, float) { return f; }
};
template <> struct Storage<2> {  // LB_BF16
    using T = __bf16;
    static __device__ __forceinline__ float ld(T v, float) { return (float)v; }
    static __device__ __forceinline__ T st(float f, float) { return (__bf16)f; }
};
template <> struct Storage<3> {  // LB_F16, stored value = 2^8 * deviation
    using T = _Float16;
    static __device__ __forceinline__ float ld(T v, float) { return (float)v * 0x1p-8f; }
    static __device__ __forceinline__ T st(float f, float) { return (_Float16)(f * 0x1p8f); }
};

// Geometry of one periodic box.
struct Geom {
    uint32_t nx, ny, nz, N, nxny;
    FastDiv div_nx, div_ny;
};

// Neighbour offsets of site s: off[c+1] for c = -1, 0, +1 along each axis is
// the index offset of the site r - c (pull source) with periodic wrap.
struct PullOffsets {
    int32_t ox_m, ox_p, oy_m, oy_p, oz_m, oz_p;  // _m: source of c=+1 (r-1); _p: source of c=-1 (r+1)
};

__device__ __forceinline__ PullOffsets pull_offsets(uint32_t s, const Geom &g, uint32_t &x, uint32_t &y, uint32_t &z)
{
    const uint32_t q = fdiv(s, g.div_nx);
    x = s - q * g.nx;
    z = fdiv(q, g.div_ny);
    y = q - z * g.ny;
    PullOffsets o;
    o.ox_m = (x == 0) ? (int32_t)(g.nx - 1) : -1;
    o.ox_p = (x == g.nx - 1) ? -(int32_t)(g.nx - 1) : 1;
    o.oy_m = (y == 0) ? (int32_t)((g.ny - 1) * g.nx) : -(int32_t)g.nx;
    o.oy_p = (y == g.ny - 1) ? -(int32_t)((g.ny - 1) * g.nx) : (int32_t)g.nx;
    o.oz_m = (z == 0) ? (int32_t)((g.nz - 1) * g.nxny) : -(int32_t)g.nxny;
    o.oz_p = (z == g.nz - 1) ? -(int32_t)((g.nz - 1) * g.nxny) : (int32_t)g.nxny;
    return o;
}

// Source site of population i for a pull at s.
__device__ __forceinline__ uint32_t pull_src(uint32_t s, const PullOffsets &o, int i)
{
    switch (i) {
    case 0: return s;
    case 1: return s + o.ox_m;
    case 2: return s + o.ox_p;
    case 3: return s + o.oy_m;
    case 4: return s + o.oy_p;
    case 5: return s + o.oz_m;
    case 6: return s + o.oz_p;
    case 7: return s + o.ox_m + o.oy_m;
    case 8: return s + o.ox_p + o.oy_p;
    case 9: return s + o.ox_m + o.oy_p;
    case 10: return s + o.ox_p + o.oy_m;
    case 11: return s + o.ox_m + o.oz_m;
    case 12: return s + o.ox_p + o.oz_p;
    case 13: return s + o.ox_m + o.oz_p;
    case 14: return s + o.ox_p + o.oz_m;
    case 15: return s + o.oy_m + o.oz_m;
    case 16: return s + o.oy_p + o.oz_p;
    case 17: return s + o.oy_m + o.oz_p;
    default: return s + o.oy_p + o.oz_m;
    }
}

// Load element idx of population plane `plane` (byte offset arithmetic kept
// in 32 bits so the load uses a scalar base and a 32-bit vector offset).
template <typename T>
__device__ __forceinline__ T ld_plane(const T *__restrict__ plane, uint32_t idx)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(plane) + (uint32_t)(idx * (uint32_t)sizeof(T)));
}

template <typename T>
__device__ __forceinline__ void st_plane(T *__restrict__ plane, uint32_t idx, T v)
{
    __builtin_nontemporal_store(v, reinterpret_cast<T *>(reinterpret_cast<char *>(plane) + (uint32_t)(idx * (uint32_t)sizeof(T))));
}

// Arguments of the fused step kernel.
struct StepArgs {
    const void *src;      // buffer A, [19][N]
    void *dst;            // buffer B, [19][N]
    Geom geo;
    CollideConst cc;
    uint32_t step;
    uint32_t xcd_remap;   // 1: map blocks so that consecutive tiles share an XCD
    double *partials;     // [gridDim][4] per-block totals (TOTALS only)
    int32_t *flags;       // bit 0: non-finite density seen
};

__device__ __forceinline__ uint32_t tile_index(uint32_t remap)
{
    const uint32_t b = blockIdx.x, G = gridDim.x;
    if (remap && (G & 7u) == 0) return (b & 7u) * (G >> 3) + (b >> 3);
    return b;
}

// Block-wide sum of 4 floats into one FP64 partial per block.
template <int NV>
__device__ __forceinline__ void block_sum_to(double *out, float v[NV])
{
    __shared__ double red[16][NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        float x = v[c];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        v[c] = x;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < NV; ++c) red[wid][c] = (double)v[c];
    __syncthreads();
    if (threadIdx.x < NV) {
        const int nw = (blockDim.x + 63) >> 6;
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

template <int ST, bool THERMAL, bool TOTALS>
__global__ void __launch_bounds__(1024) k_stream_collide(StepArgs a)
{
    using S = Storage<ST>;
    using T = typename S::T;
    const uint32_t s = tile_index(a.xcd_remap) * blockDim.x + threadIdx.x;
    const bool active = s < a.geo.N;
    float tot[4] = {0.f, 0.f, 0.f, 0.f};
    if (active) {
        uint32_t x, y, z;
        const PullOffsets o = pull_offsets(s, a.geo, x, y, z);
        const T *__restrict__ src = static_cast<const T *>(a.src);
        T *__restrict__ dst = static_cast<T *>(a.dst);
        const uint32_t N = a.geo.N;
        float d[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = S::ld(ld_plane(src + (size_t)i * N, pull_src(s, o, i)), 0.f);
        float out[Q];
        collide_site<THERMAL>(d, a.cc.g, a.cc, s, a.step, out);
        if (!__builtin_isfinite(out[0])) __hip_atomic_fetch_or(a.flags, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const T v = S::st(out[i], 0.f);
            st_plane(dst + (size_t)i * N, s, v);
            if (TOTALS) out[i] = S::ld(v, 0.f);
        }
        if (TOTALS) {
            float msum = out[0];
#pragma unroll
            for (int i = 1; i < Q; ++i) msum += out[i];
            tot[0] = msum;
            tot[1] = (out[1] - out[2]) + (out[7] - out[8]) + (out[9] - out[10]) + (out[11] - out[12]) +
                     (out[13] - out[14]);
            tot[2] = (out[3] - out[4]) + (out[7] - out[8]) - (out[9] - out[10]) + (out[15] - out[16]) +
                     (out[17] - out[18]);
            tot[3] = (out[5] - out[6]) + (out[11] - out[12]) - (out[13] - out[14]) + (out[15] - out[16]) -
                     (out[17] - out[18]);
        }
    }
    if (TOTALS) block_sum_to<4>(a.partials + 4 * (size_t)blockIdx.x, tot);
}

}  // namespace lbmi
