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

// Streaming store of element idx through a raw buffer resource built from a
// wave-uniform plane base (scalar registers): one shared 32-bit byte offset,
// non-temporal cache policy, and stores beyond `nbytes` are dropped by the
// hardware.  gfx9 resource word 3 = 0x00020000; cache-policy bit 1 = nt.
template <typename T>
__device__ __forceinline__ void st_plane_nt(void *plane, uint32_t nbytes, uint32_t idx, T v)
{
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(plane, (short)0, (int)nbytes, 0x00020000);
    if constexpr (sizeof(T) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)(idx * 4u), 0, 2);
    else
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, (int)(idx * 2u), 0, 2);
}

// Arguments of the fused step kernel.
struct StepArgs {
    const void *src;      // buffer A, [19][N]
    void *dst;            // buffer B, [19][N]
    const void *srcp[19]; // plane i of A (scalar base of every load)
    void *dstp[19];       // plane i of B (scalar base of every store)
    Geom geo;
    CollideConst cc;
    uint32_t step;
    uint32_t xcd_remap;   // 1: map blocks so that consecutive tiles share an XCD
    double *partials;     // [gridDim][4] per-block totals (TOTALS only)
    int32_t *flags;       // bit 0: non-finite density seen
    const uint32_t *fmask;  // [ceil(N/32)] 1 bit per site: bead force present (FORCE only)
    const float *force;     // [3][N] bead force density at flagged sites (FORCE only)
};

__device__ __forceinline__ uint32_t tile_index(uint32_t remap)
{
    const uint32_t b = blockIdx.x, G = gridDim.x;
    if (remap && (G & 7u) == 0) return (b & 7u) * (G >> 3) + (b >> 3);
    return b;
}

// Block-wide sums of (FP64 mass, 3 FP32 momentum components) into one FP64
// partial row per block.  Every thread of the block must call it.
__device__ __forceinline__ void block_sum_totals(double *out, double mass, float mom[3])
{
    __shared__ double red[16][4];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mass += __shfl_xor(mass, off, 64);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float x = mom[c];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        mom[c] = x;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        red[wid][0] = mass;
        red[wid][1] = (double)mom[0];
        red[wid][2] = (double)mom[1];
        red[wid][3] = (double)mom[2];
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int nw = (blockDim.x + 63) >> 6;
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// Store the post-collision populations of site s.  The rest population is
// replaced by the residual that makes the stored values of the site sum to the
// stored input values (both sums in FP64), so the site's mass changes only by
// the single rounding of that residual to the storage type.  Returns the
// stored values' FP64 mass and FP32 momentum for the totals.
template <int ST, bool TOTALS>
__device__ __forceinline__ void store_site(void *const *dstp, uint32_t plane_bytes, uint32_t s, const float d[Q],
                                           const float out[Q], double &mass, float mom[3])
{
    using S = Storage<ST>;
    using T = typename S::T;
    double m_in = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) m_in += (double)d[i];
    T v[Q];
    float back[Q];
    double sum = 0.0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        v[i] = S::st(out[i], 0.f);
        back[i] = S::ld(v[i], 0.f);
        sum += (double)back[i];
    }
    v[0] = S::st((float)(m_in - sum), 0.f);
    back[0] = S::ld(v[0], 0.f);
#pragma unroll
    for (int i = 0; i < Q; ++i) st_plane_nt<T>(dstp[i], plane_bytes, s, v[i]);
    if (TOTALS) {
        mass = (double)back[0] + sum;
        mom[0] = (back[1] - back[2]) + (back[7] - back[8]) + (back[9] - back[10]) + (back[11] - back[12]) +
                 (back[13] - back[14]);
        mom[1] = (back[3] - back[4]) + (back[7] - back[8]) - (back[9] - back[10]) + (back[15] - back[16]) +
                 (back[17] - back[18]);
        mom[2] = (back[5] - back[6]) + (back[11] - back[12]) - (back[13] - back[14]) + (back[15] - back[16]) -
                 (back[17] - back[18]);
    }
}

template <int ST, bool THERMAL, bool TOTALS, bool FORCE>
__global__ void __launch_bounds__(1024) k_stream_collide(StepArgs a)
{
    using S = Storage<ST>;
    using T = typename S::T;
    const uint32_t s = tile_index(a.xcd_remap) * blockDim.x + threadIdx.x;
    const bool active = s < a.geo.N;
    double mass = 0.0;
    float mom[3] = {0.f, 0.f, 0.f};
    if (active) {
        uint32_t x, y, z;
        const PullOffsets o = pull_offsets(s, a.geo, x, y, z);
        const uint32_t N = a.geo.N;
        float d[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = S::ld(ld_plane(static_cast<const T *>(a.srcp[i]), pull_src(s, o, i)), 0.f);
        float F[3] = {a.cc.g[0], a.cc.g[1], a.cc.g[2]};
        if (FORCE) {
            if ((a.fmask[s >> 5] >> (s & 31u)) & 1u) {
                F[0] += a.force[s];
                F[1] += a.force[(size_t)N + s];
                F[2] += a.force[2 * (size_t)N + s];
            }
        }
        float out[Q];
        collide_site<THERMAL>(d, F, a.cc, s, a.step, out);
        if (!__builtin_isfinite(out[0])) __hip_atomic_fetch_or(a.flags, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        store_site<ST, TOTALS>(a.dstp, N * (uint32_t)sizeof(T), s, d, out, mass, mom);
    }
    if (TOTALS) block_sum_totals(a.partials + 4 * (size_t)blockIdx.x, mass, mom);
}

}  // namespace lbmi
