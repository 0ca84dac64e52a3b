// Device kernels of liblbmi (gfx950): fused pull-stream + collide, state
// conversions, diagnostics and the point-particle coupling.
//
// Memory layout: two population buffers A (read) and B (written) of P N
// storage elements, z-major for a single box (pop[z][i][y][x], pop_index)
// and [P][N] for the boxes of a batch.  P = 19 planes for 16-bit storage;
// FP32 storage has P = 20: plane 19 holds the FP32 rounding residual of the
// rest population, whose value is the unevaluated sum of planes 0 and 19
// (see store_site).  The buffer the next step reads
// holds the post-collision populations of the previous step at their
// pre-streaming site, so the pre-collision state is n_i(r,t) = A_i(r - c_i)
// (pull).  One step reads A at r - c_i, collides at r and writes B at r; then
// A and B swap.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

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
    static constexpr bool rest_lo = true;  // rest population carries its residual plane
    static __device__ __forceinline__ float ld(T v, float) { return v; }
    static __device__ __forceinline__ T st(float f, float) { return f; }
};
template <> struct Storage<2> {  // LB_BF16
    using T = __bf16;
    static constexpr bool rest_lo = false;
    static __device__ __forceinline__ float ld(T v, float) { return (float)v; }
    static __device__ __forceinline__ T st(float f, float) { return (__bf16)f; }
};
template <> struct Storage<3> {  // LB_F16, stored value = 2^8 * deviation
    using T = _Float16;
    static constexpr bool rest_lo = false;
    static __device__ __forceinline__ float ld(T v, float) { return (float)v * 0x1p-8f; }
    static __device__ __forceinline__ T st(float f, float) { return (_Float16)(f * 0x1p8f); }
};

// Stochastic rounding of the step kernels' stores (16-bit storage only).
// Round to nearest even applied every step to thermally dithered values
// shrinks every population's mean deviation by a factor 1 - u^2 / (32 ln 2)
// per step (u = relative spacing of the format: the rounding cell of a power
// of two reaches a quarter spacing below and half a spacing above it), which
// acts on the hydrodynamic modes like a friction of that size: for BF16
// (u = 2^-7) 2.7e-6 per step, about 11 % of the viscous decay rate of the
// longest shear wave of a 512 box.  Stochastic rounding has no such bias:
// a value is rounded up in magnitude with probability equal to its distance
// from the lower neighbour in units of the spacing.  Here the probability is
// resolved to 1/64: with D dropped FP32 mantissa bits (16 for BF16, 13 for
// FP16) the offset r6 2^(D-6) + c is added to the magnitude bits before
// they are cut, c = 2^(D-7) - 1 + b with b a fair bit shared by the site's
// values.  Its mean is (2^D - 1) / 2, the mean of the dropped bits, so over
// the FP32 values of a cell the rounding is exactly unbiased (a constant
// c = 2^(D-7) would add half an FP32 ulp to every magnitude: a growth of
// 2^-24 per step), and every value's round-up probability is within 1/128
// of its exact one; the binade-edge term left by the 1/64 resolution is
// 4096 times smaller than that of nearest rounding.  The 6-bit fields r6
// and the bit b come from one Philox4x32-10 call of its own stream.
template <int D>
__device__ __forceinline__ uint32_t sr_offset(uint32_t r6, uint32_t b)
{
    return (r6 << (D - 6)) + ((1u << (D - 7)) - 1u) + b;
}
template <> struct Storage<4> : Storage<2> {  // LB_BF16, stochastic rounding
    static __device__ __forceinline__ T st_sr(float f, uint32_t r6, uint32_t b)
    {
        const uint32_t x = (__float_as_uint(f) + sr_offset<16>(r6, b)) >> 16;
        return __builtin_bit_cast(__bf16, (uint16_t)x);
    }
};
template <> struct Storage<5> : Storage<3> {  // LB_F16, stochastic rounding
    static __device__ __forceinline__ T st_sr(float f, uint32_t r6, uint32_t b)
    {
        // clear the 13 mantissa bits FP16 drops; the conversion of the result
        // is exact wherever 2^8 |f| is an FP16 normal number (|f| >= 2^-22)
        const uint32_t x = (__float_as_uint(f * 0x1p8f) + sr_offset<13>(r6, b)) & 0xFFFFE000u;
        return (_Float16)__uint_as_float(x);
    }
};
template <int ST> struct is_stochastic { static constexpr bool value = ST >= 4; };

// log2 of the scale of the stored value (FP16 stores 2^8 times the
// deviation): the collision's outputs come out in that scale.
template <int ST> struct out_scale { static constexpr int value = (ST == 3 || ST == 5) ? 8 : 0; };

// The four random words of one site's stochastic rounding: Philox counter
// (site, step, stream 3 << 16, box), key = seed.  Population i uses the
// 6-bit field (i % 5) of word i / 5; the site's offset bit b is bit 24 of
// the fourth word (its fields use bits 0..23).
__device__ __forceinline__ Philox4 rounding_words(uint32_t s, uint32_t step, uint32_t box, uint32_t k0, uint32_t k1)
{
    return philox4x32_10(s, step, 3u << 16, box, k0, k1);
}
__device__ __forceinline__ uint32_t rounding_field(const Philox4 &w, int i)
{
    const uint32_t word = (i < 5) ? w.v0 : (i < 10) ? w.v1 : (i < 15) ? w.v2 : w.v3;
    return (word >> (6 * (i % 5))) & 63u;
}
__device__ __forceinline__ uint32_t rounding_bit(const Philox4 &w) { return (w.v3 >> 24) & 1u; }

// Geometry of one periodic box.
struct Geom {
    uint32_t nx, ny, nz, N, nxny;
    FastDiv div_nx, div_ny;
    uint32_t walls;  // 1: stationary walls at z = -1/2 and z = nz - 1/2
    uint32_t zmajor; // population layout, see pop_index
    uint32_t planes; // planes per layer (z-major) or per box: 19, or 20 with the rest residual plane
};

// Plane of the rest population's rounding residual (FP32 storage only).
constexpr int kRestLo = 19;

// Element index of population i of site s (layer z) in a population buffer
// (i = kRestLo: the rest residual plane).
// zmajor = 1 (a single box): [z][i][y][x], the planes of one z-layer side
// by side, so that the 38 streams of a step stay within a few MB of each
// other (measured faster than [i][z][y][x] for the pull pattern); zmajor = 0
// (the boxes of a batch): [i][z][y][x].
__device__ __forceinline__ size_t pop_index(int i, uint32_t s, uint32_t z, const Geom &g)
{
    if (g.zmajor) return (size_t)(g.planes * z + (uint32_t)i) * g.nxny + (s - z * g.nxny);
    return (size_t)i * g.N + s;
}

// Element index of the adjoint lambda_i of site s (layer z): z-major with 19
// planes per layer whatever the storage (the adjoint is FP32 and has no
// residual plane).
__device__ __forceinline__ size_t lam_index(int i, uint32_t s, uint32_t z, const Geom &g)
{
    return (size_t)(19u * z + (uint32_t)i) * g.nxny + (s - z * g.nxny);
}

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

// Opposite direction of population i (pairs are adjacent: 1<->2, 3<->4, ...).
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// Stationary walls half way along the links at z = -1/2 and z = nz - 1/2
// (eq. MBB with the wall at rest, u_b = 0): a population whose link crosses a
// wall comes back reversed to the site it left.
//   pull_crosses: the pull source r - c_i of population i at layer z lies
//                 beyond a wall, so n_i(r, t+1) = A_{opp(i)}(r);
//   push_crosses: the link r -> r + c_i crosses a wall, so the stored A_i(r)
//                 is read back as n_{opp(i)}(r).
// WALLS = false compiles the wall test away (kernels instantiated for the
// periodic box); the default checks the geometry's flag at run time.
template <bool WALLS = true>
__device__ __forceinline__ bool pull_crosses(const Geom &g, uint32_t z, int i)
{
    if constexpr (!WALLS) return false;
    return g.walls && ((kCZ[i] > 0 && z == 0u) || (kCZ[i] < 0 && z + 1u == g.nz));
}
template <bool WALLS = true>
__device__ __forceinline__ bool push_crosses(const Geom &g, uint32_t z, int i)
{
    if constexpr (!WALLS) return false;
    return g.walls && ((kCZ[i] < 0 && z == 0u) || (kCZ[i] > 0 && z + 1u == g.nz));
}

// Layer of the pull source of population i at layer z (periodic).
__device__ __forceinline__ uint32_t pull_z(uint32_t z, int i, const Geom &g)
{
    if (kCZ[i] > 0) return z == 0u ? g.nz - 1u : z - 1u;
    if (kCZ[i] < 0) return z + 1u == g.nz ? 0u : z + 1u;
    return z;
}

// Element index (pop_index) of the stored value that population i of site s
// (layer z) pulls.
template <bool WALLS = true>
__device__ __forceinline__ size_t pull_index(uint32_t s, const PullOffsets &o, int i, uint32_t z, const Geom &g)
{
    if (pull_crosses<WALLS>(g, z, i)) return pop_index(opp(i), s, z, g);
    return pop_index(i, pull_src(s, o, i), pull_z(z, i, g), g);
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

// The bead force field is kept in fixed point, in units of 2^-44: the spread
// contributions of many beads then add up with integer atomics, whose sum does
// not depend on their order (coupled runs repeat bit for bit).  2^-44 is
// finer than the FP32 spacing of any force above 2^-21 and leaves |f| < 2^18
// for the sum.
constexpr double kForceScale = 17592186044416.0;  // 2^44
constexpr double kForceLimit = 262144.0;          // 2^18: larger or non-finite contributions are refused

__device__ __forceinline__ float force_value(long long q) { return (float)((double)q * (1.0 / kForceScale)); }

// Arguments of the fused step kernel.
struct StepArgs {
    const void *src;      // buffer A (layout pop_index, zmajor)
    void *dst;            // buffer B
    Geom geo;
    uint32_t tiles;       // blocks per z-layer: ceil(nxny / blockDim)
    FastDiv div_tiles;
    CollideConst cc;
    uint32_t step;
    uint32_t xcd_remap;   // 1: map blocks so that consecutive tiles share an XCD
    double *partials;     // [gridDim][4] per-block totals (TOTALS only)
    int32_t *flags;       // bit 0: non-finite density seen
    uint32_t *fmask;        // [ceil(N/32)] 1 bit per site: bead force present (FORCE only)
    long long *force;       // [3][N] bead force density at flagged sites, fixed point (FORCE only)
    uint32_t consume;       // FORCE: 1 = zero the force rows and bitmap words this step read
    // fused coupled step (k_coupled_step): the first block0 blocks of the
    // grid are the particle half, which adds the bead force of this step
    // while the site blocks run; a site block reads a flagged site's force
    // once *arrive has reached arrive_target (every particle block counted)
    uint32_t *arrive;
    uint32_t arrive_target;
    uint32_t block0;
    // MOM (recompute sweep of the reverse pass): the input state's moments
    // (rho - rho0, j) per site, 4 planes per layer [z][4][y][x], FP32 sums
    // in the order the adjoint step forms them from the same stored values
    float *moments;
};

// Tile of block b of G site blocks: with remap, consecutive tiles go to one
// XCD (hardware block b runs on XCD b mod 8).
__device__ __forceinline__ uint32_t tile_of(uint32_t b, uint32_t G, uint32_t remap)
{
    if (remap && (G & 7u) == 0) return (b & 7u) * (G >> 3) + (b >> 3);
    return b;
}

__device__ __forceinline__ uint32_t tile_index(uint32_t remap) { return tile_of(blockIdx.x, gridDim.x, remap); }

// Bound on the polls of a site wave waiting for the particle blocks of its
// launch (each poll is a device-coherent load, about a microsecond): the
// particle blocks come first in the grid and wait for nothing, so the count
// is normally reached within a few polls; if it is not, the wave gives up,
// latches bit 3 of the device flags (the host reports the step as failed)
// and goes on, so that no launch can hang.
constexpr uint32_t kArriveSpinLimit = 1u << 16;

__device__ __forceinline__ void wait_arrivals(const uint32_t *arrive, uint32_t target, int32_t *flags)
{
    for (uint32_t k = 0; k < kArriveSpinLimit; ++k) {
        const uint32_t v = __hip_atomic_load(arrive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((int32_t)(v - target) >= 0) return;
        __builtin_amdgcn_s_sleep(2);
    }
    __hip_atomic_fetch_or(flags, 8, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block-wide sums of (FP64 mass, 3 FP32 momentum components) into one FP64
// partial row per block, in a fixed order.  Every thread writes its values
// to LDS; the block's first wave adds them (each lane a strided subset, then
// across the wave with DPP, no LDS) and writes the row, so the other waves
// spend two LDS stores and a barrier on it instead of a wave reduction
// each.  Every thread of the block must call it.
// The LDS it uses is the launch's dynamic shared memory, kTotalsLds bytes
// per thread.
constexpr uint32_t kTotalsLds = 20;

// v plus the value DPP control CTRL brings from another lane (0 for a lane
// with no source, or outside ROW_MASK), for an FP64 value: both halves move
// with the same control.  Every lane of the wave must be active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double add_dpp_f64(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROW_MASK, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROW_MASK, 0xf, false);
    return v + __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over the wave's 64 lanes, complete in lane 63: an inclusive scan in
// each row of 16 lanes (row shifts by 1, 2, 4, 8), then the row totals
// carried up by the row broadcasts (lane 15 into rows 1 and 3, lane 31 into
// rows 2 and 3).
__device__ __forceinline__ double wave_sum_lane63_f64(double x)
{
    x = add_dpp_f64<0x111, 0xf>(x);  // row_shr:1
    x = add_dpp_f64<0x112, 0xf>(x);  // row_shr:2
    x = add_dpp_f64<0x114, 0xf>(x);  // row_shr:4
    x = add_dpp_f64<0x118, 0xf>(x);  // row_shr:8
    x = add_dpp_f64<0x142, 0xa>(x);  // row_bcast:15
    x = add_dpp_f64<0x143, 0xc>(x);  // row_bcast:31
    return x;
}

__device__ __forceinline__ void block_sum_totals(double *out, double mass, float mom[3])
{
    extern __shared__ __align__(8) char totals_lds[];
    double *red_m = reinterpret_cast<double *>(totals_lds);
    float *red_p = reinterpret_cast<float *>(totals_lds + 8 * blockDim.x);
    const uint32_t t = threadIdx.x, nb = blockDim.x;
    red_m[t] = mass;
    red_p[t] = mom[0];
    red_p[nb + t] = mom[1];
    red_p[2 * nb + t] = mom[2];
    __syncthreads();
    if (t >= 64) return;
    double m = 0.0;
    double p[3] = {0.0, 0.0, 0.0};
    for (uint32_t k = t; k < nb; k += 64) {
        m += red_m[k];
        p[0] += (double)red_p[k];
        p[1] += (double)red_p[nb + k];
        p[2] += (double)red_p[2 * nb + k];
    }
    m = wave_sum_lane63_f64(m);
#pragma unroll
    for (int c = 0; c < 3; ++c) p[c] = wave_sum_lane63_f64(p[c]);
    if (t == 63) {
        out[0] = m;
        out[1] = p[0];
        out[2] = p[1];
        out[3] = p[2];
    }
}

// Accumulation type of a site's mass: FP32 storage sums in FP64; 16-bit
// storage sums its (exactly FP32-representable) values in FP32, whose
// rounding is far below the 16-bit rounding of the residual.
template <int ST> using mass_acc_t = typename std::conditional<ST == 1, double, float>::type;

// Input mass of a site: the sum of its gathered deviations.  Taken right
// after the gather, so that the 19 inputs do not stay live through the
// collision (that would cost the step kernel a sixth of its occupancy).
template <int ST>
__device__ __forceinline__ mass_acc_t<ST> site_mass(const float d[Q])
{
    mass_acc_t<ST> m = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) m += (mass_acc_t<ST>)d[i];
    return m;
}

// Input mass of a site with the rest residual plane (FP32 storage): the
// gathered deviations plus the residual lo of the site's rest population.
template <int ST>
__device__ __forceinline__ mass_acc_t<ST> site_mass_lo(const float d[Q], float lo)
{
    mass_acc_t<ST> m = site_mass<ST>(d);
    if constexpr (Storage<ST>::rest_lo) m += (double)lo;
    return m;
}

// Pairs of 16-bit stored values in one 32-bit word (population 2p+1 in the
// low half, 2p+2 in the high half) and their FP32 sums with gfx950's
// two-element dot products (v_dot2c_f32_bf16 / v_dot2_f32_f16) against +-1
// (BF16) or +-2^-8 (FP16, whose stored value is 2^8 times the deviation):
// one instruction adds a pair to a sum, exactly the deviations the stored
// bits represent.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));

// pack(a, b, rw, i): a, b are in the stored scale (2^8 d for FP16);
// stochastic rounding reads the 6-bit fields i and i + 1 of rw.
template <int ST> struct Pair16;
template <> struct Pair16<2> {  // BF16, round to nearest even
    static __device__ __forceinline__ uint32_t pack(float a, float b, const Philox4 &, int)
    {
        const bf16x2_t v = {(__bf16)a, (__bf16)b};
        return __builtin_bit_cast(uint32_t, v);
    }
    static __device__ __forceinline__ float dot(uint32_t pk, float lo_c, float hi_c, float acc)
    {
        const bf16x2_t c = {(__bf16)lo_c, (__bf16)hi_c};
        return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, pk), c, acc, false);
    }
};
template <> struct Pair16<3> {  // FP16 (scaled by 2^8), round to nearest even
    static __device__ __forceinline__ uint32_t pack(float a, float b, const Philox4 &, int)
    {
        const f16x2_t v = {(_Float16)a, (_Float16)b};
        return __builtin_bit_cast(uint32_t, v);
    }
    static __device__ __forceinline__ float dot(uint32_t pk, float lo_c, float hi_c, float acc)
    {
        const f16x2_t c = {(_Float16)(lo_c * 0x1p-8f), (_Float16)(hi_c * 0x1p-8f)};
        return __builtin_amdgcn_fdot2(__builtin_bit_cast(f16x2_t, pk), c, acc, false);
    }
};

// The bits of the FP32 value f plus the stochastic-rounding offset of field
// i (sr_offset, D dropped bits): a bit-field extract of the Philox word, a
// shift-and-add and an add of the site's constant part.
template <int D>
__device__ __forceinline__ uint32_t sr_add(float f, const Philox4 &rw, int i)
{
    const uint32_t w = (i < 5) ? rw.v0 : (i < 10) ? rw.v1 : (i < 15) ? rw.v2 : rw.v3;
    const uint32_t r6 = __builtin_amdgcn_ubfe(w, 6u * (uint32_t)(i % 5), 6u);
    return __float_as_uint(f) + sr_offset<D>(r6, rounding_bit(rw));
}
template <> struct Pair16<4> : Pair16<2> {  // BF16, stochastic rounding
    static __device__ __forceinline__ uint32_t pack(float a, float b, const Philox4 &rw, int i)
    {
        // the high halves of the two offset words, a in the low half
        return __builtin_amdgcn_perm(sr_add<16>(b, rw, i + 1), sr_add<16>(a, rw, i), 0x07060302u);
    }
};
template <> struct Pair16<5> : Pair16<3> {  // FP16, stochastic rounding
    static __device__ __forceinline__ uint32_t pack(float a, float b, const Philox4 &rw, int i)
    {
        // clear the 13 mantissa bits FP16 drops; the conversion of the result
        // is exact wherever |value| >= 2^-14 (FP16 normal)
        const float ra = __uint_as_float(sr_add<13>(a, rw, i) & 0xFFFFE000u);
        const float rb = __uint_as_float(sr_add<13>(b, rw, i + 1) & 0xFFFFE000u);
        const f16x2_t v = {(_Float16)ra, (_Float16)rb};
        return __builtin_bit_cast(uint32_t, v);
    }
};

// Store of a site in 16-bit storage (the 16-bit counterpart of store_site
// below): the 18 moving populations (out[], in the stored scale) rounded in
// pairs, their stored values summed by dot products, the rest population
// set to the residual x = m_in - sum and rounded once.  With TOTALS also the stored values'
// mass (FP64) and momentum (dot products against the pairs' signs: the two
// members of every pair are opposite directions).
template <int ST, bool TOTALS>
__device__ __forceinline__ void store_site16(void *const *dstp, uint32_t plane_bytes, uint32_t s, float m_in,
                                             const float out[Q], double &mass, float mom[3], const Philox4 &rw)
{
    using S = Storage<ST>;
    using T = typename S::T;
    using P = Pair16<ST>;
    uint32_t pk[9];
    float sum = 0.f;
#pragma unroll
    for (int p = 0; p < 9; ++p) {
        pk[p] = P::pack(out[2 * p + 1], out[2 * p + 2], rw, 2 * p + 1);
        // keep the packed word as it is: the stores take its halves (the low
        // half as is, the high half shifted down; the raw buffer store has
        // no high-half form) instead of the compiler converting each value
        // a second time
        __asm__ volatile("" : "+v"(pk[p]));
        sum = P::dot(pk[p], 1.f, 1.f, sum);
    }
    const float x = m_in - sum;
    T v0;
    if constexpr (is_stochastic<ST>::value) v0 = S::st_sr(x, rounding_field(rw, 0), rounding_bit(rw));
    else v0 = S::st(x, 0.f);
    st_plane_nt<T>(dstp[0], plane_bytes, s, v0);
#pragma unroll
    for (int p = 0; p < 9; ++p) {
        st_plane_nt<T>(dstp[2 * p + 1], plane_bytes, s, __builtin_bit_cast(T, (uint16_t)pk[p]));
        st_plane_nt<T>(dstp[2 * p + 2], plane_bytes, s, __builtin_bit_cast(T, (uint16_t)(pk[p] >> 16)));
    }
    if (TOTALS) {
        mass = (double)S::ld(v0, 0.f) + (double)sum;
        // x: pairs 0 (+-x), 3, 4, 5, 6; y: 1 (+-y), 3, 4 (-), 7, 8; z: 2 (+-z), 5, 6 (-), 7, 8 (-)
        mom[0] = P::dot(pk[6], 1.f, -1.f, P::dot(pk[5], 1.f, -1.f, P::dot(pk[4], 1.f, -1.f,
                 P::dot(pk[3], 1.f, -1.f, P::dot(pk[0], 1.f, -1.f, 0.f)))));
        mom[1] = P::dot(pk[8], 1.f, -1.f, P::dot(pk[7], 1.f, -1.f, P::dot(pk[4], -1.f, 1.f,
                 P::dot(pk[3], 1.f, -1.f, P::dot(pk[1], 1.f, -1.f, 0.f)))));
        mom[2] = P::dot(pk[8], -1.f, 1.f, P::dot(pk[7], 1.f, -1.f, P::dot(pk[6], -1.f, 1.f,
                 P::dot(pk[5], 1.f, -1.f, P::dot(pk[2], 1.f, -1.f, 0.f)))));
    }
}

// Store the post-collision populations of site s.  The rest population is
// replaced by the residual x = m_in - sum_{i>=1} stored_i that makes the
// stored values of the site sum to its input mass m_in (site_mass_lo): the
// collision conserves each site's mass (the constraint on the collision after
// eq. LBE), and so does the store.  16-bit storage rounds x once.  FP32
// storage keeps x as hi + lo: hi = fp32(x) in the rest plane and
// lo = fp32(x - hi) in the residual plane dstp[kRestLo], so the site's stored
// mass differs from m_in only by the rounding of lo (below 2^-25 ulp(hi))
// and the FP64 sums (2^-53 relative): total mass is conserved to ~1e-16
// relative per step instead of random-walking by one FP32 rounding per site
// and step.  Returns the stored values' mass (FP64) and momentum (FP32) for
// the totals.
template <int ST, bool TOTALS>
__device__ __forceinline__ void store_site(void *const *dstp, uint32_t plane_bytes, uint32_t s, mass_acc_t<ST> m_in,
                                           const float out[Q], double &mass, float mom[3], const Philox4 &rw)
{
    using S = Storage<ST>;
    using T = typename S::T;
    using Acc = mass_acc_t<ST>;
    T v[Q];
    float back[Q];
    Acc sum = 0;
    static_assert(S::rest_lo, "store_site is the FP32 store; 16-bit storage uses store_site16");
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        v[i] = S::st(out[i], 0.f);
        back[i] = S::ld(v[i], 0.f);
        sum += (Acc)back[i];
    }
    const Acc x = m_in - sum;
    v[0] = S::st((float)x, 0.f);
    back[0] = S::ld(v[0], 0.f);
    float lo = 0.f;
    if constexpr (S::rest_lo) lo = (float)(x - (Acc)back[0]);
#pragma unroll
    for (int i = 0; i < Q; ++i) st_plane_nt<T>(dstp[i], plane_bytes, s, v[i]);
    if constexpr (S::rest_lo) st_plane_nt<float>(dstp[kRestLo], plane_bytes, s, lo);
    if (TOTALS) {
        mass = ((double)back[0] + (double)lo) + (double)sum;
        mom[0] = (back[1] - back[2]) + (back[7] - back[8]) + (back[9] - back[10]) + (back[11] - back[12]) +
                 (back[13] - back[14]);
        mom[1] = (back[3] - back[4]) + (back[7] - back[8]) - (back[9] - back[10]) + (back[15] - back[16]) +
                 (back[17] - back[18]);
        mom[2] = (back[5] - back[6]) + (back[11] - back[12]) - (back[13] - back[14]) + (back[15] - back[16]) -
                 (back[17] - back[18]);
    }
}

// One site of the fused step: gather with pull streaming, collide, store,
// optionally accumulate the block's totals.  Blocks are dealt out layer by
// layer (block b: layer z = b / tiles, in-layer sites r = (b - z tiles)
// blockDim + thread), so the base of every plane a block loads from or
// stores to is uniform over the block (the buffers are z-major, pop_index).
// WAIT (fused coupled step): the grid's first a.block0 blocks are not site
// blocks, and the bead force of a flagged site is taken once the particle
// blocks have all been counted (wait_arrivals), with device-scope atomic
// exchanges that read it and leave the field zero.
template <int ST, bool THERMAL, bool TOTALS, bool FORCE, bool WALLS, bool FULL, bool WAIT = false, bool MOM = false>
__device__ __forceinline__ void stream_collide_site(const StepArgs &a)
{
    using S = Storage<ST>;
    using T = typename S::T;
    const uint32_t b = WAIT ? tile_of(blockIdx.x - a.block0, gridDim.x - a.block0, a.xcd_remap) : tile_index(a.xcd_remap);
    const uint32_t z = fdiv(b, a.div_tiles);
    const uint32_t nxny = a.geo.nxny;
    const uint32_t r = (b - z * a.tiles) * blockDim.x + threadIdx.x;
    const bool active = r < nxny;
    const uint32_t s = z * nxny + r;
    const size_t plane = (size_t)nxny * sizeof(T);
    const uint32_t P = a.geo.planes;
    const char *src = static_cast<const char *>(a.src);
    char *dst = static_cast<char *>(a.dst);
    double mass = 0.0;
    float mom[3] = {0.f, 0.f, 0.f};
    if (active) {
        uint32_t x, y, zs;
        const PullOffsets o = pull_offsets(s, a.geo, x, y, zs);
        PullOffsets oxy = o;  // in-layer part of each pull; the layer picks the plane base
        oxy.oz_m = 0;
        oxy.oz_p = 0;
        const uint32_t N = a.geo.N;
        float d[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const T *base = reinterpret_cast<const T *>(src + (size_t)(P * pull_z(z, i, a.geo) + (uint32_t)i) * plane);
            d[i] = S::ld(ld_plane(base, pull_src(r, oxy, i)), 0.f);
        }
        float lo_in = 0.f;
        if constexpr (S::rest_lo)
            lo_in = ld_plane(reinterpret_cast<const float *>(src + (size_t)(P * z + (uint32_t)kRestLo) * plane), r);
        if constexpr (WALLS) {
            if (z == 0u || z + 1u == a.geo.nz) {
                // wall layers: the populations coming off a wall are the reversed ones of this site
#pragma unroll
                for (int i = 0; i < Q; ++i)
                    if (pull_crosses(a.geo, z, i))
                        d[i] = S::ld(ld_plane(reinterpret_cast<const T *>(src + (size_t)(P * z + (uint32_t)opp(i)) * plane),
                                              r),
                                     0.f);
            }
        }
        if constexpr (MOM) {
            // the input state's (rho - rho0, j) for the reverse sweep's adjoint step
            float m0 = d[0], jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                m0 += d[i];
                jx += (float)kCX[i] * d[i];
                jy += (float)kCY[i] * d[i];
                jz += (float)kCZ[i] * d[i];
            }
            float *mp = a.moments + (size_t)(4u * z) * nxny;
            st_plane_nt<float>(mp, (uint32_t)(nxny * 4u), r, m0);
            st_plane_nt<float>(mp + nxny, (uint32_t)(nxny * 4u), r, jx);
            st_plane_nt<float>(mp + 2 * (size_t)nxny, (uint32_t)(nxny * 4u), r, jy);
            st_plane_nt<float>(mp + 3 * (size_t)nxny, (uint32_t)(nxny * 4u), r, jz);
        }
        // FP32 storage: the input mass in FP64 with the rest residual (exact);
        // 16-bit storage: the collision's own FP32 sum below
        mass_acc_t<ST> m_in = 0;
        if constexpr (S::rest_lo) m_in = site_mass_lo<ST>(d, lo_in);
        float F[3] = {a.cc.g[0], a.cc.g[1], a.cc.g[2]};
        if (FORCE && WAIT) {
            const uint32_t bit = 1u << (s & 31u);
            const bool flagged = (a.fmask[s >> 5] & bit) != 0u;
            if (__any(flagged)) wait_arrivals(a.arrive, a.arrive_target, a.flags);
            if (flagged) {
                // the spread of this launch's particle blocks was performed
                // (device-scope atomics) before their count reached the
                // target; the exchanges are issued after it was seen
                long long *f = a.force;
                F[0] += force_value(__hip_atomic_exchange(&f[s], 0ll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                F[1] += force_value(
                    __hip_atomic_exchange(&f[(size_t)N + s], 0ll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                F[2] += force_value(
                    __hip_atomic_exchange(&f[2 * (size_t)N + s], 0ll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                atomicAnd(&a.fmask[s >> 5], ~bit);
            }
        } else if (FORCE) {
            const uint32_t bit = 1u << (s & 31u);
            if (a.fmask[s >> 5] & bit) {
                F[0] += force_value(a.force[s]);
                F[1] += force_value(a.force[(size_t)N + s]);
                F[2] += force_value(a.force[2 * (size_t)N + s]);
                if (a.consume) {
                    // leave the field and this site's bit zero (the other
                    // sites of the word have read or will read their own bits)
                    a.force[s] = 0;
                    a.force[(size_t)N + s] = 0;
                    a.force[2 * (size_t)N + s] = 0;
                    atomicAnd(&a.fmask[s >> 5], ~bit);
                }
            }
        }
        float out[Q], m0;
        collide_site<THERMAL, FULL, out_scale<ST>::value, ST == 1>(d, F, a.cc, s, a.step, out, m0);
        if (!__builtin_isfinite(out[0])) __hip_atomic_fetch_or(a.flags, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        Philox4 rw = {0u, 0u, 0u, 0u};
        if constexpr (is_stochastic<ST>::value) rw = rounding_words(s, a.step, a.cc.box, a.cc.key0, a.cc.key1);
        void *dstp[Q + 1];
#pragma unroll
        for (int i = 0; i < Q + (S::rest_lo ? 1 : 0); ++i) dstp[i] = dst + (size_t)(P * z + (uint32_t)i) * plane;
        if constexpr (S::rest_lo) store_site<ST, TOTALS>(dstp, (uint32_t)plane, r, m_in, out, mass, mom, rw);
        else store_site16<ST, TOTALS>(dstp, (uint32_t)plane, r, m0, out, mass, mom, rw);
    }
    if (TOTALS) block_sum_totals(a.partials + 4 * (size_t)(blockIdx.x - (WAIT ? a.block0 : 0u)), mass, mom);
}

// The fused step kernel.  Occupancy is the compiler's own allocation: the
// thermal variants need 90-99 VGPRs (5 waves per SIMD); a cap at 80 (6 waves)
// makes it keep 16-20 bytes per lane in scratch memory, whose traffic (about
// 16 B per site, 10 % of the kernel's own) costs more than the extra wave
// gains.
// FULL (thermal only): the complete-relaxation collision (every
// non-conserved gamma_k = 0).
template <int ST, bool THERMAL, bool TOTALS, bool FORCE, bool WALLS, bool FULL>
__global__ void __launch_bounds__(1024) k_stream_collide(StepArgs a)
{
    stream_collide_site<ST, THERMAL, TOTALS, FORCE, WALLS, FULL>(a);
}

}  // namespace lbmi
