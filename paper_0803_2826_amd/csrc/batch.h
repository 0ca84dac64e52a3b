// Batched form: many independent periodic replica boxes of uneven size
// advanced by ONE persistent launch per time step, replayable as a HIP graph.
//
// Layout: all boxes share two population buffers; box b owns the element
// range [off_b, off_b + P N_b) of each ([P][N_b] structure of arrays, P = 20
// with the rest residual plane of FP32 storage, else 19).
// Work list: the sites of each box are cut into tiles of blockDim sites; the
// tile -> box table is built on the host.  Each block walks a contiguous chunk
// of tiles (one tile per block when the launch search finds that faster).
//
// The step counter that keys the noise lives in device memory and is advanced
// by a one-thread kernel after each step, so a captured sequence of launches
// can be replayed unchanged.
//
// Ensemble velocity autocorrelation (sampled every step, pre-collision
// momentum j = sum_i n_i c_i, formed after the collision as the stored
// state's momentum less the force, which the collision adds to the
// conserved j exactly): for each box and each axis a, the lowest
// Fourier mode k = 2 pi / L_a of the two momentum components transverse to
// a, j_hat(k) = sum_r j(r) exp(-i k r_a) (6 complex amplitudes per box).
// Every tile writes its 12 partial sums to a row of its own (no atomics);
// k_vacf_update adds a box's rows in a fixed order, so the amplitudes, like
// the populations, do not depend on the order in which blocks run.  A ring
// buffer of the last R samples per box gives
// C_b(tau) += sum_modes Re[j_hat(t) conj(j_hat(t - tau))].  At gamma = 0 its
// mean is N_b kT rho0 lambda(k)^tau, lambda = 1 - (2/3) sin^2(k/2)
// (linear dynamics of eq. LBE with the equipartition of eq. Pdistneq).
#pragma once

#include "kernels.h"

namespace lbmi {

struct BoxDesc {
    Geom geo;
    uint64_t off;         // element offset of this box's [P][N_b] block
    uint32_t box_id;      // fourth Philox counter word
    uint32_t first_tile;  // index of the box's first tile in the work list
    float inv_L[3];       // 1 / L_x, 1 / L_y, 1 / L_z
    uint32_t pad;
};

struct BatchArgs {
    const void *src;
    void *dst;
    const BoxDesc *boxes;
    const uint32_t *tile_box;  // [ntiles] box index of each tile
    uint32_t ntiles;
    uint32_t chunk;            // tiles per block (contiguous)
    CollideConst cc;           // `box` is replaced per tile
    const uint32_t *step_ptr;  // device step counter
    float *amp;                // [ntiles][12] VACF partial sums of each tile (re, im of 6 modes)
    int32_t *flags;
};

// Sum of x over the 64 lanes of a wave, complete in lane 63 (every lane of
// the wave must be active): an inclusive scan within each row of 16 lanes
// (DPP row shifts by 1, 2, 4 and 8), then the row totals carried up by the
// row broadcasts (lane 15 into rows 1 and 3, lane 31 into rows 2 and 3).
// A lane with no source in a shift, or outside the row mask, adds 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float add_dpp(float v)
{
    const int u = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xf, false);
    return v + __builtin_bit_cast(float, u);
}
__device__ __forceinline__ float wave_sum_lane63(float x)
{
    x = add_dpp<0x111, 0xf>(x);  // row_shr:1
    x = add_dpp<0x112, 0xf>(x);  // row_shr:2
    x = add_dpp<0x114, 0xf>(x);  // row_shr:4
    x = add_dpp<0x118, 0xf>(x);  // row_shr:8
    x = add_dpp<0x142, 0xa>(x);  // row_bcast:15
    x = add_dpp<0x143, 0xc>(x);  // row_bcast:31
    return x;
}

// Block-wide sum of 12 floats into dst[0..11] (fixed order).  Every thread
// of the block must call it (it synchronises).
__device__ __forceinline__ void tile_sum12(float acc[12], float *dst)
{
    __shared__ float red[16][12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = wave_sum_lane63(acc[c]);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 63)
#pragma unroll
        for (int c = 0; c < 12; ++c) red[wid][c] = acc[c];
    __syncthreads();
    if (threadIdx.x < 12) {
        const int nw = (blockDim.x + 63) >> 6;
        float s = 0.f;
        for (int w = 0; w < nw; ++w) s += red[w][threadIdx.x];
        dst[threadIdx.x] = s;
    }
}

// FULL: the complete-relaxation collision (every non-conserved gamma_k = 0).
// Its variants are held to 80 registers (6 waves per SIMD), which they fit
// without scratch; the general-relaxation ones keep the compiler's choice.
template <int ST, bool THERMAL, bool VACF, bool FULL>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(FULL ? 6 : 1))) k_batch_step(BatchArgs a)
{
    using S = Storage<ST>;
    using T = typename S::T;
    const uint32_t step = *a.step_ptr;
    const uint32_t t_begin = blockIdx.x * a.chunk;
    const uint32_t t_end = min(t_begin + a.chunk, a.ntiles);
    CollideConst cc = a.cc;
    for (uint32_t t = t_begin; t < t_end; ++t) {
        const uint32_t box = a.tile_box[t];
        // this site's terms of the tile's 12 VACF sums, formed after the
        // store so that they hold no registers across the collision
        float acc[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = 0.f;
        const BoxDesc d = a.boxes[box];
        const uint32_t s = (t - d.first_tile) * blockDim.x + threadIdx.x;
        if (s < d.geo.N) {
            uint32_t x, y, z;
            const PullOffsets o = pull_offsets(s, d.geo, x, y, z);
            const T *__restrict__ src = static_cast<const T *>(a.src) + d.off;
            T *__restrict__ dst = static_cast<T *>(a.dst) + d.off;
            const uint32_t N = d.geo.N;
            float dd[Q];
    #pragma unroll
            for (int i = 0; i < Q; ++i) dd[i] = S::ld(ld_plane(src + (size_t)i * N, pull_src(s, o, i)), 0.f);
            float lo_in = 0.f;
            if constexpr (S::rest_lo) lo_in = ld_plane(src + (size_t)kRestLo * N, s);
            mass_acc_t<ST> m_in = 0;
            if constexpr (S::rest_lo) m_in = site_mass_lo<ST>(dd, lo_in);
            cc.box = d.box_id;
            float out[Q], m0;
            collide_site<THERMAL, FULL, out_scale<ST>::value, ST == 1>(dd, cc.g, cc, s, step, out, m0);
            if (!__builtin_isfinite(out[0])) __hip_atomic_fetch_or(a.flags, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            void *dstp[Q + 1];
    #pragma unroll
            for (int i = 0; i < Q + (S::rest_lo ? 1 : 0); ++i) dstp[i] = dst + (size_t)i * N;
            double mass;
            float mom[3];
            Philox4 rw = {0u, 0u, 0u, 0u};
            if constexpr (is_stochastic<ST>::value) rw = rounding_words(s, step, d.box_id, cc.key0, cc.key1);
            // with VACF the store also returns the stored values' momentum
            if constexpr (S::rest_lo) store_site<ST, VACF>(dstp, N * (uint32_t)sizeof(T), s, m_in, out, mass, mom, rw);
            else store_site16<ST, VACF>(dstp, N * (uint32_t)sizeof(T), s, m0, out, mass, mom, rw);
            if (VACF) {
                // the sampled momentum j = sum_i c_i n_i before the
                // collision: the collision keeps j and adds the force
                // (m*_k = m_k + g_k, k = 1..3), so j is the stored state's
                // momentum less g, up to the storage rounding
                const float jx = mom[0] - cc.g[0], jy = mom[1] - cc.g[1], jz = mom[2] - cc.g[2];
                // the site's coordinates again (cheaper than keeping them)
                const uint32_t q = fdiv(s, d.geo.div_nx);
                const uint32_t zq = fdiv(q, d.geo.div_ny);
                float fx = (float)(s - q * d.geo.nx) * d.inv_L[0];
                float fy = (float)(q - zq * d.geo.ny) * d.inv_L[1];
                float fz = (float)zq * d.inv_L[2];
                // the phases pass through an empty asm that also takes a
                // collision output, which keeps the compiler from forming
                // the six Fourier factors before the collision (where they
                // would hold registers across it)
                __asm__ volatile("" : "+v"(fx), "+v"(fy), "+v"(fz) : "v"(out[0]));
                const float cx = __builtin_amdgcn_cosf(fx), sx = __builtin_amdgcn_sinf(fx);
                const float cy = __builtin_amdgcn_cosf(fy), sy = __builtin_amdgcn_sinf(fy);
                const float cz = __builtin_amdgcn_cosf(fz), sz = __builtin_amdgcn_sinf(fz);
                // exp(-i phi) = cos - i sin
                acc[0] = jx * cz;  acc[1] = -(jx * sz);   // k along z, j_x
                acc[2] = jy * cz;  acc[3] = -(jy * sz);   // k along z, j_y
                acc[4] = jx * cy;  acc[5] = -(jx * sy);   // k along y, j_x
                acc[6] = jz * cy;  acc[7] = -(jz * sy);   // k along y, j_z
                acc[8] = jy * cx;  acc[9] = -(jy * sx);   // k along x, j_y
                acc[10] = jz * cx; acc[11] = -(jz * sx);  // k along x, j_z
            }
        }
        if (VACF) tile_sum12(acc, a.amp + 12 * (size_t)t);  // block-uniform: every thread takes part
    }
}

// Sum this step's tile rows of each box into its 12 amplitudes (FP64, fixed
// order), push them into the ring, accumulate C_b(tau).  One block per box,
// blockDim >= max(R, 64); `block` is the step kernel's tile size.
__global__ void __launch_bounds__(1024) k_vacf_update(const float *__restrict__ rows, const BoxDesc *__restrict__ boxes,
                                                      uint32_t block, float *ring, double *corr, int R,
                                                      const uint32_t *nsamp_ptr)
{
    const int b = blockIdx.x;
    const BoxDesc d = boxes[b];
    const uint32_t nt = (d.geo.N + block - 1u) / block;
    const float *rb = rows + 12 * (size_t)d.first_tile;
    double acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = 0.0;
    for (uint32_t r = threadIdx.x; r < nt; r += blockDim.x)
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] += (double)rb[12 * (size_t)r + c];
    __shared__ double red[16][12];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        double x = acc[c];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        acc[c] = x;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < 12; ++c) red[wid][c] = acc[c];
    __syncthreads();
    const uint32_t ns = *nsamp_ptr;  // samples taken before this one
    const int slot = (int)(ns % (uint32_t)R);
    float *ringb = ring + (size_t)b * R * 12;
    __shared__ float cur[12];
    if (threadIdx.x < 12) {
        const int nw = (blockDim.x + 63) >> 6;
        double v = 0.0;
        for (int w = 0; w < nw; ++w) v += red[w][threadIdx.x];
        cur[threadIdx.x] = (float)v;
        ringb[slot * 12 + threadIdx.x] = (float)v;
    }
    __syncthreads();
    const int tau = threadIdx.x;
    if (tau < R && (uint32_t)tau <= ns) {
        const float *old = ringb + ((slot - tau + R) % R) * 12;
        double sum = 0.0;
        for (int m = 0; m < 6; ++m)
            sum += (double)cur[2 * m] * old[2 * m] + (double)cur[2 * m + 1] * old[2 * m + 1];
        corr[(size_t)b * R + tau] += sum;
    }
}

// Advance the device step counter (and the VACF sample count).
__global__ void k_advance(uint32_t *step_ptr, uint32_t *nsamp_ptr, int sampled)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        step_ptr[0] += 1u;
        if (sampled) nsamp_ptr[0] += 1u;
    }
}

__global__ void k_set_u32(uint32_t *p, uint32_t v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = v;
}

}  // namespace lbmi
