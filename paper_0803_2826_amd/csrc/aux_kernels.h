// State conversion, diagnostics and reduction kernels of liblbmi.
#pragma once

#include "kernels.h"

namespace lbmi {

__device__ __forceinline__ double weight_of(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

// Push offset: site r + c_i (inverse of the pull map).
__device__ __forceinline__ uint32_t push_dst(uint32_t x, uint32_t y, uint32_t z, const Geom &g, int i)
{
    const int32_t cx = kCX[i], cy = kCY[i], cz = kCZ[i];
    const uint32_t xx = (uint32_t)((int32_t)x + cx + (int32_t)g.nx) % g.nx;
    const uint32_t yy = (uint32_t)((int32_t)y + cy + (int32_t)g.ny) % g.ny;
    const uint32_t zz = (uint32_t)((int32_t)z + cz + (int32_t)g.nz) % g.nz;
    return xx + g.nx * (yy + g.ny * zz);
}

__device__ __forceinline__ void site_xyz(uint32_t s, const Geom &g, uint32_t &x, uint32_t &y, uint32_t &z)
{
    const uint32_t q = fdiv(s, g.div_nx);
    x = s - q * g.nx;
    z = fdiv(q, g.div_ny);
    y = q - z * g.ny;
}

// Store the deviation v of population i at site s; the rest population of
// FP32 storage keeps its FP64 value as hi + lo (the residual plane, see
// store_site).
template <int ST>
__device__ __forceinline__ void store_pop(typename Storage<ST>::T *b, int i, uint32_t s, uint32_t z, const Geom &g,
                                          double v)
{
    using S = Storage<ST>;
    const typename S::T h = S::st((float)v, 0.f);
    b[pop_index(i, s, z, g)] = h;
    if constexpr (S::rest_lo)
        if (i == 0) b[pop_index(kRestLo, s, z, g)] = (float)(v - (double)S::ld(h, 0.f));
}

// Stored value of the rest population at site s as FP64 (hi + lo for FP32
// storage).
template <int ST>
__device__ __forceinline__ double load_rest(const typename Storage<ST>::T *b, uint32_t s, uint32_t z, const Geom &g)
{
    using S = Storage<ST>;
    double v = (double)S::ld(b[pop_index(0, s, z, g)], 0.f);
    if constexpr (S::rest_lo) v += (double)b[pop_index(kRestLo, s, z, g)];
    return v;
}

// Buffer A_i(r) = S_i(r + c_i) with S = n^eq(rho, u) of eq. original_equil_distrib,
// shifted by a_i rho0.
template <int ST>
__global__ void k_init_equilibrium(void *buf, Geom g, double rho0, const double *__restrict__ rho,
                                   const double *__restrict__ u)
{
    using S = Storage<ST>;
    using T = typename S::T;
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.N) return;
    uint32_t x, y, z;
    site_xyz(s, g, x, y, z);
    T *b = static_cast<T *>(buf);
    for (int i = 0; i < Q; ++i) {
        // the reader of A_i(s): population i at s + c_i, or opp(i) at s across a wall
        const bool wall = push_crosses(g, z, i);
        const int j = wall ? opp(i) : i;
        const uint32_t r = wall ? s : push_dst(x, y, z, g, i);
        const double rr = rho ? rho[r] : rho0;
        double ux = 0.0, uy = 0.0, uz = 0.0;
        if (u) {
            ux = u[r];
            uy = u[(size_t)g.N + r];
            uz = u[2 * (size_t)g.N + r];
        }
        const double uc = ux * kCX[j] + uy * kCY[j] + uz * kCZ[j];
        const double usq = ux * ux + uy * uy + uz * uz;
        const double a = weight_of(j);
        const double neq = a * rr * (1.0 + 3.0 * uc + 4.5 * uc * uc - 1.5 * usq);
        store_pop<ST>(b, i, s, z, g, neq - a * rho0);
    }
}

// Set: A_i(r) = src_i(r + c_i) (src_opp(i)(r) across a wall); src is F64 or
// F32, shifted or not.
template <int ST, typename TIn>
__global__ void k_set_pops(void *buf, Geom g, double rho0, const TIn *__restrict__ src, int shifted)
{
    using S = Storage<ST>;
    using T = typename S::T;
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.N) return;
    uint32_t x, y, z;
    site_xyz(s, g, x, y, z);
    T *b = static_cast<T *>(buf);
    for (int i = 0; i < Q; ++i) {
        const bool wall = push_crosses(g, z, i);
        const int j = wall ? opp(i) : i;
        const uint32_t r = wall ? s : push_dst(x, y, z, g, i);
        double v = (double)src[(size_t)j * g.N + r];
        if (!shifted) v -= weight_of(j) * rho0;
        store_pop<ST>(b, i, s, z, g, v);
    }
}

// Get: dst_i(r) = A_i(r - c_i) (A_opp(i)(r) across a wall).
template <int ST, typename TOut>
__global__ void k_get_pops(const void *buf, Geom g, double rho0, TOut *__restrict__ dst, int shifted)
{
    using S = Storage<ST>;
    using T = typename S::T;
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.N) return;
    uint32_t x, y, z;
    const PullOffsets o = pull_offsets(s, g, x, y, z);
    const T *b = static_cast<const T *>(buf);
    for (int i = 0; i < Q; ++i) {
        double v = i == 0 ? load_rest<ST>(b, s, z, g) : (double)S::ld(b[pull_index(s, o, i, z, g)], 0.f);
        if (!shifted) v += weight_of(i) * rho0;
        dst[(size_t)i * g.N + s] = (TOut)v;
    }
}

// rho and u = (sum n c + g/2)/rho of the pre-collision state, FP64.
template <int ST>
__global__ void k_moments(const void *buf, Geom g, double rho0, double gx, double gy, double gz,
                          double *__restrict__ rho_out, double *__restrict__ u_out)
{
    using S = Storage<ST>;
    using T = typename S::T;
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.N) return;
    uint32_t x, y, z;
    const PullOffsets o = pull_offsets(s, g, x, y, z);
    const T *b = static_cast<const T *>(buf);
    double m = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    for (int i = 0; i < Q; ++i) {
        const double v = i == 0 ? load_rest<ST>(b, s, z, g) : (double)S::ld(b[pull_index(s, o, i, z, g)], 0.f);
        m += v;
        jx += v * kCX[i];
        jy += v * kCY[i];
        jz += v * kCZ[i];
    }
    const double r = rho0 + m;
    if (rho_out) rho_out[s] = r;
    if (u_out) {
        u_out[s] = (jx + 0.5 * gx) / r;
        u_out[(size_t)g.N + s] = (jy + 0.5 * gy) / r;
        u_out[2 * (size_t)g.N + s] = (jz + 0.5 * gz) / r;
    }
}

// Block-wide FP64 sum of NV values into out[blockIdx][NV].
template <int NV>
__device__ __forceinline__ void block_sum_f64(double *out, double v[NV])
{
    __shared__ double red[16][NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        double x = v[c];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        v[c] = x;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < NV; ++c) red[wid][c] = v[c];
    __syncthreads();
    const int nw = (blockDim.x + 63) >> 6;
    for (int c = threadIdx.x; c < NV; c += blockDim.x) {
        double sacc = 0.0;
        for (int w = 0; w < nw; ++w) sacc += red[w][c];
        out[c] = sacc;
    }
}

// Exact totals of the stored state (streaming is a permutation, so the
// totals of A equal those of the pre-collision state).  Sum of deviations.
template <int ST>
__global__ void __launch_bounds__(256) k_totals_exact(const void *buf, Geom g, double *partials)
{
    using S = Storage<ST>;
    using T = typename S::T;
    const T *b = static_cast<const T *>(buf);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < g.N; s += gridDim.x * blockDim.x) {
        const uint32_t z = fdiv(fdiv(s, g.div_nx), g.div_ny);
        for (int i = 0; i < Q; ++i) {
            const double v = i == 0 ? load_rest<ST>(b, s, z, g) : (double)S::ld(b[pop_index(i, s, z, g)], 0.f);
            acc[0] += v;
            acc[1] += v * kCX[i];
            acc[2] += v * kCY[i];
            acc[3] += v * kCZ[i];
        }
    }
    block_sum_f64<4>(partials + 4 * (size_t)blockIdx.x, acc);
}

// Positivity scan of the stored state (the low-Mach guard: the quadratic
// equilibrium of Sec. "D3Q19 model I" turns negative once u is no longer
// small against the lattice speeds, and thermal noise can push populations
// below zero where a_i rho0 is small): per block, the number of sites with
// a population n_i = a_i rho0 + d_i < 0 and the smallest n_i, into
// partials[block] = {count, min}.  Grid-stride over the sites.
template <int ST>
__global__ void __launch_bounds__(256) k_negative_scan(const void *buf, Geom g, double rho0, double *partials)
{
    using S = Storage<ST>;
    using T = typename S::T;
    const T *b = static_cast<const T *>(buf);
    double cnt = 0.0, mn = __builtin_inf();
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < g.N; s += gridDim.x * blockDim.x) {
        // the populations of site s (pulled as in k_get_pops)
        uint32_t x, y, z;
        const PullOffsets o = pull_offsets(s, g, x, y, z);
        double site_min = __builtin_inf();
        for (int i = 0; i < Q; ++i) {
            const double d = i == 0 ? load_rest<ST>(b, s, z, g) : (double)S::ld(b[pull_index(s, o, i, z, g)], 0.f);
            site_min = fmin(site_min, weight_of(i) * rho0 + d);
        }
        if (site_min < 0.0) cnt += 1.0;
        mn = fmin(mn, site_min);
    }
    __shared__ double red[16][2];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        cnt += __shfl_xor(cnt, off, 64);
        mn = fmin(mn, __shfl_xor(mn, off, 64));
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        red[wid][0] = cnt;
        red[wid][1] = mn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double c = 0.0, m = __builtin_inf();
        for (int w = 0; w < (int)((blockDim.x + 63) >> 6); ++w) {
            c += red[w][0];
            m = fmin(m, red[w][1]);
        }
        partials[2 * (size_t)blockIdx.x] = c;
        partials[2 * (size_t)blockIdx.x + 1] = m;
    }
}

// Basis polynomial e_k(c) of Table 1 (integer valued).
__device__ __forceinline__ double basis_k(int k, int x, int y, int z)
{
    const int c2 = x * x + y * y + z * z;
    switch (k) {
    case 0: return 1;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return c2 - 1;
    case 5: return 3 * x * x - c2;
    case 6: return y * y - z * z;
    case 7: return x * y;
    case 8: return y * z;
    case 9: return z * x;
    case 10: return (3 * c2 - 5) * x;
    case 11: return (3 * c2 - 5) * y;
    case 12: return (3 * c2 - 5) * z;
    case 13: return (y * y - z * z) * x;
    case 14: return (z * z - x * x) * y;
    case 15: return (x * x - y * y) * z;
    case 16: return 3 * c2 * c2 - 6 * c2 + 1;
    case 17: return (2 * c2 - 3) * (3 * x * x - c2);
    default: return (2 * c2 - 3) * (y * y - z * z);
    }
}

// Per-block sums of m_k and m_k^2 of the pre-collision state (FP64),
// partials [gridDim][38].
template <int ST>
__global__ void __launch_bounds__(256) k_mode_stats(const void *buf, Geom g, double rho0, double *partials)
{
    using S = Storage<ST>;
    using T = typename S::T;
    const T *b = static_cast<const T *>(buf);
    double acc[38];
    for (int k = 0; k < 38; ++k) acc[k] = 0.0;
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < g.N; s += gridDim.x * blockDim.x) {
        uint32_t x, y, z;
        const PullOffsets o = pull_offsets(s, g, x, y, z);
        double n[Q];
        for (int i = 0; i < Q; ++i)
            n[i] = i == 0 ? load_rest<ST>(b, s, z, g) : (double)S::ld(b[pull_index(s, o, i, z, g)], 0.f);
        for (int k = 0; k < Q; ++k) {
            double m = (k == 0) ? rho0 : 0.0;
            for (int i = 0; i < Q; ++i) m += basis_k(k, kCX[i], kCY[i], kCZ[i]) * n[i];
            acc[k] += m;
            acc[19 + k] += m * m;
        }
    }
    block_sum_f64<38>(partials + 38 * (size_t)blockIdx.x, acc);
}

// Column sums of a [rows][ncols] FP64 array (deterministic order), one block
// per column, out[ncols]; add0 is added to column 0's sum (add0 + sum).
__global__ void __launch_bounds__(256) k_reduce_cols(const double *__restrict__ in, int rows, int ncols,
                                                     double *__restrict__ out, double add0)
{
    __shared__ double red[256];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int r = threadIdx.x; r < rows; r += blockDim.x) s += in[(size_t)r * ncols + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = c == 0 ? add0 + red[0] : red[0];
}

__global__ void k_noise_sample(uint32_t site0, uint32_t count, uint32_t step, CollideConst cc, float *out)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    float r[15];
    fluid_normals(site0 + t, step, cc.box, cc.key0, cc.key1, 1.0f, r);
    for (int k = 0; k < 15; ++k) out[(size_t)t * 15 + k] = r[k];
}

__global__ void k_zero_i32(int32_t *p, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t n, uint32_t v)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_zero_f32(float *p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.f;
}

}  // namespace lbmi
