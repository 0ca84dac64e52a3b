// Device-side counter-based random numbers for the fluctuating collision and
// the Langevin bead update (gfx950).
//
// Generator: Philox4x32-10 of Salmon, Moraes, Dror & Shaw (SC'11), written
// here from that publication.  Counter layout and the mapping to Gaussians
// are this library's own fixed convention (the paper only asks for
// independent zero-mean, unit-variance Gaussian variates, eq. stochupdaterule1
// and eq. langevin_momentum_update):
//   key     = (seed low word, seed high word)
//   fluid   : counter (site, step, call, box), call = 0, 1, 2
//   beads   : counter (bead, step, 1 << 16, box)
// Gaussians come from Box-Muller on 24-bit uniforms, radius uniform in (0,1],
// angle uniform in [0,1).  The transcendental steps use the hardware
// approximations (log2, sqrt, and sin/cos taking the angle in revolutions).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmi {

struct Philox4 {
    uint32_t v0, v1, v2, v3;
};

// a ^ b ^ c in one instruction (gfx950's three-input bitwise operation; the
// truth-table byte of XOR3 is 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                 uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Philox4{c0, c1, c2, c3};
}

// -2 ln(2): turns log2 into -2 ln for the Box-Muller radius.
#define LBMI_M2LN2 (-1.38629436111989061883f)

// Box-Muller radius times sqrt(scale): sqrt(-2 ln(ua) * scale), with the
// factor -2 ln 2 * scale (log2 -> ln) passed in as m2ln2_scale.
__device__ __forceinline__ float bm_radius(uint32_t field24, float m2ln2_scale)
{
    // ua = (field24 + 1) 2^-24 in (0, 1], exact: one fused multiply-add of
    // the exact conversion (the sum is a multiple of 2^-24 below 2^0)
    const float ua = __builtin_fmaf((float)field24, 0x1p-24f, 0x1p-24f);
    return __builtin_amdgcn_sqrtf(m2ln2_scale * __builtin_amdgcn_logf(ua));
}

__device__ __forceinline__ void box_muller(uint32_t fa, uint32_t fb, float m2ln2_scale, float &g0, float &g1)
{
    const float r = bm_radius(fa, m2ln2_scale);
    const float ub = (float)fb * 0x1p-24f;  // [0, 1), revolutions
    g0 = r * __builtin_amdgcn_cosf(ub);
    g1 = r * __builtin_amdgcn_sinf(ub);
}

// Fifteen Gaussians g[0..14] for modes 4..18 at (site, step, box), each
// multiplied by sqrt(scale).  Three Philox calls give words w[0..11]; each
// group of three words (a, b, c) yields 24-bit fields a>>8, b>>8, c>>8 and
// (a&255)|(b&255)<<8|(c&255)<<16; fields (2p, 2p+1) feed Box-Muller pair p.
__device__ __forceinline__ void fluid_normals(uint32_t site, uint32_t step, uint32_t box, uint32_t k0, uint32_t k1,
                                              float scale, float g[15])
{
    const float c = LBMI_M2LN2 * scale;
    const Philox4 A = philox4x32_10(site, step, 0u, box, k0, k1);
    const Philox4 B = philox4x32_10(site, step, 1u, box, k0, k1);
    const Philox4 C = philox4x32_10(site, step, 2u, box, k0, k1);
    const uint32_t w[12] = {A.v0, A.v1, A.v2, A.v3, B.v0, B.v1, B.v2, B.v3, C.v0, C.v1, C.v2, C.v3};
    uint32_t f[16];
#pragma unroll
    for (int grp = 0; grp < 4; ++grp) {
        const uint32_t wa = w[3 * grp], wb = w[3 * grp + 1], wc = w[3 * grp + 2];
        f[4 * grp + 0] = wa >> 8;
        f[4 * grp + 1] = wb >> 8;
        f[4 * grp + 2] = wc >> 8;
        // (wa & 255) | (wb & 255) << 8 | (wc & 255) << 16 with two byte
        // permutes (selector byte 0x0c gives a zero byte)
        const uint32_t ab = __builtin_amdgcn_perm(wb, wa, 0x0c0c0400u);
        f[4 * grp + 3] = __builtin_amdgcn_perm(wc, ab, 0x0c040100u);
    }
#pragma unroll
    for (int p = 0; p < 7; ++p) box_muller(f[2 * p], f[2 * p + 1], c, g[2 * p], g[2 * p + 1]);
    // last pair: only the cosine output is used
    g[14] = bm_radius(f[14], c) * __builtin_amdgcn_cosf((float)f[15] * 0x1p-24f);
}

// Three Gaussians for the Langevin noise of one bead (double precision
// transcendentals; the bead update is not on the bandwidth-critical path).
__device__ __forceinline__ void bead_normals(uint32_t bead, uint32_t step, uint32_t box, uint32_t k0, uint32_t k1,
                                             double g[3])
{
    const Philox4 A = philox4x32_10(bead, step, 1u << 16, box, k0, k1);
    const double two_pi = 6.283185307179586476925286766559;
    const double ua0 = ((double)(A.v0 >> 8) + 1.0) * 0x1p-24, ub0 = (double)(A.v1 >> 8) * 0x1p-24;
    const double ua1 = ((double)(A.v2 >> 8) + 1.0) * 0x1p-24, ub1 = (double)(A.v3 >> 8) * 0x1p-24;
    const double r0 = sqrt(-2.0 * log(ua0)), r1 = sqrt(-2.0 * log(ua1));
    g[0] = r0 * cos(two_pi * ub0);
    g[1] = r0 * sin(two_pi * ub0);
    g[2] = r1 * cos(two_pi * ub1);
}

// Three finite-range variates for the Langevin noise of one bead (Sec.
// "Force coupling", the three-point distribution given after eq.
// langevin_momentum_update): the same Philox call as bead_normals; word a
// falls in the sixth k = floor(6 w / 2^32) of the 32-bit range, k = 0 gives
// -sqrt(3), k = 5 gives +sqrt(3), the four middle sixths give 0.
__device__ __forceinline__ void bead_three_point(uint32_t bead, uint32_t step, uint32_t box, uint32_t k0,
                                                 uint32_t k1, double g[3])
{
    const Philox4 A = philox4x32_10(bead, step, 1u << 16, box, k0, k1);
    const double r3 = 1.7320508075688772;  // the double nearest sqrt(3)
    const uint32_t w[3] = {A.v0, A.v1, A.v2};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const uint32_t k = __umulhi(w[a], 6u);
        g[a] = (k == 0u) ? -r3 : (k == 5u) ? r3 : 0.0;
    }
}

}  // namespace lbmi
