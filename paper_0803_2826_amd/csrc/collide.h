// D3Q19 moment-space collision with thermal noise and forcing, FP32 math on
// shifted populations d_i = n_i - a_i rho0 (gfx950 device code).
//
// What is computed (per site), following Sec. "D3Q19 model II/III" and
// Sec. "External forces":
//   m_k = sum_i e_ki n_i with the Table 1 basis, evaluated through opposite
//     pair sums S_p = d_i + d_ibar and differences D_p = d_i - d_ibar (even
//     basis polynomials see only S_p, odd ones only D_p);
//   rho = rho0 + m_0(d), j = m_{1..3} + F/2 (eq. special_choice_momentum_density),
//     u = j / rho;
//   equilibrium moments of eq. original_equil_distrib projected on the basis:
//     m4 = j^2/rho, m5 = (2jx^2 - jy^2 - jz^2)/rho, m6 = (jy^2 - jz^2)/rho,
//     m7 = jx jy/rho, m8 = jy jz/rho, m9 = jz jx/rho, kinetic modes 0;
//   stress modes k = 4..9: m*_k = m^eq_k + gamma_k (m_k - m^eq_k)
//     + (1 + gamma_k)/2 S_k + sigma_k sqrt(rho_n) r_k, where S_k is the
//     projection of the force second moment of eq. moment_two_external_force
//     (S4 = 2u.F, S5 = 2(2uxFx - uyFy - uzFz), S6 = 2(uyFy - uzFz),
//      S7 = uxFy + uyFx, S8 = uyFz + uzFy, S9 = uzFx + uxFz);
//   kinetic modes k = 10..18: m*_k = gamma_k m_k + sigma_k sqrt(rho_n) r_k;
//   momentum modes: m*_{1..3} = m_{1..3} + F; mass mode unchanged;
//   sigma_k = sqrt(w_k mu (1 - gamma_k^2)), mu = 3 kT (eq. stochupdaterule1,
//     eq. detailedbalance1, eq. normalized_mk);
//   back-transformation n*_i = a_i sum_k e_ki m*_k / w_k (eq. back_transformation)
//     again through pair even/odd parts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rng.h"

namespace lbmi {

// Multiplication by the weights a = 1/3, 1/18, 1/36, none of which is exact
// in FP32: x * (hi + lo) with hi = fl(a), lo = fl(a - hi), so the product is
// rounded once from the (near) exact value instead of carrying the constant's
// own rounding error, which would bias every step the same way.
// OSC: the output is scaled by 2^OSC (exact), for storage types that keep a
// scaled value (FP16 stores 2^8 times the deviation).
// SPLIT = false (16-bit storage): one product with fl(a).  The constant's
// relative error (below 2^-24) is then 2^-17 of BF16's and 2^-14 of FP16's
// relative spacing, and the ALU-bound 16-bit kernels save an instruction
// per population.
template <int DEN, int OSC = 0, bool SPLIT = true>
__device__ __forceinline__ float mul_weight(float x)
{
    constexpr double a = (double)(1 << OSC) / (double)DEN;
    constexpr float hi = (float)a;
    constexpr float lo = (float)(a - (double)hi);
    if constexpr (SPLIT) return __builtin_fmaf(x, hi, x * lo);
    else return x * hi;
}

// Per-launch constants of the collision (kernel-argument resident).
struct CollideConst {
    float gam[19];   // gamma_k, modes 4..18 used
    float sig[19];   // sigma_k = sqrt(w_k mu (1 - gamma_k^2)), modes 4..18 used
    float sigw[19];  // sigma_k / w_k (the noise of a kinetic mode as it enters the back-transformation)
    float rho0;
    float sqrt_rho0;
    float g[3];      // uniform body force
    uint32_t key0, key1, box;
    int32_t noise_rho0;
};

// d[19]: shifted pre-collision populations (in), out[19]: shifted
// post-collision populations times 2^OSC, m0: the input's mass deviation
// sum_i d_i (the collision keeps it).  F: total force density at the site.
// FULL: every non-conserved gamma_k is 0 (complete relaxation, tau = 1 for
// the stress modes and the kinetic modes fully relaxed), so m*_k =
// m^eq_k + S_k/2 (+ noise) and the moments m_4..m_18 of the input are never
// needed; the result equals the general expressions at gamma = 0.
template <bool THERMAL, bool FULL = false, int OSC = 0, bool SPLIT = true>
__device__ __forceinline__ void collide_site(const float d[19], const float F[3], const CollideConst &cc,
                                             uint32_t site, uint32_t step, float out[19], float &m0)
{
    // ---- moments through opposite-pair sums/differences
    const float S1 = d[1] + d[2], D1 = d[1] - d[2];
    const float S2 = d[3] + d[4], D2 = d[3] - d[4];
    const float S3 = d[5] + d[6], D3 = d[5] - d[6];
    const float S4 = d[7] + d[8], D4 = d[7] - d[8];
    const float S5 = d[9] + d[10], D5 = d[9] - d[10];
    const float S6 = d[11] + d[12], D6 = d[11] - d[12];
    const float S7 = d[13] + d[14], D7 = d[13] - d[14];
    const float S8 = d[15] + d[16], D8 = d[15] - d[16];
    const float S9 = d[17] + d[18], D9 = d[17] - d[18];

    const float A1 = (S4 + S5) + (S6 + S7);  // diagonals with an x component
    const float A2 = S8 + S9;                // diagonals in the yz plane
    const float T2 = A1 + A2;
    const float R1 = (S1 + S2) + S3;
    const float B6 = (S4 + S5) - (S6 + S7);

    float m[19];
    m[0] = d[0] + R1 + T2;
    m[4] = T2 - d[0];
    m[16] = d[0] - 2.f * R1 + T2;
    m[5] = 2.f * S1 - (S2 + S3) + A1 - 2.f * A2;
    m[17] = -2.f * S1 + (S2 + S3) + A1 - 2.f * A2;
    m[6] = (S2 - S3) + B6;
    m[18] = (S3 - S2) + B6;
    m[7] = S4 - S5;
    m[8] = S8 - S9;
    m[9] = S6 - S7;
    const float X = (D4 + D5) + (D6 + D7);
    const float Y = (D4 - D5) + (D8 + D9);
    const float Z = (D6 - D7) + (D8 - D9);
    m[1] = D1 + X;
    m[10] = -2.f * D1 + X;
    m[2] = D2 + Y;
    m[11] = -2.f * D2 + Y;
    m[3] = D3 + Z;
    m[12] = -2.f * D3 + Z;
    m[13] = (D4 + D5) - (D6 + D7);
    m[14] = (D5 - D4) + (D8 + D9);
    m[15] = (D6 - D7) - (D8 - D9);

    m0 = m[0];

    // ---- hydrodynamic fields (1/rho from the hardware reciprocal, 1 ulp)
    const float rho = cc.rho0 + m[0];
    const float inv_rho = __builtin_amdgcn_rcpf(rho);
    const float jx = m[1] + 0.5f * F[0], jy = m[2] + 0.5f * F[1], jz = m[3] + 0.5f * F[2];
    const float ux = jx * inv_rho, uy = jy * inv_rho, uz = jz * inv_rho;

    float meq[10];
    meq[4] = (jx * ux + jy * uy) + jz * uz;
    meq[5] = 2.f * jx * ux - (jy * uy + jz * uz);
    meq[6] = jy * uy - jz * uz;
    meq[7] = jx * uy;
    meq[8] = jy * uz;
    meq[9] = jz * ux;

    float Sf[10];
    Sf[4] = 2.f * ((ux * F[0] + uy * F[1]) + uz * F[2]);
    Sf[5] = 2.f * (2.f * ux * F[0] - (uy * F[1] + uz * F[2]));
    Sf[6] = 2.f * (uy * F[1] - uz * F[2]);
    Sf[7] = ux * F[1] + uy * F[0];
    Sf[8] = uy * F[2] + uz * F[1];
    Sf[9] = uz * F[0] + ux * F[2];

    // ---- relaxation (+ noise)
    float ms[19];
    ms[0] = m[0];
    ms[1] = m[1] + F[0];
    ms[2] = m[2] + F[1];
    ms[3] = m[3] + F[2];
    if constexpr (FULL) {
#pragma unroll
        for (int k = 4; k <= 9; ++k) ms[k] = meq[k] + 0.5f * Sf[k];
#pragma unroll
        for (int k = 10; k <= 18; ++k) ms[k] = 0.f;
    } else {
#pragma unroll
        for (int k = 4; k <= 9; ++k)
            ms[k] = meq[k] + cc.gam[k] * (m[k] - meq[k]) + 0.5f * (1.f + cc.gam[k]) * Sf[k];
#pragma unroll
        for (int k = 10; k <= 18; ++k) ms[k] = cc.gam[k] * m[k];
    }

    float r[15];
    if (THERMAL) {
        // r_k sqrt(rho_n): the density factor of the amplitude rides on the
        // Box-Muller radius
        fluid_normals(site, step, cc.box, cc.key0, cc.key1, cc.noise_rho0 ? cc.rho0 : rho, r);
#pragma unroll
        for (int k = 4; k <= (FULL ? 9 : 18); ++k) ms[k] += cc.sig[k] * r[k - 4];
    }

    // ---- back-transformation: scale by 1/w_k, then pair even/odd parts
    const float u0 = ms[0];
    const float u1 = 3.f * ms[1], u2 = 3.f * ms[2], u3 = 3.f * ms[3];
    const float u4 = 1.5f * ms[4], u5 = 0.75f * ms[5], u6 = 2.25f * ms[6];
    const float u7 = 9.f * ms[7], u8 = 9.f * ms[8], u9 = 9.f * ms[9];
    float uk[19];
    if constexpr (FULL) {
        // fully relaxed kinetic modes carry only their noise: u_k = (sigma_k / w_k) r_k
#pragma unroll
        for (int k = 10; k <= 18; ++k) uk[k] = THERMAL ? cc.sigw[k] * r[k - 4] : 0.f;
    } else {
        const float inv_w[19] = {1.f, 3.f, 3.f, 3.f, 1.5f, 0.75f, 2.25f, 9.f, 9.f, 9.f,
                                 1.5f, 1.5f, 1.5f, 4.5f, 4.5f, 4.5f, 0.5f, 0.75f, 2.25f};
#pragma unroll
        for (int k = 10; k <= 18; ++k) uk[k] = inv_w[k] * ms[k];
    }
    const float u10 = uk[10], u11 = uk[11], u12 = uk[12];
    const float u13 = uk[13], u14 = uk[14], u15 = uk[15];
    const float u16 = uk[16], u17 = uk[17], u18 = uk[18];

    out[0] = mul_weight<3, OSC, SPLIT>((u0 - u4) + u16);

    // speed-1 pairs
    const float e1c = (u0 - 2.f * u16);  // common even part of the axis directions
    const float E1 = e1c + 2.f * u5 - 2.f * u17;
    const float E2 = e1c - u5 + u6 + u17 - u18;
    const float E3 = e1c - u5 - u6 + u17 + u18;
    const float O1 = u1 - 2.f * u10, O2 = u2 - 2.f * u11, O3 = u3 - 2.f * u12;
    out[1] = mul_weight<18, OSC, SPLIT>(E1 + O1);
    out[2] = mul_weight<18, OSC, SPLIT>(E1 - O1);
    out[3] = mul_weight<18, OSC, SPLIT>(E2 + O2);
    out[4] = mul_weight<18, OSC, SPLIT>(E2 - O2);
    out[5] = mul_weight<18, OSC, SPLIT>(E3 + O3);
    out[6] = mul_weight<18, OSC, SPLIT>(E3 - O3);

    // speed-sqrt2 pairs
    const float e2c = (u0 + u4) + u16;
    const float exy = e2c + u5 + u17 + (u6 + u18);  // (1,+-1,0)
    const float exz = e2c + u5 + u17 - (u6 + u18);  // (1,0,+-1)
    const float eyz = e2c - 2.f * (u5 + u17);        // (0,1,+-1)
    const float E4 = exy + u7, E5 = exy - u7;
    const float E6 = exz + u9, E7 = exz - u9;
    const float E8 = eyz + u8, E9 = eyz - u8;
    const float px = u1 + u10, py = u2 + u11, pz = u3 + u12;
    const float O4 = (px + py) + (u13 - u14);
    const float O5 = (px - py) + (u13 + u14);
    const float O6 = (px + pz) + (u15 - u13);
    const float O7 = (px - pz) - (u13 + u15);
    const float O8 = (py + pz) + (u14 - u15);
    const float O9 = (py - pz) + (u14 + u15);
    out[7] = mul_weight<36, OSC, SPLIT>(E4 + O4);
    out[8] = mul_weight<36, OSC, SPLIT>(E4 - O4);
    out[9] = mul_weight<36, OSC, SPLIT>(E5 + O5);
    out[10] = mul_weight<36, OSC, SPLIT>(E5 - O5);
    out[11] = mul_weight<36, OSC, SPLIT>(E6 + O6);
    out[12] = mul_weight<36, OSC, SPLIT>(E6 - O6);
    out[13] = mul_weight<36, OSC, SPLIT>(E7 + O7);
    out[14] = mul_weight<36, OSC, SPLIT>(E7 - O7);
    out[15] = mul_weight<36, OSC, SPLIT>(E8 + O8);
    out[16] = mul_weight<36, OSC, SPLIT>(E8 - O8);
    out[17] = mul_weight<36, OSC, SPLIT>(E9 + O9);
    out[18] = mul_weight<36, OSC, SPLIT>(E9 - O9);
}

}  // namespace lbmi
