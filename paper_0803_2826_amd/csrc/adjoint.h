// Differentiation form: adjoint (reverse mode) of the fused stream-collide
// step (gfx950 device code).
//
// Forward step (see collide.h): n*(r) = C(n(r), F) at every site, then
// n_i(r + c_i, t+1) = n*_i(r, t).  Given lambda(t+1) = dL/dn(t+1) (natural
// layout [19][N], pre-collision populations), the adjoint step computes
//   nbar*_i(r) = lambda_i(r + c_i, t+1)          (transpose of streaming)
//   lambda(r, t) = J_C(n(r, t), F)^T nbar*(r)     (transposed collision)
//   gbar += sum_r dC/dF^T nbar*(r)                (uniform body force)
// The transposed collision retraces the moment-space collision backwards:
//   msb_k = (1/w_k) sum_i a_i e_ki nbar*_i        (transpose of the back-transformation)
//   mb_k = gamma_k msb_k (k >= 4), msb_k (k < 4)
//   meq and the force moments S_k feed jbar, ubar, Fbar with weights
//     (1 - gamma_k) and (1 + gamma_k)/2;
//   local-density noise sigma_k sqrt(rho) r_k gives rhobar += msb_k sigma_k r_k / (2 sqrt rho),
//     with r_k replayed from the same Philox counters as the forward step;
//   u = j / rho, j = m_{1..3} + F/2, rho = rho0 + m_0;
//   lambda_i = sum_k e_ki mb_k                    (transpose of the moment map).
// The collision's Jacobian depends only on (rho, j) and the replayed noise,
// so the forward state needed is re-gathered from the stored step buffer.
#pragma once

#include "bead_adjoint.h"
#include "kernels.h"

namespace lbmi {

struct AdjArgs {
    const void *state;      // step buffer A_t (AB layout: pre-collision n_t(r) = A_t,i(r - c_i))
    const float *lam_in;    // lambda(t+1), z-major with 19 planes per layer (lam_index)
    float *lam_out;         // lambda(t), the state's layout
    Geom geo;
    CollideConst cc;
    uint32_t step;
    double *partials;       // [gridDim][3] block sums of Fbar, accumulated over the steps of a sweep
    // bead force of the step (FORCE variant): F = g + force at sites whose
    // bit is set in fmask; the adjoint of that force is written to fbar
    // there, and the force rows and bitmap words read are left zero (each
    // coupled step of the sweep puts its own force back first)
    long long *force;       // [3][N] fixed point (kForceScale)
    uint32_t *fmask;        // [ceil(N/32)]
    float *fbar;            // [3][N]
    // blocks are dealt out layer by layer as in the forward step: block b <
    // main_blocks = nz tiles works on layer b / tiles; blocks from
    // main_blocks on do the side jobs instead of sites
    uint32_t tiles;
    FastDiv div_tiles;
    uint32_t main_blocks;
    AdjSide side;
    // the state's moments (rho - rho0, j) per site, [z][4][y][x], written by
    // the recompute step that read this state (stream_collide_site MOM), or
    // NULL: then they are formed from the state itself (19 pulled values)
    const float *moments;
};


template <int ST, bool THERMAL, bool FORCE, bool WALLS>
__global__ void __launch_bounds__(256) k_adjoint_step(AdjArgs a)
{
    using S = Storage<ST>;
    using T = typename S::T;
    if (blockIdx.x >= a.main_blocks) {  // whole blocks: no barrier below is split
        adjoint_side_work(a.side, (int)((blockIdx.x - a.main_blocks) * blockDim.x + threadIdx.x), a.geo.N);
        return;
    }
    const uint32_t z = fdiv(blockIdx.x, a.div_tiles);
    const uint32_t nxny = a.geo.nxny;
    const uint32_t r = (blockIdx.x - z * a.tiles) * blockDim.x + threadIdx.x;
    const bool active = r < nxny;
    const uint32_t s = z * nxny + r;
    float Fbs[3] = {0.f, 0.f, 0.f};
    if (active) {
        uint32_t x, y, zs;
        const PullOffsets o = pull_offsets(s, a.geo, x, y, zs);
        PullOffsets oxy = o;  // in-layer part of each pull; the layer picks the plane base
        oxy.oz_m = 0;
        oxy.oz_p = 0;
        const uint32_t N = a.geo.N;
        const size_t plane = (size_t)nxny * sizeof(T);
        const uint32_t P = a.geo.planes;  // state planes per layer (lambda keeps 19)
        const char *st = static_cast<const char *>(a.state);
        // forward hydrodynamic fields of n(r, t): the only part of the state
        // the collision's Jacobian depends on
        float m0, jx, jy, jz;
        if (a.moments) {
            const float *mp = a.moments + (size_t)(4u * z) * nxny;
            m0 = ld_plane(mp, r);
            jx = ld_plane(mp + nxny, r);
            jy = ld_plane(mp + 2 * (size_t)nxny, r);
            jz = ld_plane(mp + 3 * (size_t)nxny, r);
        } else {
            float d[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                if (pull_crosses<WALLS>(a.geo, z, i))  // pull source beyond a wall: opp(i) of this site
                    d[i] = S::ld(ld_plane(reinterpret_cast<const T *>(st + (size_t)(P * z + (uint32_t)opp(i)) * plane),
                                          r),
                                 0.f);
                else
                    d[i] = S::ld(ld_plane(reinterpret_cast<const T *>(st + (size_t)(P * pull_z(z, i, a.geo) +
                                                                                    (uint32_t)i) *
                                                                               plane),
                                          pull_src(r, oxy, i)),
                                 0.f);
            }
            m0 = d[0];
            jx = 0.f;
            jy = 0.f;
            jz = 0.f;
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                m0 += d[i];
                jx += (float)kCX[i] * d[i];
                jy += (float)kCY[i] * d[i];
                jz += (float)kCZ[i] * d[i];
            }
        }
        float F[3] = {a.cc.g[0], a.cc.g[1], a.cc.g[2]};
        bool flagged = false;
        if (FORCE) {
            const uint32_t bit = 1u << (s & 31u);
            flagged = (a.fmask[s >> 5] & bit) != 0u;
            if (flagged) {
                F[0] += force_value(a.force[s]);
                F[1] += force_value(a.force[(size_t)N + s]);
                F[2] += force_value(a.force[2 * (size_t)N + s]);
                a.force[s] = 0;
                a.force[(size_t)N + s] = 0;
                a.force[2 * (size_t)N + s] = 0;
                atomicAnd(&a.fmask[s >> 5], ~bit);
            }
        }
        const float rho = a.cc.rho0 + m0;
        const float inv_rho = 1.0f / rho;
        jx += 0.5f * F[0];
        jy += 0.5f * F[1];
        jz += 0.5f * F[2];
        const float ux = jx * inv_rho, uy = jy * inv_rho, uz = jz * inv_rho;

        // nbar*_i(r) = lambda_i(r + c_i): r + c_i is the pull source of the opposite direction;
        // across a wall the reader of n*_i(r) is population opp(i) at r itself
        float q[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const size_t lplane = (size_t)nxny;
            const float lb = push_crosses<WALLS>(a.geo, z, i)
                                 ? ld_plane(a.lam_in + (size_t)(19u * z + (uint32_t)opp(i)) * lplane, r)
                                 : ld_plane(a.lam_in + (size_t)(19u * pull_z(z, opp(i), a.geo) + (uint32_t)i) * lplane,
                                            pull_src(r, oxy, opp(i)));
            q[i] = lb * (i == 0 ? (1.f / 3.f) : (i <= 6 ? (1.f / 18.f) : (1.f / 36.f)));
        }
        // msb_k = (1/w_k) sum_i e_ki (a_i nbar*_i): the moment map applied to q
        const float S1 = q[1] + q[2], D1 = q[1] - q[2];
        const float S2 = q[3] + q[4], D2 = q[3] - q[4];
        const float S3 = q[5] + q[6], D3 = q[5] - q[6];
        const float S4 = q[7] + q[8], D4 = q[7] - q[8];
        const float S5 = q[9] + q[10], D5 = q[9] - q[10];
        const float S6 = q[11] + q[12], D6 = q[11] - q[12];
        const float S7 = q[13] + q[14], D7 = q[13] - q[14];
        const float S8 = q[15] + q[16], D8 = q[15] - q[16];
        const float S9 = q[17] + q[18], D9 = q[17] - q[18];
        const float A1 = (S4 + S5) + (S6 + S7), A2 = S8 + S9, T2 = A1 + A2, R1 = (S1 + S2) + S3;
        const float B6 = (S4 + S5) - (S6 + S7);
        const float X = (D4 + D5) + (D6 + D7), Y = (D4 - D5) + (D8 + D9), Z = (D6 - D7) + (D8 - D9);
        float mb[Q];
        mb[0] = q[0] + R1 + T2;
        mb[1] = 3.f * (D1 + X);
        mb[2] = 3.f * (D2 + Y);
        mb[3] = 3.f * (D3 + Z);
        mb[4] = 1.5f * (T2 - q[0]);
        mb[5] = 0.75f * (2.f * S1 - (S2 + S3) + A1 - 2.f * A2);
        mb[6] = 2.25f * ((S2 - S3) + B6);
        mb[7] = 9.f * (S4 - S5);
        mb[8] = 9.f * (S8 - S9);
        mb[9] = 9.f * (S6 - S7);
        mb[10] = 1.5f * (-2.f * D1 + X);
        mb[11] = 1.5f * (-2.f * D2 + Y);
        mb[12] = 1.5f * (-2.f * D3 + Z);
        mb[13] = 4.5f * ((D4 + D5) - (D6 + D7));
        mb[14] = 4.5f * ((D5 - D4) + (D8 + D9));
        mb[15] = 4.5f * ((D6 - D7) - (D8 - D9));
        mb[16] = 0.5f * (q[0] - 2.f * R1 + T2);
        mb[17] = 0.75f * (-2.f * S1 + (S2 + S3) + A1 - 2.f * A2);
        mb[18] = 2.25f * ((S3 - S2) + B6);
        // mb now holds msb (adjoint of the post-collision moments)

        float rhob = 0.f;
        if (THERMAL && !a.cc.noise_rho0) {
            float gn[15];
            fluid_normals(s, a.step, a.cc.box, a.cc.key0, a.cc.key1, 1.0f, gn);
            const float h = 0.5f / __builtin_amdgcn_sqrtf(rho);
#pragma unroll
            for (int k = 4; k <= 18; ++k) rhob += mb[k] * a.cc.sig[k] * gn[k - 4];
            rhob *= h;
        }
        // momentum modes: ms_{1..3} = m_{1..3} + F
        Fbs[0] = mb[1];
        Fbs[1] = mb[2];
        Fbs[2] = mb[3];
        // stress modes: equilibrium (weight 1 - gamma) and force moments (weight (1 + gamma)/2).
        // Each meq_k is written as a product of j and u with u held separately
        // (m4 = j.u, m5 = 2 jx ux - jy uy - jz uz, m6 = jy uy - jz uz, m7 = jx uy,
        // m8 = jy uz, m9 = jz ux); the chain rule through u = j / rho follows.
        float e[10], f[10];
#pragma unroll
        for (int k = 4; k <= 9; ++k) {
            e[k] = (1.f - a.cc.gam[k]) * mb[k];
            f[k] = 0.5f * (1.f + a.cc.gam[k]) * mb[k];
        }
        float jbx = e[4] * ux + 2.f * e[5] * ux + e[7] * uy;
        float jby = e[4] * uy - e[5] * uy + e[6] * uy + e[8] * uz;
        float jbz = e[4] * uz - e[5] * uz - e[6] * uz + e[9] * ux;
        float ubx = e[4] * jx + 2.f * e[5] * jx + e[9] * jz;
        float uby = e[4] * jy - e[5] * jy + e[6] * jy + e[7] * jx;
        float ubz = e[4] * jz - e[5] * jz - e[6] * jz + e[8] * jy;
        ubx += 2.f * f[4] * F[0] + 4.f * f[5] * F[0] + f[7] * F[1] + f[9] * F[2];
        uby += 2.f * f[4] * F[1] - 2.f * f[5] * F[1] + 2.f * f[6] * F[1] + f[7] * F[0] + f[8] * F[2];
        ubz += 2.f * f[4] * F[2] - 2.f * f[5] * F[2] - 2.f * f[6] * F[2] + f[8] * F[1] + f[9] * F[0];
        Fbs[0] += 2.f * f[4] * ux + 4.f * f[5] * ux + f[7] * uy + f[9] * uz;
        Fbs[1] += 2.f * f[4] * uy - 2.f * f[5] * uy + 2.f * f[6] * uy + f[7] * ux + f[8] * uz;
        Fbs[2] += 2.f * f[4] * uz - 2.f * f[5] * uz - 2.f * f[6] * uz + f[8] * uy + f[9] * ux;
        // u = j / rho
        jbx += ubx * inv_rho;
        jby += uby * inv_rho;
        jbz += ubz * inv_rho;
        rhob -= (ubx * ux + uby * uy + ubz * uz) * inv_rho;
        // j = m_{1..3} + F/2, rho = rho0 + m_0
        Fbs[0] += 0.5f * jbx;
        Fbs[1] += 0.5f * jby;
        Fbs[2] += 0.5f * jbz;
        float mm[Q];
        mm[0] = mb[0] + rhob;
        mm[1] = mb[1] + jbx;
        mm[2] = mb[2] + jby;
        mm[3] = mb[3] + jbz;
#pragma unroll
        for (int k = 4; k < Q; ++k) mm[k] = a.cc.gam[k] * mb[k];
        // lambda_i = sum_k e_ki mm_k (transpose of the moment map, pair even/odd parts)
        const float u0 = mm[0], u1 = mm[1], u2 = mm[2], u3 = mm[3], u4 = mm[4], u5 = mm[5], u6 = mm[6];
        const float u7 = mm[7], u8 = mm[8], u9 = mm[9], u10 = mm[10], u11 = mm[11], u12 = mm[12];
        const float u13 = mm[13], u14 = mm[14], u15 = mm[15], u16 = mm[16], u17 = mm[17], u18 = mm[18];
        float out[Q];
        out[0] = (u0 - u4) + u16;
        const float e1c = u0 - 2.f * u16;
        const float E1 = e1c + 2.f * u5 - 2.f * u17, E2 = e1c - u5 + u6 + u17 - u18, E3 = e1c - u5 - u6 + u17 + u18;
        const float O1 = u1 - 2.f * u10, O2 = u2 - 2.f * u11, O3 = u3 - 2.f * u12;
        out[1] = E1 + O1;
        out[2] = E1 - O1;
        out[3] = E2 + O2;
        out[4] = E2 - O2;
        out[5] = E3 + O3;
        out[6] = E3 - O3;
        const float e2c = (u0 + u4) + u16;
        const float exy = e2c + u5 + u17 + (u6 + u18), exz = e2c + u5 + u17 - (u6 + u18), eyz = e2c - 2.f * (u5 + u17);
        const float E4 = exy + u7, E5 = exy - u7, E6 = exz + u9, E7 = exz - u9, E8 = eyz + u8, E9 = eyz - u8;
        const float px = u1 + u10, py = u2 + u11, pz = u3 + u12;
        const float O4 = (px + py) + (u13 - u14), O5 = (px - py) + (u13 + u14), O6 = (px + pz) + (u15 - u13);
        const float O7 = (px - pz) - (u13 + u15), O8 = (py + pz) + (u14 - u15), O9 = (py - pz) + (u14 + u15);
        out[7] = E4 + O4;
        out[8] = E4 - O4;
        out[9] = E5 + O5;
        out[10] = E5 - O5;
        out[11] = E6 + O6;
        out[12] = E6 - O6;
        out[13] = E7 + O7;
        out[14] = E7 - O7;
        out[15] = E8 + O8;
        out[16] = E8 - O8;
        out[17] = E9 + O9;
        out[18] = E9 - O9;
#pragma unroll
        for (int i = 0; i < Q; ++i)
            st_plane_nt<float>(a.lam_out + (size_t)(19u * z + (uint32_t)i) * nxny, nxny * 4u, r, out[i]);
        if (FORCE && flagged) {
            a.fbar[s] = Fbs[0];
            a.fbar[(size_t)N + s] = Fbs[1];
            a.fbar[2 * (size_t)N + s] = Fbs[2];
        }
    }
    // block sums of Fbar (FP64 partial per block)
    __shared__ double red[4][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float v = Fbs[c];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        Fbs[c] = v;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
        for (int c = 0; c < 3; ++c) red[wid][c] = (double)Fbs[c];
    __syncthreads();
    if (threadIdx.x < 3) {
        double sacc = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) sacc += red[w][threadIdx.x];
        a.partials[3 * (size_t)blockIdx.x + threadIdx.x] += sacc;
    }
}

// acc[c] += sum over rows of in[r][c] (one block per column, fixed order).
__global__ void __launch_bounds__(256) k_accumulate_cols(const double *__restrict__ in, int rows, int ncols, double *acc)
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
    if (threadIdx.x == 0) acc[c] += red[0];
}

// Conversions between the caller's [19][N] arrays and the FP32 adjoints
// (z-major, lam_index).
template <typename TIn>
__global__ void k_to_lam(const TIn *__restrict__ in, float *__restrict__ lam, Geom g)
{
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < g.N; s += gridDim.x * blockDim.x) {
        const uint32_t z = fdiv(fdiv(s, g.div_nx), g.div_ny);
        for (int i = 0; i < Q; ++i) lam[lam_index(i, s, z, g)] = (float)in[(size_t)i * g.N + s];
    }
}

template <typename TOut>
__global__ void k_from_lam(const float *__restrict__ lam, TOut *__restrict__ out, Geom g)
{
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < g.N; s += gridDim.x * blockDim.x) {
        const uint32_t z = fdiv(fdiv(s, g.div_nx), g.div_ny);
        for (int i = 0; i < Q; ++i) out[(size_t)i * g.N + s] = (TOut)lam[lam_index(i, s, z, g)];
    }
}

}  // namespace lbmi
