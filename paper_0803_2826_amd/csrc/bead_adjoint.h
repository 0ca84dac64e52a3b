// Differentiation form, particle half: adjoint (reverse mode) of one
// coupled step's bead kernels (k_bead_half with its bond forces, k_bead_update of
// couple.h; Sec. "Force coupling", Sec. "Interpolating functions").
//
// The forward map of the particle half, per bead (h = 1):
//   R' = R + (h/2) P/m                      half drift (eq. pTrotter)
//   F^c = F^c(R')                           bonds (harmonic or FENE), WCA pairs, fext
//   u_b = sum_q w_q(R') u_q,  u_q = (sum_i n_i c_i + g/2) / rho_q   (eq. ufluid_discrete)
//   P'' = C1 P + C2 (F^c + zeta u_b) + C3 theta   (eq. langevin_momentum_update)
//   I = -(P'' - P - h F^c),  f(node_q) += w_q I / h                  (eq. ftotal)
//   R_new = R' + (h/2) P''/m,  P_new = P''
// Given the adjoints of (R_new, P_new) and fbar, the adjoint of the spread
// force at every node (written by the FORCE variant of k_adjoint_step), the
// kernels below produce the adjoints of (R, P), add the interpolation's
// contribution w_q (c_i - u_q).ubar_b / rho_q to lambda_i at the bead's stencil
// nodes and w_q ubar_b / (2 rho_q) to gbar.  The stencil weights are
// differentiated with the kernels' derivatives (phi_2 where R' is off the
// node planes).  The bead noise is not needed: P'' is taken from the
// forward update's tape; the external bead force is constant.
#pragma once

#include "couple.h"

namespace lbmi {

struct BeadAdjArgs {
    const void *pop;        // state buffer A of the step (pre-collision n_t(r) = A_i(r - c_i))
    const float *moments;   // or NULL; else the step's (rho - rho0, j) per site, [z][4][y][x] (pop unused)
    Geom geo;
    double rho0;
    double g[3];
    int32_t n;
    const double *mom0;     // P at the start of the step [n][3]
    const double *mom1;     // P'' of the forward update [n][3]
    const double *mass;
    const double *zeta;
    const double *half;     // R' [n][3]
    const double *fc;       // F^c at R' [n][3]
    const float *fbar;      // [3][N] adjoint of the spread force
    const double *pos_bar;  // adjoint of R_new [n][3]
    const double *mom_bar;  // adjoint of P_new [n][3]
    double *half_bar;       // out: adjoint of R' without the bond term [n][3]
    double *fc_bar;         // out: adjoint of F^c [n][3]
    double *p_bar;          // out: adjoint of P without the half-drift term [n][3]
    float *lam;             // adjoint of n_t (lam_index layout), accumulated at the nodes
    double *gbar;           // [3] accumulated
    // fold = 1: the adjoint of (R_new, P_new) is formed here, per bead, from
    // the later coupled step's half_bar and p_bar as they stand on entry
    // (R_new bar = R'bar, P_new bar = pbar + R'bar h / (2m), m = fold_mass)
    // instead of being read from pos_bar, mom_bar; that step's WCA cell
    // heads (fold_cell_head, NULL if none) are put back to -1 on the way
    int32_t fold;
    const double *fold_mass;
    int32_t *fold_cell_head;
    const int32_t *fold_cell_of;
};

// StencilLanes<W> lanes per bead, one per stencil node (node order and
// weights as in k_bead_update).
template <int ST, int W>
__global__ void __launch_bounds__(256) k_bead_adjoint(BeadAdjArgs a)
{
    using S = Storage<ST>;
    using T = typename S::T;
    constexpr int LANES = StencilLanes<W>::value;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = t / LANES, q = t % LANES;
    const bool live = b < a.n;
    const Geom &g = a.geo;
    const double h = 1.0;
    uint32_t node = 0;
    double wq = 0.0, dw[3] = {0.0, 0.0, 0.0}, uq[3] = {0.0, 0.0, 0.0}, rho = 1.0, fb[3] = {0.0, 0.0, 0.0};
    // the bead's own inputs are loaded, and the OU constants formed, while
    // the node values are in flight (lanes past the last bead keep zeros and
    // take part in the shuffles below)
    double Rnb[3] = {0.0, 0.0, 0.0}, Pnb_in[3] = {0.0, 0.0, 0.0}, I[3] = {0.0, 0.0, 0.0};
    double m = 1.0, z = 0.0, C1 = 1.0, C2 = h;
    if (live) {
        const double R[3] = {a.half[3 * b], a.half[3 * b + 1], a.half[3 * b + 2]};
        // adjoint of the state after the step (the same expressions as
        // k_bead_adjoint_finish when folded); every lane of the bead reads it
        // before its first lane writes this step's half_bar and p_bar below
        if (a.fold) {
            const double hm = 0.5 / a.fold_mass[b];
            for (int c = 0; c < 3; ++c) {
                Rnb[c] = a.half_bar[3 * b + c];
                Pnb_in[c] = a.p_bar[3 * b + c] + hm * Rnb[c];
            }
            if (q == 0 && a.fold_cell_head) a.fold_cell_head[a.fold_cell_of[b]] = -1;
        } else {
            for (int c = 0; c < 3; ++c) {
                Rnb[c] = a.pos_bar[3 * b + c];
                Pnb_in[c] = a.mom_bar[3 * b + c];
            }
        }
        m = a.mass[b];
        z = a.zeta[b];
        for (int c = 0; c < 3; ++c) I[c] = -(a.mom1[3 * b + c] - a.mom0[3 * b + c] - h * a.fc[3 * b + c]);
        stencil_node<W>(R, q, g, node, wq, dw);
        if (q < W * W * W) {
            double ms = 0.0, j[3] = {0.0, 0.0, 0.0};
            if (a.moments) {
                const uint32_t nxny = g.nxny, zn = node / nxny, rn = node - zn * nxny;
                const float *mp = a.moments + (size_t)(4u * zn) * nxny + rn;
                ms = (double)mp[0];
                j[0] = (double)mp[nxny];
                j[1] = (double)mp[2 * (size_t)nxny];
                j[2] = (double)mp[3 * (size_t)nxny];
            } else {
                uint32_t xx, yy, zz;
                const PullOffsets o = pull_offsets(node, g, xx, yy, zz);
                const T *pop = static_cast<const T *>(a.pop);
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const double v = (double)S::ld(pop[pull_index(node, o, i, zz, g)], 0.f);
                    ms += v;
                    j[0] += v * kCX[i];
                    j[1] += v * kCY[i];
                    j[2] += v * kCZ[i];
                }
            }
            for (int c = 0; c < 3; ++c) fb[c] = (double)a.fbar[(size_t)c * g.N + node];
            rho = a.rho0 + ms;
            for (int c = 0; c < 3; ++c) uq[c] = (j[c] + 0.5 * a.g[c]) / rho;
        }
        if (z > 0.0) {
            C1 = exp(-z * h / m);
            C2 = (m / z) * (1.0 - C1);
        }
    }
    // adjoint of the spread reaction: Ibar = sum_q w_q fbar(node_q) / h
    double Ib[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) Ib[c] = bead_sum<LANES>(wq * fb[c]) / h;
    double Pnb[3], ubb[3], pb[3], fcb[3];
    for (int c = 0; c < 3; ++c) {
        // R_new = R' + (h/2) P''/m, P_new = P'';  I = -(P'' - P - h F^c)
        Pnb[c] = Pnb_in[c] + 0.5 * h / m * Rnb[c] - Ib[c];
        pb[c] = Ib[c] + C1 * Pnb[c];
        fcb[c] = h * Ib[c] + C2 * Pnb[c];
        ubb[c] = C2 * z * Pnb[c];
    }
    // weights: from the spread (I . fbar / h) and from the interpolation (ubar . u_q)
    double wb = 0.0, gq[3];
    for (int c = 0; c < 3; ++c) {
        wb += I[c] * fb[c] / h + ubb[c] * uq[c];
        gq[c] = 0.5 * wq * ubb[c] / rho;
    }
    // u_q = (sum n c + g/2) / rho: lambda_i(node) += w_q (c_i - u_q) . ubar / rho
    if (live && wq != 0.0) {
        const uint32_t node_z = fdiv(fdiv(node, g.div_nx), g.div_ny);  // lambda is z-major (lam_index)
        const double s0 = -(uq[0] * ubb[0] + uq[1] * ubb[1] + uq[2] * ubb[2]);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double v = wq * (s0 + kCX[i] * ubb[0] + kCY[i] * ubb[1] + kCZ[i] * ubb[2]) / rho;
            atomicAdd(&a.lam[lam_index(i, node, node_z, g)], (float)v);
        }
    }
    double hb[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        hb[c] = bead_sum<LANES>(wb * dw[c]);
        // dL/dg: the bead's sum (on every lane of the bead), then the beads
        // of the wave (lanes of equal q), one atomic per wave
        double v = bead_sum<LANES>(gq[c]);
#pragma unroll
        for (int off = LANES; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
        gq[c] = v;
    }
    if (live && q == 0) {
        for (int c = 0; c < 3; ++c) {
            a.half_bar[3 * b + c] = Rnb[c] + hb[c];
            a.fc_bar[3 * b + c] = fcb[c];
            a.p_bar[3 * b + c] = pb[c];
        }
    }
    if ((threadIdx.x & 63u) == 0)
        for (int c = 0; c < 3; ++c) atomicAdd(&a.gbar[c], gq[c]);
}

// Bond forces F_b = mag d, F_a = -mag d (d = R'_b - R'_a) have the
// symmetric Jacobian dF_b/dd = mag I + 2 mag'(r^2) d d^T with
//   harmonic  mag = -k (r - r0)/r,        2 mag' = -k r0 / r^3
//   FENE      mag = -k / (1 - r^2/r0^2),  2 mag' = -2 k / (r0^2 (1 - r^2/r0^2)^2)
// so dbar = (dF_b/dd)(fcbar_b - fcbar_a), half_bar_b += dbar, half_bar_a -= dbar.
__device__ __forceinline__ void bond_adjoint(const double *__restrict__ half, const double *__restrict__ fc_bar,
                                             double *half_bar, const int32_t *__restrict__ bonds, int qd, double kb,
                                             double r0, int nbeads, int fene)
{
    const int ia = bonds[2 * qd], ib = bonds[2 * qd + 1];
    if (ia < 0 || ib < 0 || ia >= nbeads || ib >= nbeads) return;
    double d[3], v[3], r2 = 0.0, dv = 0.0;
    for (int c = 0; c < 3; ++c) {
        d[c] = half[3 * ib + c] - half[3 * ia + c];
        v[c] = fc_bar[3 * ib + c] - fc_bar[3 * ia + c];
        r2 += d[c] * d[c];
        dv += d[c] * v[c];
    }
    double mag, mag2p;
    if (fene) {
        const double x = r2 / (r0 * r0);
        mag = -kb / (1.0 - x);
        mag2p = -2.0 * kb / (r0 * r0 * (1.0 - x) * (1.0 - x));
    } else {
        const double r = sqrt(r2);
        if (r == 0.0) return;
        mag = -kb * (r - r0) / r;
        mag2p = -kb * r0 / (r2 * r);
    }
    for (int c = 0; c < 3; ++c) {
        const double db = mag * v[c] + mag2p * d[c] * dv;
        atomicAdd(&half_bar[3 * ib + c], db);
        atomicAdd(&half_bar[3 * ia + c], -db);
    }
}

__global__ void k_bonds_adjoint(const double *__restrict__ half, const double *__restrict__ fc_bar, double *half_bar,
                                const int32_t *__restrict__ bonds, int nbonds, double kb, double r0, int nbeads,
                                int fene)
{
    const int qd = blockIdx.x * blockDim.x + threadIdx.x;
    if (qd < nbonds) bond_adjoint(half, fc_bar, half_bar, bonds, qd, kb, r0, nbeads, fene);
}

// R' = R + (h/2) P/m:  Rbar = R'bar,  Pbar = pbar + (h/2m) R'bar.  Threads
// below the number of tape entries also zero the spread force's adjoint at
// the nodes of the step's contributions (every bead has read it by now),
// leaving fbar zero for the next coupled step of the sweep.
// With a WCA cell list (cell_head not NULL) each bead also puts its cell's
// head back to -1.
__global__ void k_bead_adjoint_finish(int n, const double *__restrict__ mass, const double *__restrict__ half_bar,
                                      const double *__restrict__ p_bar, double *pos_bar, double *mom_bar, float *fbar,
                                      const long long *contrib, int entries, uint32_t N, int32_t *cell_head,
                                      const int32_t *__restrict__ cell_of)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < entries) {
        const long long node = contrib[4 * (size_t)b];
        if (node >= 0)
            for (int c = 0; c < 3; ++c) fbar[(size_t)c * N + (size_t)node] = 0.f;
    }
    if (b >= n) return;
    if (cell_head) cell_head[cell_of[b]] = -1;
    const double hm = 0.5 / mass[b];
    for (int c = 0; c < 3; ++c) {
        pos_bar[3 * b + c] = half_bar[3 * b + c];
        mom_bar[3 * b + c] = p_bar[3 * b + c] + hm * half_bar[3 * b + c];
    }
}

// Backward sweeps: put a taped coupled step's spread force back from the
// contributions k_bead_update recorded (one entry per bead and lane).  The
// sums are integer, so the field gets the forward's bits in any order; the
// bitmap bits are set as the forward set them.
__device__ __forceinline__ void respread_entry(const long long *__restrict__ contrib, int e, uint32_t N,
                                               long long *force, uint32_t *fmask)
{
    const long long *p = contrib + 4 * (size_t)e;
    const long long node = p[0];
    if (node < 0) return;
    for (int c = 0; c < 3; ++c)
        if (p[1 + c] != 0)
            atomicAdd(reinterpret_cast<unsigned long long *>(&force[(size_t)c * N + (size_t)node]),
                      (unsigned long long)p[1 + c]);
    atomicOr(&fmask[(uint32_t)node >> 5], 1u << ((uint32_t)node & 31u));
}

__global__ void k_respread(const long long *__restrict__ contrib, int entries, uint32_t N, long long *force,
                           uint32_t *fmask)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < entries) respread_entry(contrib, e, N, force, fmask);
}

// Small jobs of the reverse sweep that run as extra blocks of the adjoint
// step kernel (nothing in that kernel reads what they touch): put the next
// (earlier) coupled step's force back into its own field, the bond
// Jacobians of the coupled step whose particle adjoint ran last (its F^c
// adjoint is complete), and the clearing of that step's fbar at its nodes.
// A count of zero skips a job.
struct AdjSide {
    const long long *put_contrib;  // k_respread of the next step
    int put_entries;
    long long *put_force;
    uint32_t *put_fmask;
    const double *half;            // bond Jacobians of the pending step
    const double *fc_bar;
    double *half_bar;
    const int32_t *bonds;
    int nbonds, nbeads, fene;
    double kb, r0;
    float *clear_fbar;             // fbar of the pending step, cleared at its nodes
    const long long *clear_contrib;
    int clear_entries;
};

__device__ __forceinline__ void adjoint_side_work(const AdjSide &s, int e, uint32_t N)
{
    if (e < s.put_entries) respread_entry(s.put_contrib, e, N, s.put_force, s.put_fmask);
    if (e < s.nbonds) bond_adjoint(s.half, s.fc_bar, s.half_bar, s.bonds, e, s.kb, s.r0, s.nbeads, s.fene);
    if (e < s.clear_entries) {
        const long long node = s.clear_contrib[4 * (size_t)e];
        if (node >= 0)
            for (int c = 0; c < 3; ++c) s.clear_fbar[(size_t)c * N + (size_t)node] = 0.f;
    }
}

}  // namespace lbmi
