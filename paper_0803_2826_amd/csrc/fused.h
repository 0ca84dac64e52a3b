// Fused coupled time step of liblbmi (Sec. "Force coupling" with the fluid
// step of eq. LBE): the particle half of a coupled step and the fluid step
// that applies its force in ONE launch, for runs of several coupled steps
// with the same beads (lb_coupled_steps).
//
// The separate launches of a coupled step (k_bead_half, k_bead_update, then
// the step kernel) are each bound by a few dependent memory round trips,
// not by bandwidth: at 128^3 they add about 12 us to a 59 us step.  Here
//   - each bead sums the forces of its own bonds (its partners in a padded
//     table, bond-list order), so the bond pass and its accumulator go away;
//     for a bead with at most two bonds the sum has the same bits as the
//     separate launches' (0 + f1 + f2 in either order);
//   - the grid's first blocks are particle blocks: one lane per bead and
//     stencil node as in k_bead_update (phi_2, phi_3 or phi_4), reading the bead state of the step
//     from (pos_in, mom_in) and writing the next one to (pos, mom), distinct
//     arrays, so that a bead can read its partners' start state while they
//     are being updated; each block is counted in *arrive once its spread
//     atomics are performed;
//   - the site blocks run the step; a site whose bit is set in this step's
//     bitmap waits for the count before it takes its force (the particle
//     blocks are dispatched first and wait for nothing; the wait is bounded,
//     see wait_arrivals);
//   - the bitmap of a step is known before its launch: the stencil nodes of
//     R' = R + (h/2) P/m, which the previous launch's particle blocks (or
//     k_bead_nodes for the first step) mark from the state they write.
// The bead arithmetic is that of k_bead_half / k_bead_update term by term,
// so a fused run gives the same bits as the separate launches.
#pragma once

#include "bead_adjoint.h"
#include "couple.h"

namespace lbmi {

struct ParticleArgs {
    const void *pop;        // populations the step starts from (the step's source buffer)
    Geom geo;
    double rho0;
    double g[3];
    double kT;
    uint32_t key0, key1, box, step;
    int32_t n;
    const double *pos_in;   // bead state at the start of the step (not written by the launch)
    const double *mom_in;
    double *pos;            // out: state after the step (distinct from pos_in, mom_in)
    double *mom;
    const double *mass;
    const double *zeta;
    const double *fext;     // [n][3] or NULL
    const int32_t *partner; // [n][deg]: the beads bonded to each bead, bond-list order, -1 padded
    int32_t deg;
    int32_t fene;           // 1: FENE bonds, 0: harmonic
    int32_t three_point;    // bead noise: 1 the three-point variates, 0 unit Gaussians
    double kb, r0;
    int32_t *flags;         // bit 1: a FENE bond at r >= r0; bit 2: a refused spread contribution
    long long *force;       // [3][N] fixed-point force field (zero on entry outside nothing)
    uint32_t *fmask_next;   // bitmap of the next step's stencil nodes (zero on entry), or NULL
    double *half;           // [n][3] out: R'
    double *fc;             // [n][3] out: F^c
    // tape of the step (all NULL when not taping), as for k_bead_update
    double *tape_mom0;
    double *tape_momn;
    long long *tape_contrib;
    uint32_t *arrive;       // count of finished particle blocks
    // WCA pairs (the PAIRS kernels): three cell lists rotate over the steps
    // of a run; the launch of a step reads the list of its own R' (built by
    // the previous launch or k_bead_nodes), puts the heads of the previous
    // step's list back to -1, and builds the next step's list from the
    // positions it writes, so that no launch writes a list it reads
    CellGrid cg;
    const int32_t *head;           // this step's list
    const int32_t *next;
    const int32_t *cell_of;
    int32_t *head_reset;           // the previous step's list, or NULL
    const int32_t *cell_of_reset;
    int32_t *head_build;           // the next step's list, or NULL
    int32_t *next_build;
    int32_t *cell_of_build;
};

// Lanes per bead of the fused particle blocks: the stencil's, and at least
// kPairLanes with WCA pairs (one neighbour cell per lane, as k_wca).
template <int W, bool PAIRS>
struct FusedLanes {
    static constexpr int value =
        PAIRS && StencilLanes<W>::value < kPairLanes ? kPairLanes : StencilLanes<W>::value;
};

// R' = R + (h/2) P/m of bead j from the launch's start state (the expression
// of half_coord).
__device__ __forceinline__ double start_half(const ParticleArgs &a, int j, int c)
{
    return a.pos_in[3 * j + c] + 0.5 * a.mom_in[3 * j + c] / a.mass[j];
}

// Force on a bead at R'_b from its bond to bead j: mag (R'_b - R'_j) with
// mag = -k (r - r0)/r (harmonic) or -k/(1 - r^2/r0^2) (FENE, eq. ufene; NaN
// at r >= r0, latched as bit 1), added to f.  bond_force forms the same
// difference with the opposite sign for one end of the bond; the negation is
// exact, so both give the same bits.
__device__ __forceinline__ void partner_force(const ParticleArgs &a, const double Rb[3], int j, double f[3])
{
    double d[3], r2 = 0.0;
    for (int c = 0; c < 3; ++c) {
        d[c] = Rb[c] - start_half(a, j, c);
        r2 += d[c] * d[c];
    }
    double mag;
    if (a.fene) {
        const double x = r2 / (a.r0 * a.r0);
        if (x < 1.0) {
            mag = -a.kb / (1.0 - x);
        } else {
            mag = __builtin_nan("");
            __hip_atomic_fetch_or(a.flags, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    } else {
        const double r = sqrt(r2);
        if (r == 0.0) return;
        mag = -a.kb * (r - a.r0) / r;
    }
    for (int c = 0; c < 3; ++c) f[c] += mag * d[c];
}

// Marks the stencil nodes of R' = R + (h/2) P/m of every bead (nonzero
// weights) in `fmask`: the bitmap of the first step of a fused run; with
// head != NULL also links every bead at R' into that (empty) cell list.
template <int W>
__global__ void k_bead_nodes(const double *pos, const double *mom, const double *mass, int n, Geom g, uint32_t *fmask,
                             CellGrid cg, int32_t *head, int32_t *next, int32_t *cell_of)
{
    constexpr int LANES = StencilLanes<W>::value;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = t / LANES, q = t % LANES;
    if (b >= n || q >= W * W * W) return;
    double R[3];
    for (int c = 0; c < 3; ++c) R[c] = pos[3 * b + c] + 0.5 * mom[3 * b + c] / mass[b];
    uint32_t node;
    double w;
    stencil_node<W>(R, q, g, node, w, nullptr);
    if (w != 0.0) atomicOr(&fmask[node >> 5], 1u << (node & 31u));
    if (head && q == 0) cell_link(b, R, cg, cell_of, head, next);
}

// Puts the heads of a cell list back to -1 (each bead its own cell).
__global__ void k_cell_unlink(const int32_t *__restrict__ cell_of, int n, int32_t *head)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < n) head[cell_of[b]] = -1;
}

// The particle half of one coupled step, lane t = (bead, stencil node): the
// work of k_bead_half and k_bead_update for that lane (see couple.h), with
// the bead's bond forces summed over its partners.  Every thread of the
// block calls it; the block is counted in *arrive when its spread is done.
template <int ST, int W, bool PAIRS>
__device__ __forceinline__ void particle_block(const ParticleArgs &a)
{
    using S = Storage<ST>;
    using T = typename S::T;
    constexpr int LANES = FusedLanes<W, PAIRS>::value;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = t / LANES, q = t % LANES;
    const bool live = b < a.n;
    const Geom &g = a.geo;
    double ub[3] = {0.0, 0.0, 0.0}, fb[3] = {0.0, 0.0, 0.0}, fp[3] = {0.0, 0.0, 0.0};
    uint32_t node = 0;
    double wq = 0.0;
    double m = 1.0, z = 0.0, P[3] = {0.0, 0.0, 0.0}, R[3] = {0.0, 0.0, 0.0};
    const double h = 1.0;
    if (live) {
        m = a.mass[b];
        z = a.zeta[b];
        for (int c = 0; c < 3; ++c) {
            P[c] = a.mom_in[3 * b + c];
            R[c] = start_half(a, b, c);
        }
        if constexpr (PAIRS) {
            // WCA pairs (before the gather, whose values would otherwise be
            // live across the cell walks): lane q visits neighbour cell q of
            // the bead's cell, its members in increasing index (the terms
            // and order of k_wca)
            if (q < kPairLanes) {
                const CellGrid &cg = a.cg;
                const int nbc = lane_cell(a.cell_of[b], q, cg);
                for_members_in_order(nbc, b, a.n, a.head, a.next, [&](int j) {
                    const double d0 = pair_sep(R[0] - start_half(a, j, 0), cg.L[0], cg.periodic[0]);
                    const double d1 = pair_sep(R[1] - start_half(a, j, 1), cg.L[1], cg.periodic[1]);
                    const double d2 = pair_sep(R[2] - start_half(a, j, 2), cg.L[2], cg.periodic[2]);
                    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                    if (!(r2 < cg.rc2)) return;
                    const double s2 = cg.sig2 / r2;
                    const double s6 = s2 * s2 * s2;
                    const double f = cg.eps24 * (2.0 * s6 * s6 - s6) / r2;
                    fp[0] += f * d0;
                    fp[1] += f * d1;
                    fp[2] += f * d2;
                });
            }
        }
        stencil_node<W>(R, q, g, node, wq, nullptr);
        if (q < W * W * W) {
            // the node's populations, summed as soon as they arrive (the
            // launch's site blocks hold most of the registers)
            uint32_t xx, yy, zz;
            const PullOffsets o = pull_offsets(node, g, xx, yy, zz);
            const T *pop = static_cast<const T *>(a.pop);
            float v[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) v[i] = S::ld(pop[pull_index(node, o, i, zz, g)], 0.f);
            double ms = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const double vi = (double)v[i];
                ms += vi;
                j[0] += vi * kCX[i];
                j[1] += vi * kCY[i];
                j[2] += vi * kCZ[i];
            }
            const double rho = a.rho0 + ms;
            for (int c = 0; c < 3; ++c) ub[c] = wq * (j[c] + 0.5 * a.g[c]) / rho;
        }
        // the bead's bonds: lane q takes partners q, q + LANES, ...
        for (int k = q; k < a.deg; k += LANES) {
            const int j = a.partner[(size_t)b * a.deg + k];
            if (j >= 0) partner_force(a, R, j, fb);
        }
    }
    double C1 = 1.0, C2 = h, C3 = 0.0;
    if (z > 0.0) {
        C1 = exp(-z * h / m);
        C2 = (m / z) * (1.0 - C1);
        C3 = sqrt(m * a.kT * (1.0 - C1 * C1));
    }
    double th[3] = {0.0, 0.0, 0.0};
    if (live && a.kT > 0.0 && z > 0.0) {
        if (a.three_point)
            bead_three_point((uint32_t)b, a.step, a.box, a.key0, a.key1, th);
        else
            bead_normals((uint32_t)b, a.step, a.box, a.key0, a.key1, th);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        ub[c] = bead_sum<LANES>(ub[c]);
        fb[c] = bead_sum<LANES>(fb[c]);
        if constexpr (PAIRS) fp[c] = bead_sum<LANES>(fp[c]);
    }
    double Pn[3] = {0.0, 0.0, 0.0}, Fc[3] = {0.0, 0.0, 0.0};
    long long iv[3] = {0, 0, 0};
    if (live) {
        double I[3];
        for (int c = 0; c < 3; ++c) {
            // F^c = (bonds + pairs) + fext
            Fc[c] = fb[c];
            if constexpr (PAIRS) Fc[c] += fp[c];
            if (a.fext) Fc[c] += a.fext[3 * b + c];
            Pn[c] = C1 * P[c] + C2 * (Fc[c] + z * ub[c]) + C3 * th[c];
            I[c] = -(Pn[c] - P[c] - h * Fc[c]);
        }
        if (wq != 0.0) {
            for (int c = 0; c < 3; ++c) {
                const double fq = wq * I[c] / h;
                if (fabs(fq) < kForceLimit) {  // false for NaN too
                    iv[c] = __double2ll_rn(fq * kForceScale);
                    atomicAdd(reinterpret_cast<unsigned long long *>(&a.force[(size_t)c * g.N + node]),
                              (unsigned long long)iv[c]);
                } else {
                    __hip_atomic_fetch_or(a.flags, 4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
    }
    // every wave waits for its own spread atomics to be acknowledged, then
    // one release fence per block (an L2 writeback: one per wave instead
    // costs the site blocks of the launch about 4 us per step at 128^3)
    // precedes the count; the site blocks take the force only after it
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(a.arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!live) return;
    // the tape keeps one entry per bead and stencil lane (StencilLanes<W>,
    // the layout of k_bead_update's record), whatever the lanes per bead here
    constexpr int SL = StencilLanes<W>::value;
    if (a.tape_contrib && q < SL) {
        long long *e = a.tape_contrib + 4 * ((size_t)b * SL + q);
        e[0] = wq != 0.0 ? (long long)node : -1ll;
        e[1] = iv[0];
        e[2] = iv[1];
        e[3] = iv[2];
    }
    double Rn[3];
    for (int c = 0; c < 3; ++c) Rn[c] = R[c] + 0.5 * h * Pn[c] / m;
    if (q == 0)
        for (int c = 0; c < 3; ++c) {
            a.mom[3 * b + c] = Pn[c];
            a.pos[3 * b + c] = Rn[c];
            a.half[3 * b + c] = R[c];
            a.fc[3 * b + c] = Fc[c];
            if (a.tape_mom0) a.tape_mom0[3 * b + c] = P[c];
            if (a.tape_momn) a.tape_momn[3 * b + c] = Pn[c];
        }
    // the next step's stencil nodes (and cell list), from the state just
    // written (the next launch forms R' from it with the same expression)
    if (a.fmask_next && q < W * W * W) {
        double Rh[3];
        for (int c = 0; c < 3; ++c) Rh[c] = Rn[c] + 0.5 * Pn[c] / m;
        uint32_t nn;
        double wn;
        stencil_node<W>(Rh, q, g, nn, wn, nullptr);
        if (wn != 0.0) atomicOr(&a.fmask_next[nn >> 5], 1u << (nn & 31u));
        if constexpr (PAIRS)
            if (q == 0 && a.head_build) cell_link(b, Rh, a.cg, a.cell_of_build, a.head_build, a.next_build);
    }
    if constexpr (PAIRS)
        if (q == 0 && a.head_reset) a.head_reset[a.cell_of_reset[b]] = -1;
}

// One fused coupled step: blocks [0, a.block0) are the particle half
// (particle_block), the rest the fluid step with the bead force
// (stream_collide_site in WAIT mode; with MOM it also writes the input
// state's moments, a step of a moments tape).  blockDim a multiple of 64;
// a.block0 a multiple of 8 so that the site blocks keep their XCD mapping.
template <int ST, bool THERMAL, bool TOTALS, bool FULL, int W, bool PAIRS = false, bool MOM = false>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(5))) k_coupled_step(StepArgs a, ParticleArgs p)
{
    if (blockIdx.x < a.block0) {
        particle_block<ST, W, PAIRS>(p);
        return;
    }
    stream_collide_site<ST, THERMAL, TOTALS, true, false, FULL, true, MOM>(a);
}

// Recompute sweep of the reverse pass over taped steps: the fluid step (the
// sites of grid blocks [0, site_blocks)), with FORCE the bead force of its
// own field, with MOM
// writing the input state's moments for the adjoint step, and, in the grid's last
// blocks, the spread force of the next taped coupled step put back from its
// recorded contributions into the other field (k_respread's work; the
// fields alternate by step parity, so the two never touch the same field in
// one launch).  site_blocks is the step's own grid (no XCD remapping: the
// tile of block b is b).
template <int ST, bool THERMAL, bool WALLS, bool FULL, bool FORCE, bool MOM>
__global__ void __launch_bounds__(1024) k_recompute_step(StepArgs a, uint32_t site_blocks, const long long *contrib,
                                                         int entries, long long *force_next, uint32_t *fmask_next)
{
    if (blockIdx.x >= site_blocks) {
        const int e = (int)((blockIdx.x - site_blocks) * blockDim.x + threadIdx.x);
        if (e < entries) respread_entry(contrib, e, a.geo.N, force_next, fmask_next);
        return;
    }
    stream_collide_site<ST, THERMAL, false, FORCE, WALLS, FULL, false, MOM>(a);
}

}  // namespace lbmi
