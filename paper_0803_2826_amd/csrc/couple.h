// Point-particle (bead) coupling kernels of liblbmi (Sec. "Force coupling",
// Sec. "Interpolating functions").  Bead state is FP64; the fluid velocity is
// gathered from the stored populations.
//
// One coupled step on the device:
//   k_bead_half     R' = R + (h/2) P/m; harmonic or FENE bond forces at R'
//                   (FP64 atomics into a zeroed accumulator: a bead with at
//                   most two bonds gets the same bits on every run); zero the
//                   other accumulator for the next call; when taping,
//                   copy the starting momenta P to the step's tape slot
//   k_cell_* k_wca  WCA pair forces at R' with a cell list (pairs.h), when on
//   k_bead_update   one lane per stencil node (W^3 of them, W = 2, 3, 4 for the
//                   kernels phi_2, phi_3, phi_4 of eq. 2point, eq. 3point,
//                   eq. 4point): each lane gathers its node's 19 populations
//                   and forms w u(node) with u = (sum n c + g/2)/rho and the
//                   product weight of eq. Delta; a lane reduction gives u_b;
//                   F^c = (bonds + pairs) + fext, kept for the adjoint;
//                   every lane then evaluates P'' = C1 P + C2 (F^c + zeta u_b)
//                   + C3 theta (eq. langevin_momentum_update) and spreads
//                   w I / h with I = -(P'' - P - h F^c) to its own node
//                   (eq. ftotal; fixed-point integer atomics, so the sum
//                   does not depend on the order; a non-finite or absurdly
//                   large contribution is refused and latched as bit 2 of the
//                   device flags), setting the node's bit in the force bitmap;
//                   R = R' + (h/2) P''/m; when taping, P'' and each lane's
//                   fixed-point contribution go to the step's tape slot
//   (next lb_step)  the fused stream-collide kernel adds the bead force at
//                   flagged sites and leaves those force rows and bitmap
//                   words zero.
#pragma once

#include "aux_kernels.h"
#include "pairs.h"

namespace lbmi {

struct CoupleArgs {
    const void *pop;      // current buffer A
    Geom geo;
    double rho0;
    double g[3];
    double kT;
    uint32_t key0, key1, box, step;
    int32_t n;
    const double *pos_in;  // bead state the step starts from (may equal pos / mom)
    const double *mom_in;
    double *pos;           // out: state after the step
    double *mom;
    const double *mass;
    const double *zeta;
    double *half;         // [n][3] out: R'
    double *fc;           // [n][3] out: the conservative force F^c at R' (bonds + pairs + fext)
    double *fb;           // [n][3] bond forces, accumulated here (zero on entry)
    double *fb_next;      // [cap][3] the other bond accumulator, zeroed here for the next call
    int32_t cap;          // entries of fb_next to zero
    const double *fp;     // [n][3] pair (WCA) forces at R' or NULL
    const double *fext;   // [n][3] external forces or NULL
    const int32_t *bonds; // [nbonds][2]
    int32_t nbonds;
    int32_t fene;         // 1: FENE bonds, 0: harmonic
    int32_t three_point;  // bead noise: 1 the three-point variates, 0 unit Gaussians
    double kb, r0;
    int32_t *flags;       // bit 1: a FENE bond at r >= r0
    long long *force;     // [3][N] sparse force field, fixed point (zero outside touched nodes)
    uint32_t *fmask;      // [ceil(N/32)] force bitmap
    // tape of a coupled step (all NULL when not taping): P at the start
    // [n][3], P'' [n][3] and the spread contributions, one entry of four
    // int64 per (bead, lane): node (or -1: nothing spread) and the three
    // fixed-point values added there
    double *tape_mom0;
    double *tape_momn;
    long long *tape_contrib;
    // WCA cell list (cell_head NULL: no pair force): k_bead_half links each
    // bead into its cell at R', k_bead_update puts the heads back to -1
    CellGrid cg;
    int32_t *cell_head;
    int32_t *cell_next;
    int32_t *cell_of;
};

// R' = R + (h/2) P/m of bead b, component c (one expression wherever R' is
// formed, so that every kernel sees the same bits).
__device__ __forceinline__ double half_coord(const CoupleArgs &a, int b, int c)
{
    return a.pos_in[3 * b + c] + 0.5 * a.mom_in[3 * b + c] / a.mass[b];
}

// Bond forces at R': F_b = mag d = -F_a, d = R'_b - R'_a, with
// mag = -k (r - r0) / r (harmonic) or mag = -k / (1 - r^2/r0^2) (FENE,
// eq. ufene; NaN at r >= r0, latched as bit 1 of *flags), added to a.fb.
__device__ __forceinline__ void bond_force(const CoupleArgs &a, int q)
{
    const int ia = a.bonds[2 * q], ib = a.bonds[2 * q + 1];
    if (ia < 0 || ib < 0 || ia >= a.n || ib >= a.n) return;
    double d[3], r2 = 0.0;
    for (int c = 0; c < 3; ++c) {
        d[c] = half_coord(a, ib, c) - half_coord(a, ia, c);
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
    for (int c = 0; c < 3; ++c) {
        atomicAdd(&a.fb[3 * ib + c], mag * d[c]);
        atomicAdd(&a.fb[3 * ia + c], -mag * d[c]);
    }
}

// One thread per bead, per bond and per entry of the idle bond accumulator
// (grid of max(n, nbonds, cap) threads): R' of the bead, the bond's forces
// (each bond forms R' of its two beads itself, so nothing waits for the
// first role), zero the accumulator of the next call, copy P to the tape,
// link the bead into its WCA cell.
__global__ void k_bead_half(CoupleArgs a)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < a.n) {
        double R[3];
        for (int c = 0; c < 3; ++c) {
            R[c] = half_coord(a, t, c);
            a.half[3 * t + c] = R[c];
        }
        if (a.cell_head) cell_link(t, R, a.cg, a.cell_of, a.cell_head, a.cell_next);
        if (a.tape_mom0)
            for (int c = 0; c < 3; ++c) a.tape_mom0[3 * t + c] = a.mom_in[3 * t + c];
    }
    if (t < a.cap)
        for (int c = 0; c < 3; ++c) a.fb_next[3 * t + c] = 0.0;
    if (t < a.nbonds) bond_force(a, t);
}

// Interpolation kernels phi_W (eq. 2point, eq. 3point, eq. 4point) and their
// derivatives (phi_2 differentiated away from the nodes).
template <int W>
__device__ __forceinline__ double phi_kernel(double r)
{
    const double a = fabs(r);
    if constexpr (W == 2) return a < 1.0 ? 1.0 - a : 0.0;
    if constexpr (W == 3) {
        if (a <= 0.5) return (1.0 + sqrt(1.0 - 3.0 * r * r)) / 3.0;
        if (a <= 1.5) return (5.0 - 3.0 * a - sqrt(-2.0 + 6.0 * a - 3.0 * r * r)) / 6.0;
        return 0.0;
    }
    if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * r * r)) / 8.0;
    if (a <= 2.0) return (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * r * r)) / 8.0;
    return 0.0;
}

template <int W>
__device__ __forceinline__ double dphi_kernel(double r)
{
    const double a = fabs(r), sg = r < 0.0 ? -1.0 : 1.0;
    if constexpr (W == 2) return (a < 1.0) ? -sg : 0.0;
    if constexpr (W == 3) {
        if (a <= 0.5) return -r / sqrt(1.0 - 3.0 * r * r);
        if (a <= 1.5) return sg * (-0.5 - (1.0 - a) / (2.0 * sqrt(-2.0 + 6.0 * a - 3.0 * r * r)));
        return 0.0;
    }
    if (a <= 1.0) return sg * (-2.0 + (4.0 - 8.0 * a) / (2.0 * sqrt(1.0 + 4.0 * a - 4.0 * r * r))) / 8.0;
    if (a <= 2.0) return sg * (-2.0 - (12.0 - 8.0 * a) / (2.0 * sqrt(-7.0 + 12.0 * a - 4.0 * r * r))) / 8.0;
    return 0.0;
}

// Lanes per bead: W^3 stencil nodes rounded up to a power of two dividing 64,
// so that a bead's lanes never straddle a wave.
template <int W> struct StencilLanes { static constexpr int value = W == 2 ? 8 : (W == 3 ? 32 : 64); };

// Node and weight of lane q of the W-point stencil around R' (x fastest; the
// first node along an axis: floor(R) for W = 2, the nearest node minus one
// for W = 3, floor(R) - 1 for W = 4).  Lanes q >= W^3 get weight 0.  With
// dw != nullptr also the weight's gradient in R'.
template <int W>
__device__ __forceinline__ void stencil_node(const double R[3], int q, const Geom &g, uint32_t &node, double &w,
                                             double *dw)
{
    node = 0u;
    w = 0.0;
    if (dw) dw[0] = dw[1] = dw[2] = 0.0;
    if (q >= W * W * W) return;
    const int d[3] = {q % W, (q / W) % W, q / (W * W)};
    const uint32_t L[3] = {g.nx, g.ny, g.nz};
    uint32_t cpos[3];
    double f[3], df[3];
    for (int c = 0; c < 3; ++c) {
        const double first = (W == 3) ? floor(R[c] + 0.5) - 1.0 : ((W == 4) ? floor(R[c]) - 1.0 : floor(R[c]));
        const double xc = first + (double)d[c];
        const double m = xc - (double)L[c] * floor(xc / (double)L[c]);  // xc mod L in [0, L)
        // a non-finite position (a bead given a NaN) maps to node 0
        uint32_t wi = (m >= 0.0 && m < (double)L[c]) ? (uint32_t)m : 0u;
        cpos[c] = wi;
        f[c] = phi_kernel<W>(R[c] - xc);
        df[c] = dw ? dphi_kernel<W>(R[c] - xc) : 0.0;
    }
    node = cpos[0] + g.nx * (cpos[1] + g.ny * cpos[2]);
    w = f[0] * f[1] * f[2];
    if (dw) {
        dw[0] = df[0] * f[1] * f[2];
        dw[1] = f[0] * df[1] * f[2];
        dw[2] = f[0] * f[1] * df[2];
    }
}

// Sum over the LANES lanes of one bead.
template <int LANES>
__device__ __forceinline__ double bead_sum(double v)
{
#pragma unroll
    for (int off = 1; off < LANES; off <<= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// StencilLanes<W> consecutive lanes per bead (blockDim a multiple of 64).
template <int ST, int W>
__global__ void __launch_bounds__(256) k_bead_update(CoupleArgs a)
{
    using S = Storage<ST>;
    using T = typename S::T;
    constexpr int LANES = StencilLanes<W>::value;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = t / LANES, q = t % LANES;
    const bool live = b < a.n;
    const Geom &g = a.geo;
    double ub[3] = {0.0, 0.0, 0.0};
    uint32_t node = 0;
    double wq = 0.0;
    // per-bead inputs: loaded together with R' (one round trip), and the
    // OU constants and the noise computed while the gather below is in flight
    double m = 1.0, z = 0.0, P[3] = {0.0, 0.0, 0.0}, Fc[3] = {0.0, 0.0, 0.0};
    const double h = 1.0;
    float v[Q];
    if (live) {
        const double R[3] = {a.half[3 * b], a.half[3 * b + 1], a.half[3 * b + 2]};
        m = a.mass[b];
        z = a.zeta[b];
        for (int c = 0; c < 3; ++c) {
            // F^c = (bonds + pairs) + fext
            Fc[c] = a.fb[3 * b + c];
            if (a.fp) Fc[c] += a.fp[3 * b + c];
            if (a.fext) Fc[c] += a.fext[3 * b + c];
            P[c] = a.mom_in[3 * b + c];
        }
        stencil_node<W>(R, q, g, node, wq, nullptr);
        if (q < W * W * W) {
            uint32_t xx, yy, zz;
            const PullOffsets o = pull_offsets(node, g, xx, yy, zz);
            const T *pop = static_cast<const T *>(a.pop);
#pragma unroll
            for (int i = 0; i < Q; ++i) v[i] = S::ld(pop[pull_index(node, o, i, zz, g)], 0.f);
        }
    }
    double C1 = 1.0, C2 = h, C3 = 0.0;
    if (z > 0.0) {
        C1 = exp(-z * h / m);
        C2 = (m / z) * (1.0 - C1);
        C3 = sqrt(m * a.kT * (1.0 - C1 * C1));  // exp(-2 zeta h/m) = C1^2
    }
    double th[3] = {0.0, 0.0, 0.0};
    if (live && a.kT > 0.0 && z > 0.0) {
        if (a.three_point)
            bead_three_point((uint32_t)b, a.step, a.box, a.key0, a.key1, th);
        else
            bead_normals((uint32_t)b, a.step, a.box, a.key0, a.key1, th);
    }
    if (live && q < W * W * W) {
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
    // sum the node contributions of the bead (its LANES lanes)
#pragma unroll
    for (int c = 0; c < 3; ++c) ub[c] = bead_sum<LANES>(ub[c]);
    if (!live) return;
    double Pn[3], I[3];
    for (int c = 0; c < 3; ++c) {
        Pn[c] = C1 * P[c] + C2 * (Fc[c] + z * ub[c]) + C3 * th[c];
        I[c] = -(Pn[c] - P[c] - h * Fc[c]);
    }
    long long iv[3] = {0, 0, 0};
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
        atomicOr(&a.fmask[node >> 5], 1u << (node & 31u));
    }
    if (a.tape_contrib) {
        long long *e = a.tape_contrib + 4 * ((size_t)b * LANES + q);
        e[0] = wq != 0.0 ? (long long)node : -1ll;
        e[1] = iv[0];
        e[2] = iv[1];
        e[3] = iv[2];
    }
    if (q == 0)
        for (int c = 0; c < 3; ++c) {
            a.mom[3 * b + c] = Pn[c];
            a.pos[3 * b + c] = a.half[3 * b + c] + 0.5 * h * Pn[c] / m;
            a.fc[3 * b + c] = Fc[c];
            if (a.tape_momn) a.tape_momn[3 * b + c] = Pn[c];
        }
    // the pair forces were read (k_wca ran before): this bead's cell list is done
    if (q == 0 && a.cell_head) a.cell_head[a.cell_of[b]] = -1;
}

}  // namespace lbmi
