// Point-particle (bead) coupling kernels of liblbmi (Sec. "Force coupling",
// Sec. "Interpolating functions").  Bead state is FP64; the fluid velocity is
// gathered from the stored populations.
//
// One coupled step on the device:
//   k_bead_half     R' = R + (h/2) P/m, clear conservative forces
//   k_bonds         harmonic bond forces at R' (FP64 atomics; a bead with at
//                   most two bonds gets a bitwise reproducible sum)
//   k_bead_update   u_b by trilinear interpolation (phi_2 product kernel,
//                   eq. Delta/eq. 2point) of u = (sum n c + g/2)/rho,
//                   P'' = C1 P + C2 (F^c + zeta u_b) + C3 theta
//                   (eq. langevin_momentum_update), impulse
//                   I = -(P'' - P - h F^c) spread to the 8 nodes
//                   (eq. ftotal) into a sparse force field, R = R' + (h/2) P''/m
//   k_fixup         (inside the next lb_step) re-collides the touched nodes
//                   with the full force g + f(r) and clears the force field.
#pragma once

#include "aux_kernels.h"

namespace lbmi {

struct CoupleArgs {
    const void *pop;      // current buffer A
    Geom geo;
    double rho0;
    double g[3];
    double kT;
    uint32_t key0, key1, box, step;
    int32_t n;
    double *pos;
    double *mom;
    const double *mass;
    const double *zeta;
    double *half;         // [n][3]
    double *fc;           // [n][3]
    float *force;         // [3][N] sparse force field (zero outside touched nodes)
    int32_t *mark;        // [N] 1 = node already in the list
    int32_t *list;        // [8 n] touched nodes
    int32_t *count;       // number of entries in list
};

__global__ void k_bead_half(CoupleArgs a)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.n) return;
    const double m = a.mass[b];
    for (int c = 0; c < 3; ++c) {
        a.half[3 * b + c] = a.pos[3 * b + c] + 0.5 * a.mom[3 * b + c] / m;
        a.fc[3 * b + c] = 0.0;
    }
}

__global__ void k_bonds(const double *__restrict__ half, double *fc, const int32_t *__restrict__ bonds, int nbonds,
                        double kb, double r0, int nbeads)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nbonds) return;
    const int ia = bonds[2 * q], ib = bonds[2 * q + 1];
    if (ia < 0 || ib < 0 || ia >= nbeads || ib >= nbeads) return;
    double d[3], r2 = 0.0;
    for (int c = 0; c < 3; ++c) {
        d[c] = half[3 * ib + c] - half[3 * ia + c];
        r2 += d[c] * d[c];
    }
    const double r = sqrt(r2);
    if (r == 0.0) return;
    const double mag = -kb * (r - r0) / r;
    for (int c = 0; c < 3; ++c) {
        atomicAdd(&fc[3 * ib + c], mag * d[c]);
        atomicAdd(&fc[3 * ia + c], -mag * d[c]);
    }
}

__global__ void k_reset_count(int32_t *count) { *count = 0; }

template <int ST>
__global__ void k_bead_update(CoupleArgs a)
{
    using S = Storage<ST>;
    using T = typename S::T;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.n) return;
    const Geom &g = a.geo;
    const uint32_t L[3] = {g.nx, g.ny, g.nz};
    uint32_t base[3];
    double frac[3];
    for (int c = 0; c < 3; ++c) {
        const double r = a.half[3 * b + c];
        const double f = floor(r);
        frac[c] = r - f;
        double w = f - (double)L[c] * floor(f / (double)L[c]);  // f mod L in [0, L)
        uint32_t wi = (uint32_t)w;
        if (wi >= L[c]) wi = 0;
        base[c] = wi;
    }
    const T *pop = static_cast<const T *>(a.pop);
    uint32_t node[8];
    double wgt[8];
    double ub[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < 8; ++q) {
        const int dx = q & 1, dy = (q >> 1) & 1, dz = q >> 2;
        const uint32_t x = (base[0] + dx) % L[0], y = (base[1] + dy) % L[1], z = (base[2] + dz) % L[2];
        const uint32_t s = x + g.nx * (y + g.ny * z);
        node[q] = s;
        wgt[q] = (dx ? frac[0] : 1.0 - frac[0]) * (dy ? frac[1] : 1.0 - frac[1]) * (dz ? frac[2] : 1.0 - frac[2]);
        uint32_t xx, yy, zz;
        const PullOffsets o = pull_offsets(s, g, xx, yy, zz);
        double m = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q; ++i) {
            const double v = (double)S::ld(pop[(size_t)i * g.N + pull_src(s, o, i)], 0.f);
            m += v;
            j[0] += v * kCX[i];
            j[1] += v * kCY[i];
            j[2] += v * kCZ[i];
        }
        const double rho = a.rho0 + m;
        for (int c = 0; c < 3; ++c) ub[c] += wgt[q] * (j[c] + 0.5 * a.g[c]) / rho;
    }
    const double m = a.mass[b], z = a.zeta[b], h = 1.0;
    double C1, C2, C3;
    if (z > 0.0) {
        C1 = exp(-z * h / m);
        C2 = (m / z) * (1.0 - C1);
        C3 = sqrt(m * a.kT * (1.0 - exp(-2.0 * z * h / m)));
    } else {
        C1 = 1.0;
        C2 = h;
        C3 = 0.0;
    }
    double th[3] = {0.0, 0.0, 0.0};
    if (a.kT > 0.0 && z > 0.0) bead_normals((uint32_t)b, a.step, a.box, a.key0, a.key1, th);
    double Pn[3], I[3];
    for (int c = 0; c < 3; ++c) {
        const double P = a.mom[3 * b + c], Fc = a.fc[3 * b + c];
        Pn[c] = C1 * P + C2 * (Fc + z * ub[c]) + C3 * th[c];
        I[c] = -(Pn[c] - P - h * Fc);
    }
    for (int q = 0; q < 8; ++q) {
        if (wgt[q] == 0.0) continue;
        for (int c = 0; c < 3; ++c) atomicAdd(&a.force[(size_t)c * g.N + node[q]], (float)(wgt[q] * I[c] / h));
        if (atomicExch(&a.mark[node[q]], 1) == 0) {
            const int slot = atomicAdd(a.count, 1);
            a.list[slot] = (int32_t)node[q];
        }
    }
    for (int c = 0; c < 3; ++c) {
        a.mom[3 * b + c] = Pn[c];
        a.pos[3 * b + c] = a.half[3 * b + c] + 0.5 * h * Pn[c] / m;
    }
}

struct FixupArgs {
    StepArgs st;
    float *force;
    int32_t *mark;
    const int32_t *list;
    const int32_t *count;
    int32_t cap;
    double *fixpartials;  // [cap][4] totals corrections
};

// Re-collide the nodes that received bead force, with F = g + f(node); write
// over the step kernel's output at those nodes; record the change of the
// stored totals; clear the force field and marks.
template <int ST, bool THERMAL>
__global__ void k_fixup(FixupArgs f)
{
    using S = Storage<ST>;
    using T = typename S::T;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= f.cap) return;
    double *part = f.fixpartials + 4 * (size_t)idx;
    if (idx >= *f.count) {
        part[0] = part[1] = part[2] = part[3] = 0.0;
        return;
    }
    const StepArgs &a = f.st;
    const uint32_t s = (uint32_t)f.list[idx];
    const uint32_t N = a.geo.N;
    uint32_t x, y, z;
    const PullOffsets o = pull_offsets(s, a.geo, x, y, z);
    const T *src = static_cast<const T *>(a.src);
    T *dst = static_cast<T *>(a.dst);
    float d[Q];
    for (int i = 0; i < Q; ++i) d[i] = S::ld(src[(size_t)i * N + pull_src(s, o, i)], 0.f);
    float F[3];
    for (int c = 0; c < 3; ++c) {
        F[c] = a.cc.g[c] + f.force[(size_t)c * N + s];
        f.force[(size_t)c * N + s] = 0.f;
    }
    f.mark[s] = 0;
    float out[Q];
    collide_site<THERMAL>(d, F, a.cc, s, a.step, out);
    double dm = 0.0, dp[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        const double old = (double)S::ld(dst[(size_t)i * N + s], 0.f);
        const T v = S::st(out[i], 0.f);
        dst[(size_t)i * N + s] = v;
        const double diff = (double)S::ld(v, 0.f) - old;
        dm += diff;
        dp[0] += diff * kCX[i];
        dp[1] += diff * kCY[i];
        dp[2] += diff * kCZ[i];
    }
    if (!__builtin_isfinite(out[0])) __hip_atomic_fetch_or(a.flags, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    part[0] = dm;
    part[1] = dp[0];
    part[2] = dp[1];
    part[3] = dp[2];
}

}  // namespace lbmi
