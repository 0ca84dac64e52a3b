// Kremer-Grest bead-spring interactions on the device (Sec. "Coarse-grained
// models"): the purely repulsive Lennard-Jones (WCA) pair force of
// eq. ulennardjones between all beads within r_c = 2^(1/6) sigma of each
// other (minimum image along periodic axes; z is not periodic between
// walls), found with a cell list.
//
// Cell list, rebuilt on every coupled step from the half-step positions R':
//   cells per axis  n_a = floor(L_a / r_c) capped at a size tied to the bead
//                   count, so that a cell is never narrower than r_c; an axis
//                   with fewer than 3 cells gets one cell (then all beads along
//                   it are candidates and the minimum image picks the pair's
//                   single image within r_c < L_a / 2)
//   linking         (in k_bead_half, or k_cell_link for the adjoint) the cell
//                   of each bead and next[b] = the cell's previous head, the
//                   head swapped to b atomically; heads are -1 at rest (set
//                   at allocation; the kernel after the last reader of a
//                   step's list puts its beads' heads back to -1)
//   k_wca           32 lanes per bead, lane l visits neighbour cell l (27
//                   cells, fewer on one-cell axes) and takes the cell's
//                   members in increasing bead index, whatever order the
//                   linking left them in (batches of the 16 smallest
//                   indices above the last one done, one walk of the list
//                   per batch); a fixed butterfly sums the lanes.  Every pair is
//                   evaluated from both ends, so no atomics are needed and
//                   the bits are the same on every run.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace lbmi {

struct CellGrid {
    int32_t nc[3];     // cells per axis (1 or >= 3)
    int32_t periodic[3];  // 1: periodic axis (minimum image); 0: z between walls
    double L[3];       // box extents
    double inv_w[3];   // nc / L
    double rc2;        // squared cutoff 2^(1/3) sigma^2
    double sig2;       // sigma^2
    double eps24;      // 24 epsilon
};

// Cell coordinate along one axis of a (possibly unwrapped, possibly
// non-finite) position: always in [0, nc).  A periodic axis wraps the
// position into the box; a non-periodic one clamps it to the edge cells, so
// beads beyond a wall share the edge cell with those next to it.
__device__ __forceinline__ int cell_coord(double x, double L, double inv_w, int nc, int periodic)
{
    const double xw = periodic ? x - L * floor(x / L) : x;
    double t = floor(xw * inv_w);
    if (!(t >= 0.0)) t = 0.0;
    if (t > (double)(nc - 1)) t = (double)(nc - 1);
    return (int)t;
}

__device__ __forceinline__ double nearest_image(double d, double L) { return d - L * floor(d / L + 0.5); }

// Pair separation along one axis: the minimum image if periodic.
__device__ __forceinline__ double pair_sep(double d, double L, int periodic)
{
    return periodic ? nearest_image(d, L) : d;
}

// Neighbour cell along one axis at offset o from c: wrapped on a periodic
// axis, -1 (none) past the end of a non-periodic one.
__device__ __forceinline__ int neighbour_cell(int c, int o, int nc, int periodic)
{
    int cn = c + o;
    if (cn < 0) return periodic ? cn + nc : -1;
    if (cn >= nc) return periodic ? cn - nc : -1;
    return cn;
}

// Cell of a position (flattened).
__device__ __forceinline__ int cell_index(const double R[3], const CellGrid &cg)
{
    int c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) c[a] = cell_coord(R[a], cg.L[a], cg.inv_w[a], cg.nc[a], cg.periodic[a]);
    return c[0] + cg.nc[0] * (c[1] + cg.nc[1] * c[2]);
}

// Put bead b at R into its cell's list.
__device__ __forceinline__ void cell_link(int b, const double R[3], const CellGrid &cg, int32_t *cell_of,
                                          int32_t *head, int32_t *next)
{
    const int cell = cell_index(R, cg);
    cell_of[b] = cell;
    next[b] = atomicExch(&head[cell], b);
}

__global__ void k_cell_link(const double *__restrict__ half, int n, CellGrid cg, int32_t *cell_of, int32_t *head,
                            int32_t *next)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const double R[3] = {half[3 * b], half[3 * b + 1], half[3 * b + 2]};
    cell_link(b, R, cg, cell_of, head, next);
}

// Neighbour cell l of `cell` (flattened), or -1 past a wall or beyond the
// neighbourhood (lanes l >= the number of neighbour cells).
__device__ __forceinline__ int lane_cell(int cell, int l, const CellGrid &cg)
{
    const int span[3] = {cg.nc[0] >= 3 ? 1 : 0, cg.nc[1] >= 3 ? 1 : 0, cg.nc[2] >= 3 ? 1 : 0};
    const int w0 = 2 * span[0] + 1, w1 = 2 * span[1] + 1, w2 = 2 * span[2] + 1;
    if (l >= w0 * w1 * w2) return -1;
    const int o[3] = {l % w0 - span[0], (l / w0) % w1 - span[1], l / (w0 * w1) - span[2]};
    const int ci[3] = {cell % cg.nc[0], (cell / cg.nc[0]) % cg.nc[1], cell / (cg.nc[0] * cg.nc[1])};
    int cn[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) cn[a] = neighbour_cell(ci[a], o[a], cg.nc[a], cg.periodic[a]);
    return (cn[0] < 0 || cn[1] < 0 || cn[2] < 0) ? -1 : cn[0] + cg.nc[0] * (cn[1] + cg.nc[1] * cn[2]);
}

// Calls f(j) for every member j != self of cell `cell`'s list in increasing
// index order.  Each walk keeps the 16 smallest indices above the last one
// done in a sorted register array (a compare-exchange chain).  The walks are
// bounded (n hops, indices checked against n), so a list that is not what
// the linking left could only give wrong members, never run away.
template <typename F>
__device__ __forceinline__ void for_members_in_order(int cell, int self, int n, const int32_t *__restrict__ head,
                                                     const int32_t *__restrict__ next, F &&f)
{
    if (cell < 0) return;
    const int first = head[cell];
    constexpr int B = 16;
    constexpr int kNone = 0x7fffffff;
    int last = -1;
    for (int batch = 0; batch <= n / B; ++batch) {
        int a[B];
#pragma unroll
        for (int u = 0; u < B; ++u) a[u] = kNone;
        int j = first;
        for (int hops = 0; j >= 0 && j < n && hops < n; ++hops) {
            if (j > last && j != self) {
                int x = j;
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    const int lo = min(a[u], x);
                    x = max(a[u], x);
                    a[u] = lo;
                }
            }
            j = next[j];
        }
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (a[u] != kNone) f(a[u]);
        if (a[B - 1] == kNone) return;
        last = a[B - 1];
    }
}

constexpr int kPairLanes = 32;

// fp_i = sum_j f(r_ij) (R_i - R_j) over beads j != i within r_c, with
// f = 24 eps (2 (sigma/r)^12 - (sigma/r)^6) / r^2 = -V'(r)/r of eq. ulennardjones.
// kPairLanes consecutive lanes per bead (blockDim a multiple of 64).
__global__ void __launch_bounds__(256) k_wca(const double *__restrict__ half, int n, CellGrid cg,
                                             const int32_t *__restrict__ cell_of, const int32_t *__restrict__ head,
                                             const int32_t *__restrict__ next, double *fp)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = t / kPairLanes, l = t % kPairLanes;
    double F[3] = {0.0, 0.0, 0.0};
    if (i < n) {
        const int nb = lane_cell(cell_of[i], l, cg);
        const double Ri[3] = {half[3 * i], half[3 * i + 1], half[3 * i + 2]};
        for_members_in_order(nb, i, n, head, next, [&](int j) {
            const double d0 = pair_sep(Ri[0] - half[3 * j], cg.L[0], cg.periodic[0]);
            const double d1 = pair_sep(Ri[1] - half[3 * j + 1], cg.L[1], cg.periodic[1]);
            const double d2 = pair_sep(Ri[2] - half[3 * j + 2], cg.L[2], cg.periodic[2]);
            const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
            if (!(r2 < cg.rc2)) return;
            const double s2 = cg.sig2 / r2;
            const double s6 = s2 * s2 * s2;
            const double f = cg.eps24 * (2.0 * s6 * s6 - s6) / r2;
            F[0] += f * d0;
            F[1] += f * d1;
            F[2] += f * d2;
        });
    }
    // butterfly over the bead's lanes (every lane ends with the same bits)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int off = 1; off < kPairLanes; off <<= 1) F[a] += __shfl_xor(F[a], off, 64);
    if (i < n && l == 0)
#pragma unroll
        for (int a = 0; a < 3; ++a) fp[3 * i + a] = F[a];
}

// Adjoint of the pair forces: with fp_i = sum_j mag(r^2) d_ij, d_ij = R_i - R_j,
// mag = 24 eps (2 s^2 - s)/r^2, s = (sigma^2/r^2)^3, the Jacobian of each term
// is J = mag I + 2 mag' d d^T, 2 mag' = 24 eps (-28 s^2 + 8 s)/r^4, symmetric
// and even in d, so half_bar_i += sum_j J(d_ij) (fc_bar_i - fc_bar_j).  Same
// lanes and cell order as k_wca (fixed sums, no atomics).
__global__ void __launch_bounds__(256) k_wca_adjoint(const double *__restrict__ half, int n, CellGrid cg,
                                                     const int32_t *__restrict__ cell_of,
                                                     const int32_t *__restrict__ head,
                                                     const int32_t *__restrict__ next,
                                                     const double *__restrict__ fc_bar, double *half_bar)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = t / kPairLanes, l = t % kPairLanes;
    double B[3] = {0.0, 0.0, 0.0};
    if (i < n) {
        const int nb = lane_cell(cell_of[i], l, cg);
        const double Ri[3] = {half[3 * i], half[3 * i + 1], half[3 * i + 2]};
        const double Gi[3] = {fc_bar[3 * i], fc_bar[3 * i + 1], fc_bar[3 * i + 2]};
        for_members_in_order(nb, i, n, head, next, [&](int j) {
            double d[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) d[a] = pair_sep(Ri[a] - half[3 * j + a], cg.L[a], cg.periodic[a]);
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (!(r2 < cg.rc2)) return;
            double v[3], dv = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                v[a] = Gi[a] - fc_bar[3 * j + a];
                dv += d[a] * v[a];
            }
            const double s2 = cg.sig2 / r2;
            const double s6 = s2 * s2 * s2;
            const double mag = cg.eps24 * (2.0 * s6 * s6 - s6) / r2;
            const double mag2p = cg.eps24 * (-28.0 * s6 * s6 + 8.0 * s6) / (r2 * r2);
#pragma unroll
            for (int a = 0; a < 3; ++a) B[a] += mag * v[a] + mag2p * d[a] * dv;
        });
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int off = 1; off < kPairLanes; off <<= 1) B[a] += __shfl_xor(B[a], off, 64);
    if (i < n && l == 0)
#pragma unroll
        for (int a = 0; a < 3; ++a) half_bar[3 * i + a] += B[a];
}

}  // namespace lbmi
