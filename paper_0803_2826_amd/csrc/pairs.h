// Kremer-Grest bead-spring interactions on the device (Sec. "Coarse-grained
// models"): the purely repulsive Lennard-Jones (WCA) pair force of
// eq. ulennardjones between all beads within r_c = 2^(1/6) sigma of each
// other at their periodic minimum-image distance, found with a cell list.
//
// Cell list, rebuilt on every coupled step from the half-step positions R':
//   cells per axis  n_a = floor(L_a / r_c) capped at a size tied to the bead
//                   count, so that a cell is never narrower than r_c; an axis
//                   with fewer than 3 cells gets one cell (then all beads along
//                   it are candidates and the minimum image picks the pair's
//                   single image within r_c < L_a / 2)
//   k_cell_count    cell of each bead, its slot = atomic increment of the
//                   cell's count
//   (scan)          exclusive prefix sum of the counts: first entry per cell
//   k_cell_fill     sorted[start[cell] + slot] = bead
//   k_cell_order    per cell, the bead indices in ascending order, so that the
//                   force sums below run in a fixed order (reproducible bits)
//   k_wca           one thread per bead: the 27 neighbour cells (3 per axis,
//                   1 on a one-cell axis) in a fixed order; every pair is
//                   evaluated from both ends, so no atomics are needed.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace lbmi {

struct CellGrid {
    int32_t nc[3];     // cells per axis (1 or >= 3)
    double L[3];       // periodic box extents
    double inv_w[3];   // nc / L
    double rc2;        // squared cutoff 2^(1/3) sigma^2
    double sig2;       // sigma^2
    double eps24;      // 24 epsilon
};

// Cell coordinate along one axis of a (possibly unwrapped, possibly
// non-finite) position: always in [0, nc).
__device__ __forceinline__ int cell_coord(double x, double L, double inv_w, int nc)
{
    const double xw = x - L * floor(x / L);
    double t = floor(xw * inv_w);
    if (!(t >= 0.0)) t = 0.0;
    if (t > (double)(nc - 1)) t = (double)(nc - 1);
    return (int)t;
}

__device__ __forceinline__ double nearest_image(double d, double L) { return d - L * floor(d / L + 0.5); }

// count has ncell + 1 entries, zero on entry (the last stays zero, so the
// exclusive scan's last entry is the bead count).
__global__ void k_cell_count(const double *__restrict__ half, int n, CellGrid cg, int32_t *cell_of, int32_t *slot,
                             int32_t *count)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    int c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) c[a] = cell_coord(half[3 * b + a], cg.L[a], cg.inv_w[a], cg.nc[a]);
    const int cell = c[0] + cg.nc[0] * (c[1] + cg.nc[1] * c[2]);
    cell_of[b] = cell;
    slot[b] = atomicAdd(&count[cell], 1);
}

__global__ void k_cell_fill(int n, const int32_t *__restrict__ cell_of, const int32_t *__restrict__ slot,
                            const int32_t *__restrict__ start, int32_t *sorted)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    sorted[start[cell_of[b]] + slot[b]] = b;
}

// Insertion sort of each cell's (short) bead list.
__global__ void k_cell_order(int ncell, const int32_t *__restrict__ start, int32_t *sorted)
{
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= ncell) return;
    const int lo = start[cell], hi = start[cell + 1];
    for (int k = lo + 1; k < hi; ++k) {
        const int32_t v = sorted[k];
        int m = k - 1;
        while (m >= lo && sorted[m] > v) {
            sorted[m + 1] = sorted[m];
            --m;
        }
        sorted[m + 1] = v;
    }
}

// F_i += sum_j f(r_ij) (R_i - R_j) over beads j != i within r_c, with
// f = 24 eps (2 (sigma/r)^12 - (sigma/r)^6) / r^2 = -V'(r)/r of eq. ulennardjones.
__global__ void __launch_bounds__(256) k_wca(const double *__restrict__ half, int n, CellGrid cg,
                                             const int32_t *__restrict__ cell_of, const int32_t *__restrict__ start,
                                             const int32_t *__restrict__ sorted, double *fc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double Ri[3] = {half[3 * i], half[3 * i + 1], half[3 * i + 2]};
    const int cell = cell_of[i];
    const int ci[3] = {cell % cg.nc[0], (cell / cg.nc[0]) % cg.nc[1], cell / (cg.nc[0] * cg.nc[1])};
    const int span[3] = {cg.nc[0] >= 3 ? 1 : 0, cg.nc[1] >= 3 ? 1 : 0, cg.nc[2] >= 3 ? 1 : 0};
    double F[3] = {0.0, 0.0, 0.0};
    for (int oz = -span[2]; oz <= span[2]; ++oz) {
        int cz = ci[2] + oz;
        cz += cz < 0 ? cg.nc[2] : (cz >= cg.nc[2] ? -cg.nc[2] : 0);
        for (int oy = -span[1]; oy <= span[1]; ++oy) {
            int cy = ci[1] + oy;
            cy += cy < 0 ? cg.nc[1] : (cy >= cg.nc[1] ? -cg.nc[1] : 0);
            for (int ox = -span[0]; ox <= span[0]; ++ox) {
                int cx = ci[0] + ox;
                cx += cx < 0 ? cg.nc[0] : (cx >= cg.nc[0] ? -cg.nc[0] : 0);
                const int nb = cx + cg.nc[0] * (cy + cg.nc[1] * cz);
                const int hi = start[nb + 1];
                for (int k = start[nb]; k < hi; ++k) {
                    const int j = sorted[k];
                    if (j == i) continue;
                    double d[3], r2 = 0.0;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        d[a] = nearest_image(Ri[a] - half[3 * j + a], cg.L[a]);
                        r2 += d[a] * d[a];
                    }
                    if (!(r2 < cg.rc2)) continue;
                    const double s2 = cg.sig2 / r2;
                    const double s6 = s2 * s2 * s2;
                    const double f = cg.eps24 * (2.0 * s6 * s6 - s6) / r2;
#pragma unroll
                    for (int a = 0; a < 3; ++a) F[a] += f * d[a];
                }
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) fc[3 * i + a] += F[a];
}

}  // namespace lbmi
