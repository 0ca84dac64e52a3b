/*
 * FP64 CPU oracle for the fluctuating D3Q19 lattice-Boltzmann method with
 * frictional point-particle coupling (Duenweg & Ladd, "Lattice Boltzmann
 * simulations of soft matter systems").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or generator with the HIP library: every constant below is
 * written out here from the paper, and the counter-based random number
 * generator is implemented here from its published definition.
 *
 * Arithmetic is IEEE double, compiled without floating-point contraction.
 * Loops are written the way the paper states the algorithm: moments by a
 * full 19x19 matrix-vector product, the equilibrium from its closed form,
 * relaxation mode by mode, the back-transformation by the weighted basis,
 * the forcing term in population space.  No pair sums, no fusion.
 *
 * Conventions (readings where the paper is silent; each is listed with its
 * reason in the design notes):
 *   - lattice units b = h = 1, c_s^2 = 1/3, so mu = kT / c_s^2 = 3 kT;
 *   - velocity order: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 the twelve
 *     diagonal directions in opposite pairs (see CV below);
 *   - state array layout n[i*N + s], s = x + nx*(y + ny*z), periodic box;
 *   - the stored state is the pre-collision population n(r,t); one step is
 *     collide at every site then stream, n_i(r+c_i,t+1) = n*_i(r,t);
 *   - random numbers: Philox4x32-10 keyed by the seed, counter
 *     (site, step, stream<<16 | call, box); 24-bit uniforms; Box-Muller.
 *
 * Parity status of every exported function is stated at its definition.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19

/* Number of threads the whole-lattice loops use. */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Lattice tables (Sec. "D3Q19 model I/II", Table 1)                         */
/* ------------------------------------------------------------------------ */

/* The 19 velocities of D3Q19: rest, 6 nearest and 12 next-nearest
 * neighbours (D3Q19 classification in the introduction of the fluctuating LB
 * section).  The paper fixes the set, not the order; opposite directions are
 * adjacent here. */
static const int CV[Q][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

/* Weights a^{c_i}: 1/3 for the rest particle, 1/18 for speed 1, 1/36 for
 * speed sqrt(2) (text after eq. original_equil_distrib). */
static double weight_of_speed2(int c2)
{
    if (c2 == 0) return 1.0 / 3.0;
    if (c2 == 1) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

/* Basis polynomials e_ki of Table 1, evaluated at c_i (c = b/h = 1, so the
 * hatted and plain velocities coincide). */
static double basis(int k, int cx, int cy, int cz)
{
    const double x = cx, y = cy, z = cz;
    const double c2 = x * x + y * y + z * z;
    switch (k) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return c2 - 1.0;
    case 5: return 3.0 * x * x - c2;
    case 6: return y * y - z * z;
    case 7: return x * y;
    case 8: return y * z;
    case 9: return z * x;
    case 10: return (3.0 * c2 - 5.0) * x;
    case 11: return (3.0 * c2 - 5.0) * y;
    case 12: return (3.0 * c2 - 5.0) * z;
    case 13: return (y * y - z * z) * x;
    case 14: return (z * z - x * x) * y;
    case 15: return (x * x - y * y) * z;
    case 16: return 3.0 * c2 * c2 - 6.0 * c2 + 1.0;
    case 17: return (2.0 * c2 - 3.0) * (3.0 * x * x - c2);
    case 18: return (2.0 * c2 - 3.0) * (y * y - z * z);
    }
    return 0.0;
}

/* Normalisation factors w_k, third column of Table 1. */
static const double WK[Q] = {1.0,       1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0, 2.0 / 3.0,
                             4.0 / 3.0, 4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                             2.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0, 2.0 / 9.0, 2.0 / 9.0,
                             2.0 / 9.0, 2.0,       4.0 / 3.0, 4.0 / 9.0};

static const double CS2 = 1.0 / 3.0; /* c_s^2 = (1/3)(b/h)^2 */

static double A[Q];     /* a^{c_i} */
static double E[Q][Q];  /* e_ki */
static int tables_ready = 0;

static void init_tables(void)
{
    if (tables_ready) return;
    for (int i = 0; i < Q; ++i) {
        const int c2 = CV[i][0] * CV[i][0] + CV[i][1] * CV[i][1] + CV[i][2] * CV[i][2];
        A[i] = weight_of_speed2(c2);
        for (int k = 0; k < Q; ++k) E[k][i] = basis(k, CV[i][0], CV[i][1], CV[i][2]);
    }
    tables_ready = 1;
}

/* Parity pinned: tests check sum a = 1, isotropy of the second and fourth
 * moments (eq. w1-w4 with C4' = 0, C4 = C2^2), and that the weighted Gram
 * matrix of e_ki is diag(w_k) (eq. orthogonality with q = a). */
void orc_tables(int32_t *c_out, double *a_out, double *e_out, double *w_out)
{
    init_tables();
    for (int i = 0; i < Q; ++i) {
        for (int d = 0; d < 3; ++d) c_out[3 * i + d] = CV[i][d];
        a_out[i] = A[i];
    }
    for (int k = 0; k < Q; ++k) {
        w_out[k] = WK[k];
        for (int i = 0; i < Q; ++i) e_out[k * Q + i] = E[k][i];
    }
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Gaussian variates   */
/* ------------------------------------------------------------------------ */

/* Parity pinned against an independent library implementation (rocRAND's
 * philox engine, compiled for the host) by the test suite. */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u; /* round multipliers */
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u; /* Weyl key increments */
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)M0 * (uint64_t)c[0];
        const uint64_t p1 = (uint64_t)M1 * (uint64_t)c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c[1] ^ k0;
        const uint32_t n1 = lo1;
        const uint32_t n2 = hi0 ^ c[3] ^ k1;
        const uint32_t n3 = lo0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

static const double TWO_M24 = 1.0 / 16777216.0; /* 2^-24 */
static const double TWO_PI = 6.283185307179586476925286766559;

/* Box-Muller: radius from a uniform in (0,1], angle from a uniform in [0,1). */
static void box_muller(uint32_t fa, uint32_t fb, double *g0, double *g1)
{
    const double ua = ((double)fa + 1.0) * TWO_M24;
    const double ub = (double)fb * TWO_M24;
    const double r = sqrt(-2.0 * log(ua));
    *g0 = r * cos(TWO_PI * ub);
    *g1 = r * sin(TWO_PI * ub);
}

/* Sixteen unit Gaussians for the fluid noise at (site, step, box).  Three
 * Philox calls (counter word 2 = call 0,1,2; stream 0) give twelve 32-bit
 * words; each group of three words w0,w1,w2 yields four 24-bit fields
 * w0>>8, w1>>8, w2>>8 and the three low bytes (w0&255)|(w1&255)<<8|(w2&255)<<16.
 * Field pairs (2p, 2p+1) feed Box-Muller pair p.  Mode k = 4..18 takes g[k-4].
 * Parity pinned: distribution tests (moments, independence) in the suite;
 * the integer stream is pinned through orc_philox4x32_10. */
void orc_fluid_normals(uint64_t seed, uint32_t site, uint32_t step, uint32_t box, double g[16])
{
    const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t w[12];
    for (uint32_t call = 0; call < 3; ++call) {
        const uint32_t ctr[4] = {site, step, (0u << 16) | call, box};
        orc_philox4x32_10(ctr, key, &w[4 * call]);
    }
    uint32_t f[16];
    for (int grp = 0; grp < 4; ++grp) {
        const uint32_t a = w[3 * grp], b = w[3 * grp + 1], c = w[3 * grp + 2];
        f[4 * grp + 0] = a >> 8;
        f[4 * grp + 1] = b >> 8;
        f[4 * grp + 2] = c >> 8;
        f[4 * grp + 3] = (a & 0xffu) | ((b & 0xffu) << 8) | ((c & 0xffu) << 16);
    }
    for (int p = 0; p < 8; ++p) box_muller(f[2 * p], f[2 * p + 1], &g[2 * p], &g[2 * p + 1]);
}

/* Three unit Gaussians for the Langevin noise of bead `bead` at `step`
 * (stream 1, one Philox call; fields w0>>8,w1>>8 and w2>>8,w3>>8). */
void orc_bead_normals(uint64_t seed, uint32_t bead, uint32_t step, uint32_t box, double g[3])
{
    const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    const uint32_t ctr[4] = {bead, step, (1u << 16) | 0u, box};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    double g3;
    box_muller(w[0] >> 8, w[1] >> 8, &g[0], &g[1]);
    box_muller(w[2] >> 8, w[3] >> 8, &g[2], &g3);
}

/* Three finite-range variates for the Langevin noise of bead `bead` at
 * `step` (Sec. "Force coupling", the three-point distribution given after
 * eq. langevin_momentum_update: theta = 0 with probability 2/3 and
 * +-sqrt(3) with probability 1/6 each, so that its moments match a unit
 * Gaussian's through the fourth).  The same Philox call as the Gaussian
 * variant (stream 1); word a picks a sixth k = floor(6 w_a / 2^32) of the
 * 32-bit range: k = 0 gives -sqrt(3), k = 5 gives +sqrt(3), any other k 0.
 * Parity pinned: the sixth is checked against exact rational thresholds
 * on the words orc_philox4x32_10 returns, and the frozen-fluid OU variance
 * holds with these variates. */
void orc_bead_three_point(uint64_t seed, uint32_t bead, uint32_t step, uint32_t box, double g[3])
{
    const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    const uint32_t ctr[4] = {bead, step, (1u << 16) | 0u, box};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    for (int a = 0; a < 3; ++a) {
        const uint64_t k = ((uint64_t)w[a] * 6u) >> 32;
        g[a] = (k == 0) ? -sqrt(3.0) : (k == 5) ? sqrt(3.0) : 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Parameters                                                                */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t nx, ny, nz;
    int32_t noise_rho0;   /* 0: noise amplitude uses local rho, 1: uses rho0 */
    double rho0;
    double gamma_shear, gamma_bulk, gamma_3a, gamma_3b, gamma_4a, gamma_4b;
    double kT;
    double g[3];          /* uniform body-force density */
    uint64_t seed;
    uint32_t box;
    uint32_t walls;       /* 1: stationary walls at z = -1/2 and z = nz - 1/2 */
} orc_params;

/* Opposite direction of velocity i (the table keeps opposites adjacent). */
static int opposite(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

/* Whether the link from site z along velocity i crosses a stationary wall. */
static int crosses_wall(const orc_params *p, int z, int i)
{
    const int zz = z + CV[i][2];
    return p->walls && (zz < 0 || zz >= p->nz);
}

/* Eigenvalue gamma_k of each mode (Sec. "D3Q19 model II"): bulk mode 4,
 * shear modes 5-9, kinetic groups 10-12, 13-15, 16, 17-18.  Conserved
 * modes 0-3 are left untouched by the relaxation. */
static void mode_gammas(const orc_params *p, double gam[Q])
{
    for (int k = 0; k < 4; ++k) gam[k] = 1.0;
    gam[4] = p->gamma_bulk;
    for (int k = 5; k <= 9; ++k) gam[k] = p->gamma_shear;
    for (int k = 10; k <= 12; ++k) gam[k] = p->gamma_3a;
    for (int k = 13; k <= 15; ++k) gam[k] = p->gamma_3b;
    gam[16] = p->gamma_4a;
    gam[17] = p->gamma_4b;
    gam[18] = p->gamma_4b;
}

/* ------------------------------------------------------------------------ */
/* Single-site operations                                                    */
/* ------------------------------------------------------------------------ */

/* Equilibrium populations, eq. original_equil_distrib.
 * Parity pinned: tests check its mass, momentum and second moment against
 * eq. MBeq0-MBeq2 (rho, rho u, rho c_s^2 delta + rho u u). */
void orc_equilibrium(double rho, const double u[3], double neq[Q])
{
    init_tables();
    const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        const double uc = u[0] * CV[i][0] + u[1] * CV[i][1] + u[2] * CV[i][2];
        neq[i] = A[i] * rho * (1.0 + uc / CS2 + uc * uc / (2.0 * CS2 * CS2) - usq / (2.0 * CS2));
    }
}

/* Moments m_k = sum_i e_ki n_i (eq. "forward"). */
void orc_moments_site(const double n[Q], double m[Q])
{
    init_tables();
    for (int k = 0; k < Q; ++k) {
        double s = 0.0;
        for (int i = 0; i < Q; ++i) s += E[k][i] * n[i];
        m[k] = s;
    }
}

/* Back-transformation n_i = a_i sum_k e_ki m_k / w_k (eq. back_transformation
 * with q = a). */
void orc_back_site(const double m[Q], double n[Q])
{
    init_tables();
    for (int i = 0; i < Q; ++i) {
        double s = 0.0;
        for (int k = 0; k < Q; ++k) s += E[k][i] * m[k] / WK[k];
        n[i] = A[i] * s;
    }
}

/* One stochastic collision at one site, with force density F (Sec. "D3Q19
 * model II/III", Sec. "External forces"):
 *   1. m_k = sum_i e_ki n_i;  rho = m_0;  j = sum_i n_i c_i + F/2
 *      (eq. special_choice_momentum_density);  u = j / rho;
 *   2. n^eq(rho, u) from eq. original_equil_distrib, m^eq = E n^eq;
 *   3. for the non-conserved modes k >= 4 (eq. lco_update and
 *      eq. stochupdaterule1 with m-hat = m / sqrt(w_k mu rho),
 *      eq. normalized_mk):
 *        m*_k = m^eq_k + gamma_k (m_k - m^eq_k)
 *               + sqrt(w_k mu rho_n) sqrt(1 - gamma_k^2) r_k,
 *      mu = kT / c_s^2 (eq. EOS2 and the kT = mu b^3 c_s^2 relation), with
 *      r_k the unit Gaussians g[k-4]; the conserved modes are unchanged;
 *   4. back-transformation to populations;
 *   5. add the forcing term Delta''_i of Sec. "External forces" with the
 *      second moment Sigma of eq. moment_two_external_force.
 * `g` may be NULL when kT = 0.  The result is written to nstar. */
void orc_collide_site(const orc_params *p, const double n[Q], const double F[3], const double *gnoise,
                      double nstar[Q])
{
    init_tables();
    double gam[Q];
    mode_gammas(p, gam);

    double m[Q];
    orc_moments_site(n, m);
    const double rho = m[0];
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = (m[1 + a] + 0.5 * F[a]) / rho;

    double neq[Q], meq[Q];
    orc_equilibrium(rho, u, neq);
    orc_moments_site(neq, meq);

    const double mu = p->kT / CS2;
    const double rho_n = p->noise_rho0 ? p->rho0 : rho;
    double mstar[Q];
    for (int k = 0; k < Q; ++k) {
        if (k < 4) {
            mstar[k] = m[k];
            continue;
        }
        mstar[k] = meq[k] + gam[k] * (m[k] - meq[k]);
        if (p->kT > 0.0) {
            const double phi = sqrt(1.0 - gam[k] * gam[k]);
            mstar[k] += sqrt(WK[k] * mu * rho_n) * phi * gnoise[k - 4];
        }
    }
    orc_back_site(mstar, nstar);

    /* Forcing term Delta''_i (Sec. "External forces", h = 1). */
    const double uf = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    double sig[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            const double dab = (a == b) ? 1.0 : 0.0;
            sig[a][b] = 0.5 * (1.0 + p->gamma_shear) * (u[a] * F[b] + u[b] * F[a] - (2.0 / 3.0) * uf * dab) +
                        (1.0 / 3.0) * (1.0 + p->gamma_bulk) * uf * dab;
        }
    for (int i = 0; i < Q; ++i) {
        double fc = 0.0, sc = 0.0;
        for (int a = 0; a < 3; ++a) {
            fc += F[a] * CV[i][a];
            for (int b = 0; b < 3; ++b) {
                const double dab = (a == b) ? 1.0 : 0.0;
                sc += sig[a][b] * (CV[i][a] * CV[i][b] - CS2 * dab);
            }
        }
        nstar[i] += A[i] * (fc / CS2 + sc / (2.0 * CS2 * CS2));
    }
}

/* ------------------------------------------------------------------------ */
/* Whole-lattice operations                                                  */
/* ------------------------------------------------------------------------ */

static int64_t site_index(const orc_params *p, int x, int y, int z)
{
    return (int64_t)x + (int64_t)p->nx * ((int64_t)y + (int64_t)p->ny * (int64_t)z);
}

static int wrap(int v, int n)
{
    int r = v % n;
    return r < 0 ? r + n : r;
}

/* Initialise every site to n^eq(rho(r), u(r)).  rho may be NULL (rho0);
 * u may be NULL (rest).  u is laid out [3][N]. */
void orc_init_equilibrium(const orc_params *p, const double *rho, const double *u, double *n)
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    for (int64_t s = 0; s < N; ++s) {
        const double r = rho ? rho[s] : p->rho0;
        double v[3] = {0.0, 0.0, 0.0};
        if (u)
            for (int a = 0; a < 3; ++a) v[a] = u[a * N + s];
        double neq[Q];
        orc_equilibrium(r, v, neq);
        for (int i = 0; i < Q; ++i) n[i * N + s] = neq[i];
    }
}

/* One lattice-Boltzmann time step, eq. LBE: collide at every site with force
 * density g + extra(r) (extra may be NULL, layout [3][N]), then stream
 * n_i(r + c_i, t+1) = n*_i(r, t) with periodic wrap.  With walls, a
 * population whose link crosses a wall returns to its own site reversed,
 * n_{-i}(r, t+1) = n*_i(r, t) (eq. MBB with a wall at rest, u_b = 0, the wall
 * half way along the link).  `step` keys the noise.
 * `work` is caller scratch of 19*N doubles.  Parity pinned by the shear-wave,
 * Kolmogorov, conservation and noise-variance tests. */
void orc_step(const orc_params *p, double *n, double *work, const double *extra, uint32_t step)
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; ++s) {
        double ns[Q], nst[Q], F[3], gn[16];
        for (int i = 0; i < Q; ++i) ns[i] = n[i * N + s];
        for (int a = 0; a < 3; ++a) F[a] = p->g[a] + (extra ? extra[a * N + s] : 0.0);
        if (p->kT > 0.0) orc_fluid_normals(p->seed, (uint32_t)s, step, p->box, gn);
        orc_collide_site(p, ns, F, gn, nst);
        for (int i = 0; i < Q; ++i) work[i * N + s] = nst[i];
    }
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                const int64_t s = site_index(p, x, y, z);
                for (int i = 0; i < Q; ++i) {
                    if (crosses_wall(p, z, i)) {
                        n[opposite(i) * N + s] = work[i * N + s];
                        continue;
                    }
                    const int64_t d = site_index(p, wrap(x + CV[i][0], p->nx), wrap(y + CV[i][1], p->ny),
                                                 wrap(z + CV[i][2], p->nz));
                    n[i * N + d] = work[i * N + s];
                }
            }
}

/* nsteps consecutive steps starting at step counter `step0`, no particles. */
void orc_run(const orc_params *p, double *n, int32_t nsteps, uint32_t step0)
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    double *work = (double *)malloc(sizeof(double) * Q * (size_t)N);
    for (int32_t t = 0; t < nsteps; ++t) orc_step(p, n, work, NULL, step0 + (uint32_t)t);
    free(work);
}

/* Density and velocity at every site: rho = sum n, u = (sum n c + g/2)/rho
 * (eq. special_choice_momentum_density with the uniform body force only).
 * u is laid out [3][N]. */
void orc_fields(const orc_params *p, const double *n, double *rho, double *u)
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    for (int64_t s = 0; s < N; ++s) {
        double r = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q; ++i) {
            const double v = n[i * N + s];
            r += v;
            for (int a = 0; a < 3; ++a) j[a] += v * CV[i][a];
        }
        rho[s] = r;
        for (int a = 0; a < 3; ++a) u[a * N + s] = (j[a] + 0.5 * p->g[a]) / r;
    }
}

/* Total mass and momentum: out = {sum rho, sum j_x, sum j_y, sum j_z}, with
 * j = sum_i n_i c_i (no force shift). */
void orc_totals(const orc_params *p, const double *n, double out[4])
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    double M = 0.0, P[3] = {0.0, 0.0, 0.0};
    for (int64_t s = 0; s < N; ++s)
        for (int i = 0; i < Q; ++i) {
            const double v = n[i * N + s];
            M += v;
            for (int a = 0; a < 3; ++a) P[a] += v * CV[i][a];
        }
    out[0] = M;
    out[1] = P[0];
    out[2] = P[1];
    out[3] = P[2];
}

/* All 19 moments at every site, layout [19][N]. */
void orc_mode_field(const orc_params *p, const double *n, double *m)
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    for (int64_t s = 0; s < N; ++s) {
        double ns[Q], ms[Q];
        for (int i = 0; i < Q; ++i) ns[i] = n[i * N + s];
        orc_moments_site(ns, ms);
        for (int k = 0; k < Q; ++k) m[k * N + s] = ms[k];
    }
}

/* Lowest transverse Fourier amplitudes of the momentum density
 * j(r) = sum_i c_i n_i(r) of the populations n at the start of a step (the
 * momentum that step's collision sees and keeps).  For each axis a,
 * k = 2 pi / L_a and the two components c normal to a,
 *   j_hat_c(k) = sum_r j_c(r) exp(-i k r_a),
 * the shear modes whose decay (eq. LBE at gamma = 0) and equal-time variance
 * (the equipartition of eq. Pdistneq) the batch form's ensemble VACF
 * samples.  out[12]: (re, im) of (k along z: j_x, j_y), (k along y: j_x,
 * j_z), (k along x: j_y, j_z).  Plain sums over the sites. */
void orc_transverse_modes(const orc_params *p, const double *n, double out[12])
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    const double two_pi = 6.283185307179586476925286766559;
    for (int k = 0; k < 12; ++k) out[k] = 0.0;
    for (int64_t s = 0; s < N; ++s) {
        const int64_t x = s % p->nx, y = (s / p->nx) % p->ny, z = s / ((int64_t)p->nx * p->ny);
        double j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q; ++i)
            for (int a = 0; a < 3; ++a) j[a] += n[i * N + s] * CV[i][a];
        const double fz = two_pi * (double)z / (double)p->nz;
        const double fy = two_pi * (double)y / (double)p->ny;
        const double fx = two_pi * (double)x / (double)p->nx;
        /* exp(-i phi) = cos phi - i sin phi */
        out[0] += j[0] * cos(fz);
        out[1] -= j[0] * sin(fz);
        out[2] += j[1] * cos(fz);
        out[3] -= j[1] * sin(fz);
        out[4] += j[0] * cos(fy);
        out[5] -= j[0] * sin(fy);
        out[6] += j[2] * cos(fy);
        out[7] -= j[2] * sin(fy);
        out[8] += j[1] * cos(fx);
        out[9] -= j[1] * sin(fx);
        out[10] += j[2] * cos(fx);
        out[11] -= j[2] * sin(fx);
    }
}

/* ------------------------------------------------------------------------ */
/* Point-particle coupling (Sec. "Force coupling", "Interpolating functions")*/
/* ------------------------------------------------------------------------ */

/* Interpolation kernels phi_W of eq. 2point, eq. 3point and eq. 4point
 * (W = 2, 3, 4 points per axis) and their derivatives (phi_3 and phi_4 have
 * continuous first derivatives; phi_2 is differentiated away from the
 * nodes). */
static double phi2(double r)
{
    const double a = fabs(r);
    return a < 1.0 ? 1.0 - a : 0.0;
}

static double phi3(double r)
{
    const double a = fabs(r);
    if (a <= 0.5) return (1.0 + sqrt(1.0 - 3.0 * r * r)) / 3.0;
    if (a <= 1.5) return (5.0 - 3.0 * a - sqrt(-2.0 + 6.0 * a - 3.0 * r * r)) / 6.0;
    return 0.0;
}

static double phi4(double r)
{
    const double a = fabs(r);
    if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * r * r)) / 8.0;
    if (a <= 2.0) return (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * r * r)) / 8.0;
    return 0.0;
}

static double dphi2(double r)
{
    if (r <= -1.0 || r >= 1.0) return 0.0;
    return r > 0.0 ? -1.0 : 1.0;
}

static double dphi3(double r)
{
    const double a = fabs(r), sg = r < 0.0 ? -1.0 : 1.0;
    if (a <= 0.5) return -r / sqrt(1.0 - 3.0 * r * r);
    if (a <= 1.5) return sg * (-0.5 - (1.0 - a) / (2.0 * sqrt(-2.0 + 6.0 * a - 3.0 * r * r)));
    return 0.0;
}

static double dphi4(double r)
{
    const double a = fabs(r), sg = r < 0.0 ? -1.0 : 1.0;
    if (a <= 1.0) return sg * (-2.0 + (4.0 - 8.0 * a) / (2.0 * sqrt(1.0 + 4.0 * a - 4.0 * r * r))) / 8.0;
    if (a <= 2.0) return sg * (-2.0 - (12.0 - 8.0 * a) / (2.0 * sqrt(-7.0 + 12.0 * a - 4.0 * r * r))) / 8.0;
    return 0.0;
}

static double phi_w(int W, double r) { return W == 3 ? phi3(r) : (W == 4 ? phi4(r) : phi2(r)); }
static double dphi_w(int W, double r) { return W == 3 ? dphi3(r) : (W == 4 ? dphi4(r) : dphi2(r)); }

/* First node of the W-point stencil along one axis: every node within the
 * kernel's support, floor(R) for W = 2, the nearest node minus one for
 * W = 3, floor(R) - 1 for W = 4. */
static double stencil_first(int W, double R)
{
    if (W == 3) return floor(R + 0.5) - 1.0;
    if (W == 4) return floor(R) - 1.0;
    return floor(R);
}

/* The W^3 lattice nodes around position R (periodic box, x fastest) and
 * their weights Delta(r - R) = phi_W(x) phi_W(y) phi_W(z) (eq. Delta); with
 * dw != NULL also d Delta / d R.  Nodes sit at integer coordinates.
 * Returns W^3. */
int orc_stencil_w(const orc_params *p, const double R[3], int32_t W, int64_t *node, double *wgt, double *dw)
{
    const int L[3] = {p->nx, p->ny, p->nz};
    double first[3];
    for (int a = 0; a < 3; ++a) first[a] = stencil_first(W, R[a]);
    int q = 0;
    for (int dz = 0; dz < W; ++dz)
        for (int dy = 0; dy < W; ++dy)
            for (int dx = 0; dx < W; ++dx) {
                const double c[3] = {first[0] + dx, first[1] + dy, first[2] + dz};
                int idx[3];
                double f[3], d[3];
                for (int a = 0; a < 3; ++a) {
                    const double m = c[a] - (double)L[a] * floor(c[a] / (double)L[a]);
                    idx[a] = wrap((int)m, L[a]);
                    f[a] = phi_w(W, R[a] - c[a]);
                    d[a] = dphi_w(W, R[a] - c[a]);
                }
                node[q] = site_index(p, idx[0], idx[1], idx[2]);
                wgt[q] = f[0] * f[1] * f[2];
                if (dw) {
                    dw[3 * q + 0] = d[0] * f[1] * f[2];
                    dw[3 * q + 1] = f[0] * d[1] * f[2];
                    dw[3 * q + 2] = f[0] * f[1] * d[2];
                }
                ++q;
            }
    return q;
}

/* The 8-node two-point stencil (orc_stencil_w with W = 2). */
void orc_stencil(const orc_params *p, const double R[3], int64_t node[8], double wgt[8])
{
    orc_stencil_w(p, R, 2, node, wgt, NULL);
}

/* One 1-D kernel value phi_W(r) and derivative (for the kernel pins). */
void orc_phi(int32_t W, double r, double out[2])
{
    out[0] = phi_w(W, r);
    out[1] = dphi_w(W, r);
}

/* Bead set of the particle half: masses, frictions, bonds (pairs (a,b),
 * d = R_b - R_a) that are either harmonic, V = (k/2)(|d| - r0)^2, or FENE
 * (eq. ufene), V = -(k/2) R0^2 ln(1 - |d|^2/R0^2) with R0 = r0; the purely
 * repulsive Lennard-Jones (WCA) interaction of eq. ulennardjones between all
 * pairs (off when wca_eps = 0); the interpolation kernel's width and an
 * optional external force per bead (added to the conservative force,
 * constant in time). */
typedef struct {
    int32_t n, nbonds;
    const double *mass, *zeta;
    const int32_t *bonds;
    double kbond, r0;
    int32_t stencil;      /* 2, 3 or 4: phi_2 (8 nodes), phi_3 (27), phi_4 (64) */
    int32_t fene;         /* 0: harmonic bonds, 1: FENE bonds */
    const double *fext;   /* [n][3] or NULL */
    double wca_eps, wca_sigma;
    int32_t three_point;  /* bead noise: 0 unit Gaussians, 1 the three-point variates */
} orc_beadset;

/* The bead noise theta of eq. langevin_momentum_update for bead b at `step`. */
static void bead_noise(const orc_params *p, const orc_beadset *bs, int b, uint32_t step, double th[3])
{
    if (bs->three_point)
        orc_bead_three_point(p->seed, (uint32_t)b, step, p->box, th);
    else
        orc_bead_normals(p->seed, (uint32_t)b, step, p->box, th);
}

static int bs_width(const orc_beadset *bs) { return (bs->stencil == 3 || bs->stencil == 4) ? bs->stencil : 2; }

/* WCA force on bead j from bead i, F_j = -dV/dR_j for eq. ulennardjones:
 * d = R_j - R_i (minimum image), f(r) d with f = 24 eps (2 (s/r)^12 - (s/r)^6)
 * / r^2 below the cutoff 2^(1/6) s, zero above. */
static double wca_factor(double eps, double sigma, double r2)
{
    const double rc2 = pow(2.0, 1.0 / 3.0) * sigma * sigma;
    if (r2 >= rc2) return 0.0;
    const double s6 = pow(sigma * sigma / r2, 3.0);
    return 24.0 * eps * (2.0 * s6 * s6 - s6) / r2;
}

/* Minimum-image difference along one periodic axis of length L. */
static double min_image(double d, double L) { return d - L * floor(d / L + 0.5); }

/* Pair separation along axis a: the minimum image along periodic axes; with
 * walls the z axis is not periodic and the plain difference is used. */
static double pair_sep(const orc_params *p, int a, double d, double L)
{
    return (a == 2 && p->walls) ? d : min_image(d, L);
}

/* Half-step positions R' = R + (h/2) P/m and conservative forces at R':
 * bonds (harmonic or FENE), WCA between all pairs (minimum image along the
 * periodic axes; with walls z is not periodic), plus the external force.  A FENE bond stretched to
 * |d| >= R0 has no finite force (NaN). */
static void half_and_forces(const orc_params *p, const orc_beadset *bs, const double *pos, const double *mom,
                            double *half, double *fc)
{
    const double h = 1.0;
    const double Lb[3] = {(double)p->nx, (double)p->ny, (double)p->nz};
    for (int b = 0; b < bs->n; ++b)
        for (int a = 0; a < 3; ++a) {
            half[3 * b + a] = pos[3 * b + a] + 0.5 * h * mom[3 * b + a] / bs->mass[b];
            fc[3 * b + a] = bs->fext ? bs->fext[3 * b + a] : 0.0;
        }
    for (int q = 0; q < bs->nbonds; ++q) {
        const int ia = bs->bonds[2 * q], ib = bs->bonds[2 * q + 1];
        double d[3], r2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            d[a] = half[3 * ib + a] - half[3 * ia + a];
            r2 += d[a] * d[a];
        }
        double mag;
        if (bs->fene) {
            const double R02 = bs->r0 * bs->r0;
            mag = r2 < R02 ? -bs->kbond / (1.0 - r2 / R02) : NAN;
        } else {
            const double r = sqrt(r2);
            if (r == 0.0) continue;
            mag = -bs->kbond * (r - bs->r0) / r;
        }
        for (int a = 0; a < 3; ++a) {
            fc[3 * ib + a] += mag * d[a];
            fc[3 * ia + a] -= mag * d[a];
        }
    }
    if (bs->wca_eps > 0.0)
        for (int i = 0; i < bs->n; ++i)
            for (int j = i + 1; j < bs->n; ++j) {
                double d[3], r2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    d[a] = pair_sep(p, a, half[3 * j + a] - half[3 * i + a], Lb[a]);
                    r2 += d[a] * d[a];
                }
                const double f = wca_factor(bs->wca_eps, bs->wca_sigma, r2);
                if (f == 0.0) continue;
                for (int a = 0; a < 3; ++a) {
                    fc[3 * j + a] += f * d[a];
                    fc[3 * i + a] -= f * d[a];
                }
            }
}

/* Conservative forces (bonds, WCA, external) at given positions, for the
 * pins of the interaction potentials. */
void orc_bead_forces(const orc_params *p, const orc_beadset *bs, const double *R, double *fc)
{
    const size_t nb3 = 3 * (size_t)(bs->n > 0 ? bs->n : 1);
    double *zero = (double *)calloc(nb3, sizeof(double));
    double *half = (double *)malloc(sizeof(double) * nb3);
    half_and_forces(p, bs, R, zero, half, fc);
    free(zero);
    free(half);
}

/* Momentum-update constants of eq. langevin_momentum_update. */
static void ou_constants(double m, double z, double kT, double *C1, double *C2, double *C3)
{
    const double h = 1.0;
    if (z > 0.0) {
        *C1 = exp(-z * h / m);
        *C2 = (m / z) * (1.0 - *C1);
        *C3 = sqrt(m * kT * (1.0 - exp(-2.0 * z * h / m)));
    } else {
        *C1 = 1.0;
        *C2 = h;
        *C3 = 0.0;
    }
}

/* u = (sum n c + g/2) / rho at one site of the pre-collision state. */
static void site_velocity(const orc_params *p, const double *n, int64_t N, int64_t s, double *rho, double u[3])
{
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        const double v = n[i * N + s];
        r += v;
        for (int a = 0; a < 3; ++a) j[a] += v * CV[i][a];
    }
    *rho = r;
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * p->g[a]) / r;
}

/* Particle half of one coupled time step (Sec. "Force coupling": the
 * Trotter splitting eq. pTrotter, the momentum update
 * eq. langevin_momentum_update, the interpolation eq. ufluid_discrete and
 * the reaction force eq. ftotal):
 *   1. R' = R + (h/2) P/m for every bead;
 *   2. conservative forces F^c at R': harmonic bonds plus the external force;
 *   3. u_b = sum over the W^3 nodes of Delta * u(node), u(node) from the
 *      current (pre-collision) populations n: u = (sum n c + g/2)/rho;
 *   4. P'' = C1 P + C2 (F^c + zeta u_b) + C3 theta, with
 *      C1 = exp(-zeta h/m), C2 = (m/zeta)(1 - C1),
 *      C3 = sqrt(m kT (1 - exp(-2 zeta h/m))), theta unit Gaussians or,
 *      with three_point set, the three-point variates;
 *   5. the fluid receives the momentum the bead exchanged with it,
 *      I = -(P'' - P - h F^c), spread as force density I Delta / h into
 *      `force` (layout [3][N], accumulated);
 *   6. R = R' + (h/2) P''/m, P = P''.
 * pos, mom: [3*n] interleaved (x,y,z per bead), unwrapped positions.
 * `step` keys the bead noise.  Parity pinned by the frozen-fluid OU tests,
 * the partition-of-unity and transpose tests, and the total-momentum test. */
void orc_couple(const orc_params *p, const double *n, uint32_t step, const orc_beadset *bs, double *pos, double *mom,
                double *force)
{
    init_tables();
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    const double h = 1.0;
    const int nb = bs->n, W = bs_width(bs);
    const size_t nb3 = 3 * (size_t)(nb > 0 ? nb : 1);
    double *half = (double *)malloc(sizeof(double) * nb3);
    double *fc = (double *)malloc(sizeof(double) * nb3);
    half_and_forces(p, bs, pos, mom, half, fc);
    for (int b = 0; b < nb; ++b) {
        int64_t node[64];
        double wgt[64];
        const int nq = orc_stencil_w(p, &half[3 * b], W, node, wgt, NULL);
        double ub[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < nq; ++q) {
            double r, u[3];
            site_velocity(p, n, N, node[q], &r, u);
            for (int a = 0; a < 3; ++a) ub[a] += wgt[q] * u[a];
        }
        const double m = bs->mass[b], z = bs->zeta[b];
        double C1, C2, C3;
        ou_constants(m, z, p->kT, &C1, &C2, &C3);
        double th[3] = {0.0, 0.0, 0.0};
        if (p->kT > 0.0 && z > 0.0) bead_noise(p, bs, b, step, th);
        double Pn[3], I[3];
        for (int a = 0; a < 3; ++a) {
            Pn[a] = C1 * mom[3 * b + a] + C2 * (fc[3 * b + a] + z * ub[a]) + C3 * th[a];
            I[a] = -(Pn[a] - mom[3 * b + a] - h * fc[3 * b + a]);
        }
        for (int q = 0; q < nq; ++q)
            for (int a = 0; a < 3; ++a) force[a * N + node[q]] += wgt[q] * I[a] / h;
        for (int a = 0; a < 3; ++a) {
            mom[3 * b + a] = Pn[a];
            pos[3 * b + a] = half[3 * b + a] + 0.5 * h * Pn[a] / m;
        }
    }
    free(half);
    free(fc);
}

/* One full coupled step (particle update, spreading, then one LB step with
 * the spread force in the collision).  `work` is 19*N doubles and `force`
 * is 3*N doubles of caller scratch. */
void orc_coupled_step(const orc_params *p, double *n, double *work, double *force, uint32_t step,
                      const orc_beadset *bs, double *pos, double *mom)
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    memset(force, 0, sizeof(double) * 3 * (size_t)N);
    orc_couple(p, n, step, bs, pos, mom, force);
    orc_step(p, n, work, force, step);
}

/* ------------------------------------------------------------------------ */
/* Adjoint (reverse mode) of the fluid step                                  */
/* ------------------------------------------------------------------------ */

/* Transpose of the Jacobian of orc_collide_site with respect to the
 * pre-collision populations n and the force density F, applied to nbs (the
 * adjoint of n*).  The steps of orc_collide_site are taken back in reverse
 * order (forcing term, back-transformation, relaxation + noise, equilibrium,
 * velocity, moments).  The noise variates g are replayed: only the
 * sqrt(rho) amplitude of the local-density noise depends on the state.
 * Outputs: nb (adjoint of n, overwritten), Fb (adjoint of F, accumulated).
 * Parity pinned by central finite differences of orc_collide_site. */
void orc_collide_site_adjoint(const orc_params *p, const double n[Q], const double F[3], const double *gnoise,
                              const double nbs[Q], double nb[Q], double Fb[3])
{
    init_tables();
    double gam[Q];
    mode_gammas(p, gam);

    /* forward quantities */
    double m[Q];
    orc_moments_site(n, m);
    const double rho = m[0];
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = (m[1 + a] + 0.5 * F[a]) / rho;
    const double uf = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    (void)uf;

    double ub[3] = {0.0, 0.0, 0.0};
    double rhob = 0.0;

    /* 5. forcing term Delta''_i = a_i (F.c_i / cs2 + Sigma : (c c - cs2 I) / (2 cs4)) */
    double Sb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int i = 0; i < Q; ++i)
        for (int a = 0; a < 3; ++a) {
            Fb[a] += nbs[i] * A[i] * CV[i][a] / CS2;
            for (int b = 0; b < 3; ++b) {
                const double dab = (a == b) ? 1.0 : 0.0;
                Sb[a][b] += nbs[i] * A[i] * (CV[i][a] * CV[i][b] - CS2 * dab) / (2.0 * CS2 * CS2);
            }
        }
    /* Sigma = As (u F + F u - (2/3) u.F I) + (1/3)(1 + gamma_bulk) u.F I */
    const double As = 0.5 * (1.0 + p->gamma_shear);
    const double Bs = -(2.0 / 3.0) * As + (1.0 / 3.0) * (1.0 + p->gamma_bulk);
    const double trSb = Sb[0][0] + Sb[1][1] + Sb[2][2];
    for (int g = 0; g < 3; ++g) {
        double sF = 0.0, sTF = 0.0, su = 0.0, sTu = 0.0;
        for (int a = 0; a < 3; ++a) {
            sF += Sb[g][a] * F[a];
            sTF += Sb[a][g] * F[a];
            su += Sb[g][a] * u[a];
            sTu += Sb[a][g] * u[a];
        }
        ub[g] += As * (sF + sTF) + Bs * F[g] * trSb;
        Fb[g] += As * (su + sTu) + Bs * u[g] * trSb;
    }

    /* 4. back-transformation n_pre_i = a_i sum_k e_ki m*_k / w_k */
    double msb[Q];
    for (int k = 0; k < Q; ++k) {
        double s = 0.0;
        for (int i = 0; i < Q; ++i) s += A[i] * E[k][i] * nbs[i];
        msb[k] = s / WK[k];
    }

    /* 3. relaxation + noise */
    double mb[Q], meqb[Q];
    for (int k = 0; k < Q; ++k) {
        meqb[k] = 0.0;
        if (k < 4) {
            mb[k] = msb[k];
            continue;
        }
        mb[k] = gam[k] * msb[k];
        meqb[k] = (1.0 - gam[k]) * msb[k];
        if (p->kT > 0.0 && !p->noise_rho0) {
            const double mu = p->kT / CS2;
            const double phi = sqrt(1.0 - gam[k] * gam[k]);
            rhob += msb[k] * sqrt(WK[k] * mu) * phi * gnoise[k - 4] * 0.5 / sqrt(rho);
        }
    }

    /* 2. equilibrium moments m^eq = E n^eq(rho, u) */
    for (int i = 0; i < Q; ++i) {
        double neqb = 0.0;
        for (int k = 4; k < Q; ++k) neqb += E[k][i] * meqb[k];
        const double uc = u[0] * CV[i][0] + u[1] * CV[i][1] + u[2] * CV[i][2];
        rhob += neqb * A[i] * (1.0 + uc / CS2 + uc * uc / (2.0 * CS2 * CS2) - usq / (2.0 * CS2));
        for (int a = 0; a < 3; ++a)
            ub[a] += neqb * A[i] * rho * (CV[i][a] / CS2 + uc * CV[i][a] / (CS2 * CS2) - u[a] / CS2);
    }

    /* 1. u = (m_{1..3} + F/2) / rho, rho = m_0 */
    for (int a = 0; a < 3; ++a) {
        mb[1 + a] += ub[a] / rho;
        Fb[a] += 0.5 * ub[a] / rho;
        rhob -= ub[a] * u[a] / rho;
    }
    mb[0] += rhob;

    /* 0. m = E n */
    for (int i = 0; i < Q; ++i) {
        double s = 0.0;
        for (int k = 0; k < Q; ++k) s += E[k][i] * mb[k];
        nb[i] = s;
    }
}

/* Adjoint of one orc_step.  n: pre-collision state at step `step`;
 * lam: on entry the adjoint of the state after the step (pre-collision at
 * step+1), on exit the adjoint of n.  Streaming n_i(r + c_i) = n*_i(r) is a
 * permutation, so the adjoint of n* at r is lam_i(r + c_i), or lam_{-i}(r)
 * where the link crosses a wall.  extra: the
 * extra force field of the step or NULL; its adjoint is accumulated into
 * extra_bar ([3][N]) when not NULL.  gbar accumulates the adjoint of the
 * uniform body force.  work: 19*N doubles of caller scratch. */
void orc_step_adjoint(const orc_params *p, const double *n, double *lam, double *work, const double *extra,
                      double *extra_bar, uint32_t step, double gbar[3])
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    double gsum[3] = {0.0, 0.0, 0.0};
#pragma omp parallel
    {
        double gloc[3] = {0.0, 0.0, 0.0};
#pragma omp for schedule(static)
        for (int z = 0; z < p->nz; ++z)
            for (int y = 0; y < p->ny; ++y)
                for (int x = 0; x < p->nx; ++x) {
                    const int64_t s = site_index(p, x, y, z);
                    double ns[Q], nbs[Q], nb[Q], F[3], Fb[3] = {0.0, 0.0, 0.0}, gn[16];
                    for (int i = 0; i < Q; ++i) {
                        ns[i] = n[i * N + s];
                        if (crosses_wall(p, z, i)) {
                            nbs[i] = lam[opposite(i) * N + s];
                            continue;
                        }
                        const int64_t d = site_index(p, wrap(x + CV[i][0], p->nx), wrap(y + CV[i][1], p->ny),
                                                     wrap(z + CV[i][2], p->nz));
                        nbs[i] = lam[i * N + d];
                    }
                    for (int a = 0; a < 3; ++a) F[a] = p->g[a] + (extra ? extra[a * N + s] : 0.0);
                    if (p->kT > 0.0) orc_fluid_normals(p->seed, (uint32_t)s, step, p->box, gn);
                    orc_collide_site_adjoint(p, ns, F, gn, nbs, nb, Fb);
                    for (int i = 0; i < Q; ++i) work[i * N + s] = nb[i];
                    for (int a = 0; a < 3; ++a) {
                        gloc[a] += Fb[a];
                        if (extra_bar) extra_bar[a * N + s] += Fb[a];
                    }
                }
#pragma omp critical
        for (int a = 0; a < 3; ++a) gsum[a] += gloc[a];
    }
    memcpy(lam, work, sizeof(double) * Q * (size_t)N);
    for (int a = 0; a < 3; ++a) gbar[a] += gsum[a];
}

/* Reverse-mode gradient of a loss of the state after nsteps fluid steps
 * (no particles), starting from n0 at step counter step0.  lam: on entry
 * dL/dn(T), on exit dL/dn(0).  gbar: dL/dg (uniform body force) through the
 * dynamics, accumulated.  Stores all intermediate states (plain and slow). */
void orc_backward(const orc_params *p, const double *n0, int32_t nsteps, uint32_t step0, double *lam, double gbar[3])
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    const size_t sz = sizeof(double) * Q * (size_t)N;
    double *states = (double *)malloc(sz * (size_t)(nsteps > 0 ? nsteps : 1));
    double *work = (double *)malloc(sz);
    memcpy(states, n0, sz);
    for (int32_t t = 0; t + 1 < nsteps; ++t) {
        memcpy(states + (size_t)(t + 1) * Q * N, states + (size_t)t * Q * N, sz);
        orc_step(p, states + (size_t)(t + 1) * Q * N, work, NULL, step0 + (uint32_t)t);
    }
    for (int32_t t = nsteps - 1; t >= 0; --t)
        orc_step_adjoint(p, states + (size_t)t * Q * N, lam, work, NULL, NULL, step0 + (uint32_t)t, gbar);
    free(work);
    free(states);
}

/* ------------------------------------------------------------------------ */
/* Adjoint (reverse mode) of the particle half of a coupled step             */
/* ------------------------------------------------------------------------ */

/* Transpose of the Jacobian of orc_couple (with its bead noise replayed).
 * Inputs: the fluid state n and bead state (pos, mom) the step started
 * from, and force_bar ([3][N]), the adjoint of the spread force field
 * (from orc_step_adjoint's extra_bar).  pos_bar, mom_bar: on entry the
 * adjoints of the bead state after the step, on exit those of the state
 * before it.  lam ([19][N], the adjoint of n) and gbar accumulate the
 * contributions of the interpolated velocity u = (sum n c + g/2)/rho.
 * The forward map is retraced in reverse: R = R' + (h/2)P''/m, the reaction
 * I = -(P'' - P - h F^c) spread with the weights Delta(R'), the momentum
 * update P'' = C1 P + C2 (F^c + zeta u_b), the interpolation
 * u_b = sum Delta u(node), the bond forces F^c(R') and the half drift
 * R' = R + (h/2) P/m.  The weights are differentiated with the kernels'
 * derivatives (phi_2: where R' is off the node planes).  The external force
 * is constant and has no adjoint.  Conservative forces F = mag(r^2) d along
 * a separation d (bonds: d = R'_b - R'_a; WCA pairs: R'_j - R'_i at the
 * minimum image along periodic axes) have the symmetric Jacobian dF/dd = mag I + 2 mag'(r^2) d d^T:
 *   harmonic  mag = -k (r - r0)/r,           2 mag' = -k r0 / r^3
 *   FENE      mag = -k / (1 - r^2/R0^2),     2 mag' = -2 k / (R0^2 (1 - r^2/R0^2)^2)
 *   WCA       mag = 24 eps (2 s^2 - s)/r^2,  2 mag' = 24 eps (-28 s^2 + 8 s) / r^4,
 *             s = (sigma^2/r^2)^3, below the cutoff (zero above).
 * Parity pinned by central finite differences of the coupled forward map. */
void orc_couple_adjoint(const orc_params *p, const double *n, uint32_t step, const orc_beadset *bs,
                        const double *pos, const double *mom, const double *force_bar, double *pos_bar,
                        double *mom_bar, double *lam, double gbar[3])
{
    init_tables();
    (void)step;
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    const double h = 1.0;
    const int nb = bs->n, W = bs_width(bs);
    const size_t nb3 = 3 * (size_t)(nb > 0 ? nb : 1);
    double *half = (double *)malloc(sizeof(double) * nb3);
    double *fc = (double *)malloc(sizeof(double) * nb3);
    double *half_bar = (double *)calloc(nb3, sizeof(double));
    double *fc_bar = (double *)calloc(nb3, sizeof(double));
    double *p_bar = (double *)calloc(nb3, sizeof(double));
    half_and_forces(p, bs, pos, mom, half, fc);

    for (int b = 0; b < nb; ++b) {
        const double m = bs->mass[b], z = bs->zeta[b];
        int64_t node[64];
        double wgt[64], dw[192], un[64][3], rn[64];
        const int nq = orc_stencil_w(p, &half[3 * b], W, node, wgt, dw);
        double ub[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < nq; ++q) {
            site_velocity(p, n, N, node[q], &rn[q], un[q]);
            for (int a = 0; a < 3; ++a) ub[a] += wgt[q] * un[q][a];
        }
        double C1, C2, C3;
        ou_constants(m, z, p->kT, &C1, &C2, &C3);
        double th[3] = {0.0, 0.0, 0.0};
        if (p->kT > 0.0 && z > 0.0) bead_noise(p, bs, b, step, th);
        double I[3];
        for (int a = 0; a < 3; ++a) {
            const double Pn = C1 * mom[3 * b + a] + C2 * (fc[3 * b + a] + z * ub[a]) + C3 * th[a];
            I[a] = -(Pn - mom[3 * b + a] - h * fc[3 * b + a]);
        }

        /* reverse: R_new = R' + (h/2) P''/m, P_new = P'' */
        double Pn_bar[3], I_bar[3] = {0.0, 0.0, 0.0}, ub_bar[3];
        for (int a = 0; a < 3; ++a) {
            half_bar[3 * b + a] = pos_bar[3 * b + a];
            Pn_bar[a] = mom_bar[3 * b + a] + 0.5 * h / m * pos_bar[3 * b + a];
        }
        /* force[node] += Delta I / h */
        for (int q = 0; q < nq; ++q)
            for (int a = 0; a < 3; ++a) I_bar[a] += wgt[q] * force_bar[a * N + node[q]] / h;
        double wgt_bar[64];
        for (int q = 0; q < nq; ++q) {
            wgt_bar[q] = 0.0;
            for (int a = 0; a < 3; ++a) wgt_bar[q] += I[a] * force_bar[a * N + node[q]] / h;
        }
        /* I = -(P'' - P - h F^c) */
        for (int a = 0; a < 3; ++a) {
            Pn_bar[a] -= I_bar[a];
            p_bar[3 * b + a] = I_bar[a];
            fc_bar[3 * b + a] = h * I_bar[a];
        }
        /* P'' = C1 P + C2 (F^c + zeta u_b) + C3 theta */
        for (int a = 0; a < 3; ++a) {
            p_bar[3 * b + a] += C1 * Pn_bar[a];
            fc_bar[3 * b + a] += C2 * Pn_bar[a];
            ub_bar[a] = C2 * z * Pn_bar[a];
        }
        /* u_b = sum Delta u(node); u = (sum n c + g/2) / rho */
        for (int q = 0; q < nq; ++q) {
            double uq_bar[3];
            for (int a = 0; a < 3; ++a) {
                wgt_bar[q] += ub_bar[a] * un[q][a];
                uq_bar[a] = wgt[q] * ub_bar[a];
                gbar[a] += 0.5 * uq_bar[a] / rn[q];
            }
            for (int i = 0; i < Q; ++i) {
                double s = 0.0;
                for (int a = 0; a < 3; ++a) s += (CV[i][a] - un[q][a]) * uq_bar[a];
                lam[i * N + node[q]] += s / rn[q];
            }
        }
        /* the weights depend on R' */
        for (int q = 0; q < nq; ++q)
            for (int a = 0; a < 3; ++a) half_bar[3 * b + a] += wgt_bar[q] * dw[3 * q + a];
    }

    /* bond forces F_b = mag d, F_a = -mag d, d = R'_b - R'_a */
    for (int q = 0; q < bs->nbonds; ++q) {
        const int ia = bs->bonds[2 * q], ib = bs->bonds[2 * q + 1];
        double d[3], r2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            d[a] = half[3 * ib + a] - half[3 * ia + a];
            r2 += d[a] * d[a];
        }
        double mag, mag2p; /* mag and 2 dmag/d(r^2) */
        if (bs->fene) {
            const double x = r2 / (bs->r0 * bs->r0);
            mag = -bs->kbond / (1.0 - x);
            mag2p = -2.0 * bs->kbond / (bs->r0 * bs->r0 * (1.0 - x) * (1.0 - x));
        } else {
            const double r = sqrt(r2);
            if (r == 0.0) continue;
            mag = -bs->kbond * (r - bs->r0) / r;
            mag2p = -bs->kbond * bs->r0 / (r * r * r);
        }
        double v[3], dv = 0.0;
        for (int a = 0; a < 3; ++a) {
            v[a] = fc_bar[3 * ib + a] - fc_bar[3 * ia + a];
            dv += d[a] * v[a];
        }
        for (int a = 0; a < 3; ++a) {
            const double d_bar = mag * v[a] + mag2p * d[a] * dv;
            half_bar[3 * ib + a] += d_bar;
            half_bar[3 * ia + a] -= d_bar;
        }
    }

    /* WCA pairs F_j = mag d, F_i = -mag d, d = pair_sep of R'_j - R'_i */
    if (bs->wca_eps > 0.0) {
        const double Lb[3] = {(double)p->nx, (double)p->ny, (double)p->nz};
        const double rc2 = pow(2.0, 1.0 / 3.0) * bs->wca_sigma * bs->wca_sigma;
        for (int i = 0; i < nb; ++i)
            for (int j = i + 1; j < nb; ++j) {
                double d[3], r2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    d[a] = pair_sep(p, a, half[3 * j + a] - half[3 * i + a], Lb[a]);
                    r2 += d[a] * d[a];
                }
                if (r2 >= rc2) continue;
                const double s6 = pow(bs->wca_sigma * bs->wca_sigma / r2, 3.0);
                const double mag = 24.0 * bs->wca_eps * (2.0 * s6 * s6 - s6) / r2;
                const double mag2p = 24.0 * bs->wca_eps * (-28.0 * s6 * s6 + 8.0 * s6) / (r2 * r2);
                double v[3], dv = 0.0;
                for (int a = 0; a < 3; ++a) {
                    v[a] = fc_bar[3 * j + a] - fc_bar[3 * i + a];
                    dv += d[a] * v[a];
                }
                for (int a = 0; a < 3; ++a) {
                    const double d_bar = mag * v[a] + mag2p * d[a] * dv;
                    half_bar[3 * j + a] += d_bar;
                    half_bar[3 * i + a] -= d_bar;
                }
            }
    }

    /* R' = R + (h/2) P/m */
    for (int b = 0; b < nb; ++b)
        for (int a = 0; a < 3; ++a) {
            pos_bar[3 * b + a] = half_bar[3 * b + a];
            mom_bar[3 * b + a] = p_bar[3 * b + a] + 0.5 * h / bs->mass[b] * half_bar[3 * b + a];
        }
    free(half);
    free(fc);
    free(half_bar);
    free(fc_bar);
    free(p_bar);
}

/* Reverse-mode gradient through nsteps coupled steps (orc_coupled_step)
 * from n0 and the bead state (pos0, mom0) at step counter step0.
 * lam: on entry dL/dn(T), on exit dL/dn(0); pos_bar, mom_bar: on entry
 * dL/dR(T), dL/dP(T), on exit dL/dR(0), dL/dP(0); gbar accumulates dL/dg.
 * Per step, in reverse: the fluid step's adjoint (which also gives the
 * adjoint of the spread force at every site), then the particle half's.
 * Stores all intermediate states (plain and slow). */
void orc_backward_coupled(const orc_params *p, const double *n0, int32_t nsteps, uint32_t step0,
                          const orc_beadset *bs, const double *pos0, const double *mom0, double *lam, double gbar[3],
                          double *pos_bar, double *mom_bar)
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    const int nb = bs->n;
    const size_t sz = sizeof(double) * Q * (size_t)N;
    const size_t bsz = sizeof(double) * 3 * (size_t)(nb > 0 ? nb : 1);
    const size_t T = (size_t)(nsteps > 0 ? nsteps : 1);
    double *states = (double *)malloc(sz * T);
    double *bpos = (double *)malloc(bsz * T);
    double *bmom = (double *)malloc(bsz * T);
    double *work = (double *)malloc(sz);
    double *force = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    double *force_bar = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    double *tp = (double *)malloc(bsz), *tm = (double *)malloc(bsz);
    memcpy(states, n0, sz);
    memcpy(bpos, pos0, bsz);
    memcpy(bmom, mom0, bsz);
    for (int32_t t = 0; t + 1 < nsteps; ++t) {
        double *nt = states + (size_t)(t + 1) * Q * N;
        memcpy(nt, states + (size_t)t * Q * N, sz);
        memcpy(bpos + (size_t)(t + 1) * 3 * nb, bpos + (size_t)t * 3 * nb, bsz);
        memcpy(bmom + (size_t)(t + 1) * 3 * nb, bmom + (size_t)t * 3 * nb, bsz);
        orc_coupled_step(p, nt, work, force, step0 + (uint32_t)t, bs, bpos + (size_t)(t + 1) * 3 * nb,
                         bmom + (size_t)(t + 1) * 3 * nb);
    }
    for (int32_t t = nsteps - 1; t >= 0; --t) {
        const double *nt = states + (size_t)t * Q * N;
        const uint32_t st = step0 + (uint32_t)t;
        /* the spread force of step t, from the bead state it started with */
        memcpy(tp, bpos + (size_t)t * 3 * nb, bsz);
        memcpy(tm, bmom + (size_t)t * 3 * nb, bsz);
        memset(force, 0, sizeof(double) * 3 * (size_t)N);
        orc_couple(p, nt, st, bs, tp, tm, force);
        memset(force_bar, 0, sizeof(double) * 3 * (size_t)N);
        orc_step_adjoint(p, nt, lam, work, force, force_bar, st, gbar);
        orc_couple_adjoint(p, nt, st, bs, bpos + (size_t)t * 3 * nb, bmom + (size_t)t * 3 * nb, force_bar, pos_bar,
                           mom_bar, lam, gbar);
    }
    free(tp);
    free(tm);
    free(force_bar);
    free(force);
    free(work);
    free(bmom);
    free(bpos);
    free(states);
}
