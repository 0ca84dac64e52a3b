/*
 * lb.h -- C ABI of the MI355X (gfx950) fluctuating lattice-Boltzmann library
 * (liblbmi.so).
 *
 * The library advances a periodic D3Q19 fluid with the stochastic
 * multiple-relaxation-time collision of Duenweg & Ladd ("Lattice Boltzmann
 * simulations of soft matter systems": Sec. "D3Q19 model I-III", Sec.
 * "External forces") and couples point particles to it by friction
 * (Sec. "Force coupling", Sec. "Interpolating functions").
 *
 * Units are lattice units: spacing b = 1, time step h = 1, c_s^2 = 1/3, so
 * the mass density of one LB particle is mu = kT / c_s^2 = 3 kT.
 *
 * Conventions shared by every entry point:
 *   - Velocity order: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 =
 *     (+,+,0),(-,-,0),(+,-,0),(-,+,0),(+,0,+),(-,0,-),(+,0,-),(-,0,+),
 *     (0,+,+),(0,-,-),(0,+,-),(0,-,+).  Opposite directions are adjacent.
 *   - Site index s = x + nx*(y + ny*z); population arrays are [19][N]
 *     (structure of arrays), vector fields are [3][N].  (The library's own
 *     state buffers use a layout of their own; every entry point takes and
 *     returns this one.)
 *   - "The state" is the pre-collision population n_i(r,t) of eq. LBE.
 *     One step is collision at every site followed by streaming
 *     n_i(r + c_i, t+1) = n*_i(r, t).
 *   - All pointers passed to the library are DEVICE pointers on the device
 *     that was current at lb_create, unless a parameter says "host".
 *     The caller owns them; the library never frees or retains them past
 *     the call (stream-ordered: the work may still be in flight on the
 *     context stream when the call returns).
 *   - A call on a context makes the context's device current
 *     (hipSetDevice) when another one is, and leaves it current.
 *   - All work is enqueued on the stream given to lb_create, in call order.
 *     Calls that return data to host memory synchronise that stream.
 *   - Every function returns LB_OK (0) or a negative status.  Argument errors
 *     are detected on the host before anything is enqueued and leave the
 *     context unchanged.  Errors found on the device (non-finite
 *     populations) latch and are returned by the next synchronising call
 *     (lb_totals, lb_mode_stats, lb_sync).  lb_last_error() gives a message.
 *   - LB_ENOMEM: a device allocation was refused; the context stays
 *     usable (the runtime's record of the refusal is cleared, so later
 *     launches do not report it).
 *   - A context is not thread-safe.
 */
#ifndef LB_H
#define LB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LB_OK = 0,
    LB_EINVAL = -1,       /* invalid argument (shape, parameter range, NULL) */
    LB_ENOMEM = -2,       /* device allocation failed */
    LB_EDEVICE = -3,      /* HIP runtime error (message in lb_last_error) */
    LB_ENONFINITE = -4,   /* a NaN or Inf population was seen on the device */
    LB_ESTATE = -5,       /* call order violated (e.g. two lb_couple without lb_step) */
    LB_EUNSUPPORTED = -6, /* valid request the library does not implement */
    LB_EIO = -7           /* checkpoint file missing, unwritable, truncated or of another layout */
};

/* Storage type of populations (the collision always computes in FP32). */
typedef enum { LB_F64 = 0, LB_F32 = 1, LB_BF16 = 2, LB_F16 = 3 } lb_dtype;

/* Rounding of the step kernels' 16-bit stores.
 * LB_ROUND_NEAREST: round to nearest even.  Every step rounds every stored
 *   deviation, and with thermally dithered values this shrinks each
 *   population's mean by the factor 1 - u^2 / (32 ln 2) per step, u the
 *   relative spacing (2^-7 BF16, 2^-10 FP16): an extra damping of all
 *   hydrodynamic modes of 2.7e-6 (BF16) or 4.3e-8 (FP16) per step, to be
 *   compared with the viscous rate nu k^2 (Sec. "D3Q19 model III": the shear
 *   wave rate of a 512 box is 2.5e-5 per step).
 * LB_ROUND_STOCHASTIC: unbiased stochastic rounding with 6-bit probability
 *   resolution (a value is stored as one of its two representable
 *   neighbours, the one away from zero with probability equal, to within
 *   1/128, to its position between them, and exactly so on average over the
 *   FP32 values between them); the random bits come from Philox4x32-10 with counter
 *   (site, step, 3 << 16, box) and key seed, so runs stay reproducible.
 *   Only with LB_BF16 or LB_F16 storage. */
typedef enum { LB_ROUND_NEAREST = 0, LB_ROUND_STOCHASTIC = 1 } lb_rounding;

/* Fluid parameters.
 * gamma_*: eigenvalues of the linearised collision operator per mode group
 *   (eq. lco_update; groups per Sec. "D3Q19 model II": bulk mode 4, shear
 *   modes 5-9, kinetic modes 10-12, 13-15, 16, 17-18).  Stability requires
 *   |gamma| <= 1 (text after eq. lco_update); gamma_shear and gamma_bulk must
 *   satisfy |gamma| < 1 so that the viscosities of eq. shearviscosity /
 *   eq. bulkviscosity are finite.  nu = (1/6)(1+gamma_shear)/(1-gamma_shear).
 * kT: temperature; the noise of eq. stochupdaterule1 has amplitude
 *   sqrt(w_k mu rho (1 - gamma_k^2)) per mode k >= 4 (eq. detailedbalance1,
 *   eq. normalized_mk), mu = 3 kT.  kT = 0 gives the deterministic model.
 * body_force: uniform force density g (Sec. "External forces").
 * seed: key of the Philox4x32-10 generator (noise keyed by site, step, mode).
 * storage: LB_F32, LB_BF16 or LB_F16; populations are stored as deviations
 *   n_i - a_i rho0 (FP16 additionally scaled by 2^8 before rounding).
 * noise_rho0: 0 = noise amplitude uses the local density rho = m_0,
 *   1 = uses rho0.
 * block: threads per block of the fused step kernel (64..1024, multiple of
 *   64); 0 selects 256 for a single box; -1 (and 0 for a batch) lets the
 *   library time the candidates on the first lb_step and keep the fastest:
 *   for a single box threads per block x mapping of consecutive tiles to one
 *   XCD, separately for steps with and without a pending bead force; for a
 *   batch threads per block x blocks per step (see lb_launch_config).  The
 *   launch configuration never changes the results.
 * rounding: see lb_rounding; LB_ROUND_STOCHASTIC needs 16-bit storage.
 * walls: 0 = periodic in every direction; 1 = a plane channel: stationary
 *   solid walls half way along the links at z = -1/2 and z = nz - 1/2
 *   (Sec. "Boundary conditions", eq. MBB with the wall at rest): a population
 *   whose link crosses a wall returns reversed to the site it left,
 *   n_{-i}(r, t+1) = n*_i(r, t).  x and y stay periodic.  Mass is conserved,
 *   momentum is exchanged with the walls.  Every entry point (state access,
 *   moments, coupling, the adjoint) follows the same rule.  Beads must keep
 *   0 <= z < nz - 1 so that their 8-node stencil stays inside the channel.
 *   Not available for a batch (LB_EUNSUPPORTED).
 * track_totals: 1 = the step kernel also accumulates FP64 totals of mass and
 *   momentum every step (read with lb_totals); 0 = totals are computed on
 *   demand by lb_totals with a separate pass. */
typedef struct {
    int32_t nx, ny, nz;
    int32_t storage;
    double rho0;
    double gamma_shear, gamma_bulk;
    double gamma_3a, gamma_3b, gamma_4a, gamma_4b;
    double kT;
    double body_force[3];
    uint64_t seed;
    int32_t noise_rho0;
    int32_t block;
    int32_t track_totals;
    int32_t box_id;        /* fourth Philox counter word (replica index) */
    int32_t vacf_lags;     /* batch only: lags R of the on-device ensemble VACF (0 = off, <= 1024) */
    int32_t graph_steps;   /* batch only: steps per captured HIP graph (even, 0 = no graph) */
    int32_t rounding;      /* lb_rounding of the step kernels' stores (16-bit storage) */
    int32_t walls;         /* 1: stationary walls at z = -1/2 and z = nz - 1/2 (single box only) */
} lb_params;

/* Bond potential of lb_beads.bonds, with d the bond vector and r = |d|:
 * LB_BOND_HARMONIC: (k_bond/2)(r - r0)^2;
 * LB_BOND_FENE: -(k_bond/2) r0^2 ln(1 - r^2/r0^2) for r < r0 (eq. ufene,
 *   r0 = R_0 the maximum extension).  A bond at r >= r0 has no finite
 *   force: the step gives its beads' momenta a NaN (as the oracle does),
 *   does not spread their non-finite impulse (the fluid stays finite; the
 *   oracle spreads the NaN) and latches a device flag that the next
 *   synchronising call reports as LB_ENONFINITE. */
typedef enum { LB_BOND_HARMONIC = 0, LB_BOND_FENE = 1 } lb_bond;

/* Distribution of the bead noise theta in the momentum update of eq.
 * langevin_momentum_update (Sec. "Force coupling"):
 * LB_NOISE_GAUSSIAN: unit Gaussians (Box-Muller);
 * LB_NOISE_THREE_POINT: the finite-range distribution given after that
 *   equation, theta = 0 with probability 2/3 and +-sqrt(3) with
 *   probability 1/6 each; its moments agree with a unit Gaussian's up to
 *   the fourth, which keeps the update's O(h^2) accuracy, and no draw is
 *   ever large.  Both read the same Philox call (stream 1, keyed by bead,
 *   step and box), so a taped run replays either exactly. */
typedef enum { LB_NOISE_GAUSSIAN = 0, LB_NOISE_THREE_POINT = 1 } lb_noise;

/* Point particles with bonds and an optional purely repulsive pair
 * potential (Sec. "Force coupling"; the Kremer-Grest bead-spring model of
 * Sec. "Coarse-grained models").  All arrays are device FP64 (bonds int32), caller-owned:
 *   pos  [n][3]  unwrapped positions (in/out)
 *   mom  [n][3]  momenta p (in/out)
 *   mass [n]     m_i > 0
 *   zeta [n]     friction Gamma_i >= 0 (eq. fdrag)
 *   bonds [nbonds][2]  bead index pairs with the potential `bond` (lb_bond)
 *                of parameters k_bond, r0
 *   fext [n][3]  external force on each bead, added to the conservative force
 *                (constant over the call; its reaction is not given to the
 *                fluid), or NULL
 *   stencil      points per axis of the interpolation kernel (Sec.
 *                "Interpolating functions"): 2 = phi_2 (eq. 2point, 8 nodes;
 *                also selected by 0), 3 = phi_3 (eq. 3point, 27 nodes),
 *                4 = phi_4 (eq. 4point, 64 nodes); the kernel is used for
 *                both the interpolation and the spreading
 *   wca_epsilon, wca_sigma  the Lennard-Jones potential of eq. ulennardjones
 *                cut and shifted at its minimum r_c = 2^(1/6) sigma (purely
 *                repulsive) between every pair of beads, bonded or not, at
 *                their minimum-image distance along the periodic axes (with
 *                walls the z axis is not periodic: no pair interacts through
 *                a wall); wca_epsilon = 0 switches it off.  Pairs are found
 *                with a cell list of cells no narrower than r_c, rebuilt
 *                every call; r_c must be below half of every periodic extent.
 *   noise        distribution of the bead noise (lb_noise)
 * Units are lattice units (spacing a = 1, time step h = 1). */
typedef struct {
    int32_t n;
    int32_t nbonds;
    double *pos;
    double *mom;
    const double *mass;
    const double *zeta;
    const int32_t *bonds;
    double k_bond;
    double r0;
    const double *fext;
    int32_t stencil;
    int32_t bond;      /* lb_bond */
    double wca_epsilon;
    double wca_sigma;
    int32_t noise;     /* lb_noise */
} lb_beads;

typedef struct lb_ctx lb_ctx;

/* Two-rate relaxation (Sec. "D3Q19 model II": one even rate for the bulk,
 * shear and even kinetic modes, one odd rate for the odd kinetic modes):
 * sets gamma_shear = gamma_bulk = gamma_4a = gamma_4b = gamma_e and
 * gamma_3a = gamma_3b = gamma_o in *params (the other fields are left as
 * they are), with gamma_o chosen so that the product of the two relaxation
 * times, Lambda = (1/(1 - gamma_e) - 1/2)(1/(1 - gamma_o) - 1/2), equals
 * `magic`.  magic = 3/16 puts a stationary mid-link bounce-back wall
 * exactly half way along the link for plane Poiseuille flow at every
 * viscosity.  Host only.  Errors: LB_EINVAL (params NULL, |gamma_e| >= 1,
 * magic <= 0 or not finite). */
int lb_params_two_rate(double gamma_e, double magic, lb_params *params);

/* Create a context: allocates two population buffers (2 * P * N * storage
 * bytes) and small bookkeeping on the current device, enqueues on `stream`
 * (a hipStream_t; NULL = the null stream).  P = 20 for LB_F32 storage,
 * whose rest population is held as its FP32 value plus its FP32 rounding
 * residual, so that every step keeps each site's mass to ~1e-17 (the
 * collision conserves mass: the constraint after eq. LBE); P = 19 for 16-bit
 * storage, which rounds that residual once per site and step.  The state is uninitialised until
 * lb_init_equilibrium or lb_set_populations.  The step counter starts at 0.
 * Errors: LB_EINVAL (any extent < 2, N >= 2^30, |gamma| out of range,
 * kT < 0, rho0 <= 0, unknown storage, bad block), LB_ENOMEM, LB_EDEVICE. */
int lb_create(const lb_params *params, void *stream, lb_ctx **out);

/* Batched form: nbox independent periodic replica boxes of extents
 * dims[3*b .. 3*b+2] (host array), all with the physical parameters of
 * `params` (its extents are ignored).  Box b uses box id params->box_id + b
 * as the fourth Philox counter word, so every replica draws its own noise.
 * All boxes advance together: one launch per step walks a list of (box,
 * tile) work items, each block a contiguous run of them (a run of one when
 * no VACF is sampled and the launch search finds it faster); with
 * graph_steps > 0 the launches of graph_steps
 * steps are captured once into a HIP graph and replayed.  Populations of all
 * boxes live in one allocation, box after box, each [19][N_b].  The context
 * runs on its own stream, ordered after / before the caller's `stream` at the
 * entry / exit of every call.  Bead coupling is not available on a batch
 * (lb_couple returns LB_EUNSUPPORTED).  With vacf_lags = R > 0 every step also
 * samples, per box, the lowest transverse Fourier modes of the momentum
 * density (k = 2 pi / L_a along each axis a, the two components normal to a)
 * and accumulates their autocorrelation on the device (read with lb_vacf).
 * Layout of the batch forms of lb_init_equilibrium / lb_set_populations /
 * lb_get_populations / lb_moments: box after box, each in the single-box
 * layout.  Errors: as lb_create, plus LB_EINVAL for nbox < 1, a box extent
 * < 2, a box of 2^30 sites or more, a total site count >= 2^31, odd
 * graph_steps or vacf_lags > 1024. */
int lb_create_batch(const lb_params *params, int32_t nbox, const int32_t *dims, void *stream, lb_ctx **out);

/* Ensemble velocity autocorrelation of a batch: host out[nbox][vacf_lags],
 * out[b][tau] = mean over samples t and the 6 modes of
 * Re[j_hat(k, t + tau) conj(j_hat(k, t))] / (N_b kT rho0), which at gamma = 0
 * should decay as lambda(k)^tau, lambda = 1 - (2/3) sin^2(k/2) (eq. LBE with
 * the equipartition of eq. Pdistneq).  *nsamples receives the number of
 * sampled steps.  Synchronises.  LB_EINVAL if the context has no VACF. */
int lb_vacf(lb_ctx *ctx, double *out, int64_t *nsamples);

/* Launch configuration of the step kernel: out[0] = threads per block,
 * out[1] = blocks per step, out[2] = tiles per block (batch) or 1, out[3] =
 * 1 if consecutive tiles are mapped to one XCD (single box) or 0.  For a
 * single box `force` selects the variant that runs after lb_couple (its
 * configuration is searched separately, on its first use); a batch ignores
 * it.  Before the first lb_step of a searching context the entries hold the
 * defaults (256 threads, no XCD mapping). */
int lb_launch_config(lb_ctx *ctx, int32_t force, int32_t out[4]);

/* Checkpoint / resume.  lb_save writes the current state (the stored
 * populations of every box, bit for bit, with the step counter, the
 * parameters and the box extents) to the host file `path`; lb_load reads
 * such a file into a context of the same layout (box extents, box count,
 * storage type) and sets its step counter, so that, with the same
 * parameters and seed, the run continues exactly as the saved one would
 * have (the noise is keyed by site and step).  The parameters stored in the
 * file are not applied.  Bead state is caller-owned and saved by the caller;
 * a batch's VACF accumulators are not saved.  Both synchronise.  Errors:
 * LB_EIO (open / read / write failure, not a checkpoint, other layout),
 * LB_ESTATE (called between lb_couple and lb_step).  lb_load ends a tape
 * (see lb_tape_begin). */
int lb_save(lb_ctx *ctx, const char *path);
int lb_load(lb_ctx *ctx, const char *path);

/* Release all device memory of the context (synchronises its stream). */
int lb_destroy(lb_ctx *ctx);

/* Set every site to the equilibrium n^eq(rho(r), u(r)) of
 * eq. original_equil_distrib.  rho: device FP64 [N] or NULL (rho0);
 * u: device FP64 [3][N] or NULL (rest). */
int lb_init_equilibrium(lb_ctx *ctx, const double *rho, const double *u);

/* Copy the state in / out.  src/dst: device arrays [19][N] of type `dtype`
 * (LB_F64 or LB_F32).  shifted = 0: full populations n_i; shifted = 1:
 * deviations n_i - a_i rho0.  Storage rounding applies on the way in (the
 * rest population of LB_F32 storage keeps its FP64 value as value plus
 * residual).  lb_set_populations and lb_init_equilibrium end a tape (see
 * lb_tape_begin). */
int lb_set_populations(lb_ctx *ctx, const void *src, int32_t dtype, int32_t shifted);
int lb_get_populations(lb_ctx *ctx, void *dst, int32_t dtype, int32_t shifted);

/* Advance nsteps >= 0 time steps (eq. LBE with the collision of
 * eq. coll_operator_plus_noise_plus_force, noise keyed by the step counter).
 * A force spread by a preceding lb_couple enters the first of these steps
 * only; the counter increases by nsteps. */
int lb_step(lb_ctx *ctx, int32_t nsteps);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  One step
 * of lb_step (the fused collision and pull streaming, no bead force) without
 * a context and without any allocation: it reads the stored state `src` of
 * step `step` (the step counter keys the noise) and writes the stored state
 * of step + 1 to `dst`; with `totals` != NULL it also writes the FP64 totals
 * of the new state to device memory totals[4] = {sum rho, sum j_x, sum j_y,
 * sum j_z}, the same bits lb_totals gives for a context with track_totals
 * and the same block.  Nothing is synchronised; all work is enqueued on
 * `stream` (a hipStream_t; NULL = null stream) of the current device, and
 * src, dst, totals are device memory of that device, owned by the caller.
 *   params: as for lb_create (walls, rounding and storage included), with
 *           block 0 (256 threads) or 64..1024; -1 is refused (no launch
 *           search without a context).
 *   src, dst: the stored form of the state, P * N elements of the storage
 *           type (P = 20 for LB_F32, 19 for 16-bit storage), non-overlapping.
 *           Stored form: element (P z + i) nx ny + x + nx y holds, for
 *           i < 19, A_i(r) = n_i(r + c_i) - a_i rho0 (the pre-collision
 *           population of the site it streams to, shifted; FP16 values are
 *           scaled by 2^8; with walls, n_{opp(i)}(r) - a_i rho0 where the
 *           link r -> r + c_i crosses a wall), and for i = 19 (LB_F32 only)
 *           the FP32 residual of the rest population, whose value is
 *           A_0 + A_19.  A caller builds it once from [19][N] populations,
 *           e.g. outside the captured region.
 * The step kernel's per-block totals go to a static device array of
 * 2^19 rows (16 MiB per device, held until the process ends): steps with
 * more than 2^19 blocks (nz * ceil(nx ny / block)) are refused with
 * LB_EINVAL; use a larger block.  Every call on a device shares that array:
 * calls that overlap on one device (other streams, other threads) race on
 * it and their totals are undefined; calls ordered on one stream do not.
 * The first call on each device resolves the array's address
 * (hipGetSymbolAddress), which allocates nothing.  Errors (LB_EINVAL for a
 * bad argument, LB_EDEVICE for a launch failure) leave a message for
 * lb_last_error(NULL); non-finite populations show up as non-finite
 * totals. */
int lb_step_noalloc(const lb_params *params, const void *src, void *dst, uint64_t step, double *totals,
                    void *stream);

/* Particle half of one coupled time step (Sec. "Force coupling"): half
 * drift; conservative forces at the half-step positions (bonds, WCA pairs,
 * fext); interpolation of u at each bead with the stencil's kernel
 * (eq. ufluid_discrete; trilinear for phi_2, eq. 2point); the exact Langevin
 * momentum update eq. langevin_momentum_update; spreading of the exchanged
 * impulse over the same stencil nodes (eq. ftotal); second half drift.  The
 * interpolated velocity is u = (sum_i n_i c_i + g/2)/rho from the current
 * state.  The spread force is applied by the next lb_step.  Bead noise is
 * keyed by (bead index, step counter).  Errors: LB_EINVAL (n < 0, NULL
 * arrays with n > 0, unknown stencil or bond kind, non-finite or negative
 * bond or WCA parameters, r_c >= half a periodic box extent), LB_ESTATE (a
 * previous lb_couple's force not yet consumed). */
int lb_couple(lb_ctx *ctx, const lb_beads *beads);

/* nsteps >= 0 coupled time steps with the same beads: the same result, bit
 * for bit, as nsteps times lb_couple then lb_step(ctx, 1) (taped or not),
 * the bead state in beads->pos, beads->mom advanced in place.  Without
 * walls, with at most 64 bonds per bead and nsteps >= 2 (any of the
 * stencils phi_2, phi_3, phi_4; with WCA pairs phi_2, the cell lists built
 * by the launches themselves), each step is ONE launch (the particle half runs in
 * the first blocks of the fluid step's grid, each bead sums its own bond
 * forces); otherwise the separate launches run.  Before the first step the
 * bond list is copied to the host (one synchronisation).  Errors: those of
 * lb_couple and lb_step; a fused step whose site blocks stopped waiting for
 * its particle blocks (not expected) is reported as LB_EDEVICE by the next
 * call that reads the device flags (lb_totals, lb_sync). */
int lb_coupled_steps(lb_ctx *ctx, const lb_beads *beads, int32_t nsteps);

/* Density and velocity of the current state: rho = sum_i n_i,
 * u = (sum_i n_i c_i + g/2) / rho (eq. special_choice_momentum_density with
 * the uniform body force).  rho: device FP64 [N]; u: device FP64 [3][N];
 * either may be NULL. */
int lb_moments(lb_ctx *ctx, double *rho, double *u);

/* FP64 totals of the current state, host out[4] = {sum rho, sum j_x, sum j_y,
 * sum j_z} with j = sum_i n_i c_i: the conserved quantities of eq. LBE
 * (mass exactly, momentum up to the forcing of eq. moment_one_external_force).  With track_totals the values come from
 * the last step's fused accumulation (stored, rounded populations);
 * otherwise (or before any step) from a full reduction pass.  Synchronises;
 * returns LB_ENONFINITE if a non-finite population was seen. */
int lb_totals(lb_ctx *ctx, double out[4]);

/* Low-Mach guard: the number of sites of the current state (all boxes of a
 * batch) with a negative population n_i = a_i rho0 + d_i, and the smallest
 * n_i (host out; either may be NULL).  The method assumes Ma = u/c_s << 1
 * (Sec. "The fluctuating lattice-Boltzmann equation"); the quadratic
 * equilibrium of Sec. "D3Q19 model I" goes negative once u is not small,
 * and thermal noise can push the populations with small a_i below zero.  A
 * scan of the stored state (one read of it), not part of the step, so that
 * it costs nothing unless called; non-finite values are not counted (the
 * step latches them, LB_ENONFINITE).  Synchronises. */
int lb_negative_count(lb_ctx *ctx, uint64_t *sites, double *min_pop);

/* Same as lb_totals but always runs the full reduction pass. */
int lb_totals_exact(lb_ctx *ctx, double out[4]);

/* Per-mode statistics of the current state: host var[19] =
 * mean over sites of (m_k - mean m_k)^2 with m_k = sum_i e_ki n_i (Table 1
 * basis).  At equilibrium var[k] = mu w_k rho0 (variance of eq. Pdistneq).
 * Synchronises. */
int lb_mode_stats(lb_ctx *ctx, double var[19]);

/* The fifteen unit Gaussians r_k (k = 4..18, eq. stochupdaterule1) that the
 * collision at sites site0 .. site0+count-1 draws at step `step`, with this
 * context's seed and box id.  out: device FP32 [count][15].  Lets a caller
 * check the device generator against an independent implementation.
 * Errors: LB_EINVAL (out NULL, site range beyond N). */
int lb_noise_sample(lb_ctx *ctx, uint32_t site0, uint32_t count, uint32_t step, float *out);

/* Differentiation form.  lb_tape_begin starts recording at the current step:
 * the state is checkpointed now and after every `checkpoint_every` steps
 * (device copies of the population buffer, P * N * storage bytes each).
 * lb_backward then returns, for the T steps taken since lb_tape_begin,
 *   dL_dn_0 = dL/dn(t0) given dL_dn_T = dL/dn(t0 + T)   (device [19][N] of
 *             `dtype` LB_F64 or LB_F32, full populations, natural layout),
 *   dL_dg   = dL/dg through the dynamics (host out[3]; a loss that also
 *             uses g directly adds that part itself),
 * by reverse-mode differentiation of eq. LBE: the transpose of streaming
 * and of the moment-space collision (eq. lco_update, eq. stochupdaterule1,
 * eq. moment_two_external_force), segment by segment from the checkpoints
 * with the states of a segment recomputed forward, the noise replayed from
 * its Philox counters.  lb_tape_begin allocates checkpoint_every step
 * buffers, and the taped steps write each segment's states into them, so the
 * reverse sweep recomputes no step of the last segment (none at all when
 * checkpoint_every >= T; a second lb_backward on the same tape recomputes
 * every segment if the first one had more than one).  If they do not fit,
 * recording goes on without them and lb_backward allocates them itself;
 * they are also left to lb_backward when they would take more than half of
 * the device's free memory (T is not known at lb_tape_begin).
 * checkpoint_every = 0 records a moments tape instead: no checkpoints, and
 * every taped step writes the moments (rho - rho0, j) of the state it
 * starts from, 16 bytes per site and step in FP32 (the only part of the
 * state the collision's Jacobian depends on), so the reverse sweep
 * recomputes nothing and reads 16 B per site of each step instead of a
 * state; the slots are allocated in chunks of up to 64 steps and 1 GiB by
 * the steps (or lb_tape_reserve) and freed when the tape ends.  The taped
 * steps take no fused totals (lb_totals forms them from the state), and
 * taped coupled steps with phi_3 or phi_4 take the separate launches.
 * A tape lasts until the next lb_tape_begin; a call that replaces the state
 * or the step counter (lb_set_populations, lb_init_equilibrium,
 * lb_set_step_count, lb_load) ends it, so a later lb_backward returns
 * LB_ESTATE.
 * Taped coupled steps (lb_couple before lb_step) are differentiated too:
 * each lb_couple while recording keeps its particle half on the device (P
 * at the start, R', F^c and P'': 12 doubles per bead, and each stencil
 * node's fixed-point spread contribution: 32 bytes per entry, 8, 32 or 64
 * entries per bead for phi_2, phi_3, phi_4) and the lb_beads descriptor, so the arrays mass, zeta and
 * bonds must stay valid and unchanged until lb_backward, the bead count
 * must be the same in every taped coupled step, and the bead state must
 * change only through lb_couple between taped steps.  Both sweeps put a
 * coupled step's spread force back from its recorded contributions (the
 * bead kernels do not run again); in the reverse sweep the fluid adjoint
 * also yields the adjoint of the bead force at the touched nodes, and the
 * adjoint of the particle half (half drift, harmonic or FENE bonds and WCA
 * pairs (their Jacobians mag I + 2 mag' d d^T), the interpolation with the
 * stencil weights differentiated in R, the momentum update
 * eq. langevin_momentum_update, the spread reaction eq. ftotal) carries the
 * bead adjoints back and adds the interpolation's share to dL/dn and
 * dL/dg.
 * lb_backward_coupled takes and returns the bead adjoints as well:
 *   dL_dR_T, dL_dP_T: dL/dR, dL/dP of the bead state after the last step
 *                     (device FP64 [n][3]; NULL = zero),
 *   dL_dR_0, dL_dP_0: dL/dR, dL/dP of the bead state at the first taped
 *                     coupled step (device FP64 [n][3]; NULL = not wanted);
 * without taped coupled steps they are ignored.  lb_backward is
 * lb_backward_coupled with all four NULL.
 * Errors: LB_EINVAL (checkpoint_every < 0), LB_ESTATE (no tape, a tape
 * ended by one of the calls above, or called between lb_couple and lb_step;
 * lb_tape_begin between lb_couple and lb_step), LB_EUNSUPPORTED (a batch
 * context; the bead count changed between taped coupled steps), LB_ENOMEM
 * (from lb_tape_begin: no tape is left). */
int lb_tape_begin(lb_ctx *ctx, int32_t checkpoint_every);

/* Allocates now what the next nsteps >= 0 taped steps will take while they
 * run: their checkpoints (or moment slots) and, with beads != NULL, room in the bead tape for
 * nsteps coupled steps of these beads and the coupled steps' device buffers
 * (force field, bitmaps, bond partner table, cell lists); so that no
 * allocation falls inside a timed or latency-bound run.  Only allocates
 * (and synchronises once for the bond table).  Errors: LB_ESTATE (no tape),
 * LB_EINVAL (nsteps < 0, or the checks of lb_couple on beads),
 * LB_EUNSUPPORTED (a bead count other than the tape's), LB_ENOMEM. */
int lb_tape_reserve(lb_ctx *ctx, int32_t nsteps, const lb_beads *beads);
int lb_backward(lb_ctx *ctx, const void *dL_dn_T, int32_t dtype, void *dL_dn_0, double dL_dg[3]);
int lb_backward_coupled(lb_ctx *ctx, const void *dL_dn_T, int32_t dtype, const double *dL_dR_T, const double *dL_dP_T,
                        void *dL_dn_0, double dL_dg[3], double *dL_dR_0, double *dL_dP_0);

/* Synchronise the context stream and report latched device errors. */
int lb_sync(lb_ctx *ctx);

/* Step counter (keys the noise).  lb_set_step_count lets a restarted run
 * continue the same random stream; it ends a tape (see lb_tape_begin) and
 * returns LB_ESTATE between lb_couple and lb_step. */
uint64_t lb_step_count(const lb_ctx *ctx);
int lb_set_step_count(lb_ctx *ctx, uint64_t step);

/* Message for the last error on this context ("" if none). ctx may be NULL
 * (then: the last failure of lb_create, lb_create_batch or
 * lb_step_noalloc). */
const char *lb_last_error(const lb_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* LB_H */
