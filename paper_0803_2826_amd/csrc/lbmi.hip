// liblbmi: host side of the C ABI declared in include/lb.h.
//
// Owns the two population buffers of a periodic box, enqueues the fused
// stream-collide kernel and the coupling kernels on the caller's stream, and
// keeps the step counter that keys the noise.  No CPU fallback exists: every
// numerical step runs in the HIP kernels of this directory.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/lb.h"
#include "couple.h"

using namespace lbmi;

struct lb_ctx {
    lb_params p;
    int device = 0;
    hipStream_t stream = nullptr;
    Geom geo{};
    CollideConst cc{};
    size_t elem = 4;
    void *bufA = nullptr;
    void *bufB = nullptr;
    uint64_t step = 0;
    int block = 256;
    int nblocks = 0;
    double *partials = nullptr;      // [nblocks][4] fused totals of the last step
    double *scratch = nullptr;       // reduction scratch (mode stats partials / outputs)
    size_t scratch_bytes = 0;
    double *dev_out = nullptr;       // [64] reduced outputs
    int32_t *flags = nullptr;        // latched device errors
    bool totals_valid = false;       // fused totals of the last step are in `partials`
    bool thermal = false;
    // bead coupling (allocated on first lb_couple)
    float *force = nullptr;          // [3][N]
    uint32_t *fmask = nullptr;       // [ceil(N/32)] bit per site: bead force present
    int32_t *list = nullptr;         // touched nodes of the pending force
    int32_t *count = nullptr;
    int list_cap = 0;
    double *half = nullptr;
    double *fc = nullptr;
    int bead_cap = 0;
    bool pending_force = false;
    int pending_rows = 0;            // upper bound of touched nodes (8 per bead)
    std::string err;
};

static std::string g_create_error;

namespace {

int fail(lb_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    else g_create_error = msg;
    return code;
}

int check(lb_ctx *c, hipError_t e, const char *what)
{
    if (e == hipSuccess) return LB_OK;
    return fail(c, LB_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define LB_TRY(expr)                   \
    do {                               \
        const int _rc = (expr);        \
        if (_rc != LB_OK) return _rc;  \
    } while (0)

#define LB_LAUNCH_CHECK(c, what) LB_TRY(check((c), hipGetLastError(), (what)))

int use_device(lb_ctx *c)
{
    int cur = -1;
    LB_TRY(check(c, hipGetDevice(&cur), "hipGetDevice"));
    if (cur != c->device) LB_TRY(check(c, hipSetDevice(c->device), "hipSetDevice"));
    return LB_OK;
}

size_t storage_bytes(int st)
{
    switch (st) {
    case LB_F32: return 4;
    case LB_BF16: return 2;
    case LB_F16: return 2;
    default: return 0;
    }
}

unsigned grid_for(size_t n, int block) { return (unsigned)((n + block - 1) / block); }

int validate(const lb_params *p, std::string &msg)
{
    if (!p) { msg = "params is NULL"; return LB_EINVAL; }
    if (p->nx < 2 || p->ny < 2 || p->nz < 2) { msg = "every extent must be >= 2"; return LB_EINVAL; }
    const uint64_t N = (uint64_t)p->nx * (uint64_t)p->ny * (uint64_t)p->nz;
    if (N >= (1ull << 30)) { msg = "N = nx*ny*nz must be < 2^30"; return LB_EINVAL; }
    if (storage_bytes(p->storage) == 0) { msg = "storage must be LB_F32, LB_BF16 or LB_F16"; return LB_EINVAL; }
    if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0)) { msg = "rho0 must be > 0"; return LB_EINVAL; }
    if (!(p->kT >= 0.0) || !std::isfinite(p->kT)) { msg = "kT must be >= 0"; return LB_EINVAL; }
    if (!(std::fabs(p->gamma_shear) < 1.0) || !(std::fabs(p->gamma_bulk) < 1.0)) {
        msg = "|gamma_shear| and |gamma_bulk| must be < 1 (finite viscosity)";
        return LB_EINVAL;
    }
    const double kin[4] = {p->gamma_3a, p->gamma_3b, p->gamma_4a, p->gamma_4b};
    for (double gk : kin)
        if (!(std::fabs(gk) <= 1.0)) { msg = "kinetic eigenvalues must satisfy |gamma| <= 1"; return LB_EINVAL; }
    for (int c = 0; c < 3; ++c)
        if (!std::isfinite(p->body_force[c])) { msg = "body force must be finite"; return LB_EINVAL; }
    if (p->block != 0 && (p->block < 64 || p->block > 1024 || (p->block % 64) != 0)) {
        msg = "block must be 0 or a multiple of 64 in [64, 1024]";
        return LB_EINVAL;
    }
    return LB_OK;
}

void fill_collide_const(lb_ctx *c)
{
    const lb_params &p = c->p;
    static const double wk[19] = {1.0,       1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0, 2.0 / 3.0, 4.0 / 3.0, 4.0 / 9.0,
                                  1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 2.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0, 2.0 / 9.0,
                                  2.0 / 9.0, 2.0 / 9.0, 2.0,       4.0 / 3.0, 4.0 / 9.0};
    double gam[19];
    for (int k = 0; k < 4; ++k) gam[k] = 1.0;
    gam[4] = p.gamma_bulk;
    for (int k = 5; k <= 9; ++k) gam[k] = p.gamma_shear;
    for (int k = 10; k <= 12; ++k) gam[k] = p.gamma_3a;
    for (int k = 13; k <= 15; ++k) gam[k] = p.gamma_3b;
    gam[16] = p.gamma_4a;
    gam[17] = gam[18] = p.gamma_4b;
    const double mu = 3.0 * p.kT;
    for (int k = 0; k < 19; ++k) {
        c->cc.gam[k] = (float)gam[k];
        c->cc.sig[k] = (k >= 4) ? (float)std::sqrt(wk[k] * mu * (1.0 - gam[k] * gam[k])) : 0.f;
    }
    c->cc.rho0 = (float)p.rho0;
    c->cc.sqrt_rho0 = (float)std::sqrt(p.rho0);
    for (int a = 0; a < 3; ++a) c->cc.g[a] = (float)p.body_force[a];
    c->cc.key0 = (uint32_t)(p.seed & 0xffffffffu);
    c->cc.key1 = (uint32_t)(p.seed >> 32);
    c->cc.box = (uint32_t)p.box_id;
    c->cc.noise_rho0 = p.noise_rho0 ? 1 : 0;
    c->thermal = p.kT > 0.0;
}

template <int ST, bool TH, bool TOT, bool FRC>
void launch_step_t(lb_ctx *c, const StepArgs &a)
{
    hipLaunchKernelGGL((k_stream_collide<ST, TH, TOT, FRC>), dim3(c->nblocks), dim3(c->block), 0, c->stream, a);
}

template <int ST, bool TH, bool TOT>
void launch_step_f(lb_ctx *c, const StepArgs &a, bool frc)
{
    if (frc) launch_step_t<ST, TH, TOT, true>(c, a);
    else launch_step_t<ST, TH, TOT, false>(c, a);
}

template <int ST>
void launch_step_st(lb_ctx *c, const StepArgs &a, bool tot, bool frc)
{
    if (c->thermal) {
        if (tot) launch_step_f<ST, true, true>(c, a, frc);
        else launch_step_f<ST, true, false>(c, a, frc);
    } else {
        if (tot) launch_step_f<ST, false, true>(c, a, frc);
        else launch_step_f<ST, false, false>(c, a, frc);
    }
}

// Dispatch on the storage type: F(integral_constant<int, ST>) for ST in {1,2,3}.
template <typename F>
void by_storage(int st, F &&fn)
{
    switch (st) {
    case LB_F32: fn(std::integral_constant<int, LB_F32>{}); break;
    case LB_BF16: fn(std::integral_constant<int, LB_BF16>{}); break;
    default: fn(std::integral_constant<int, LB_F16>{}); break;
    }
}

int ensure_scratch(lb_ctx *c, size_t bytes)
{
    if (c->scratch_bytes >= bytes) return LB_OK;
    if (c->scratch) (void)hipFree(c->scratch);
    c->scratch = nullptr;
    c->scratch_bytes = 0;
    if (hipMalloc(&c->scratch, bytes) != hipSuccess) return fail(c, LB_ENOMEM, "scratch allocation failed");
    c->scratch_bytes = bytes;
    return LB_OK;
}

int read_flags(lb_ctx *c)
{
    int32_t h = 0;
    LB_TRY(check(c, hipMemcpyAsync(&h, c->flags, sizeof(h), hipMemcpyDeviceToHost, c->stream), "flags copy"));
    LB_TRY(check(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize"));
    if (h & 1) return fail(c, LB_ENONFINITE, "non-finite population encountered on the device");
    return LB_OK;
}

int ensure_bead_buffers(lb_ctx *c, int n)
{
    const size_t N = c->geo.N;
    const size_t nwords = (N + 31) / 32;
    if (!c->force) {
        if (hipMalloc(&c->force, 3 * N * sizeof(float)) != hipSuccess ||
            hipMalloc(&c->fmask, nwords * sizeof(uint32_t)) != hipSuccess ||
            hipMalloc(&c->count, sizeof(int32_t)) != hipSuccess)
            return fail(c, LB_ENOMEM, "bead force field allocation failed");
        hipLaunchKernelGGL(k_zero_f32, dim3(1024), dim3(256), 0, c->stream, c->force, 3 * N);
        hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(nwords, 256)), dim3(256), 0, c->stream,
                           reinterpret_cast<int32_t *>(c->fmask), (uint32_t)nwords);
        LB_LAUNCH_CHECK(c, "zero force field");
    }
    if (n > c->bead_cap) {
        (void)hipFree(c->half);
        (void)hipFree(c->fc);
        (void)hipFree(c->list);
        c->half = c->fc = nullptr;
        c->list = nullptr;
        const int cap = n < 64 ? 64 : n;
        if (hipMalloc(&c->half, 3 * (size_t)cap * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->fc, 3 * (size_t)cap * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->list, 8 * (size_t)cap * sizeof(int32_t)) != hipSuccess)
            return fail(c, LB_ENOMEM, "bead scratch allocation failed");
        c->bead_cap = cap;
        c->list_cap = 8 * cap;
    }
    return LB_OK;
}

}  // namespace

extern "C" {

int lb_create(const lb_params *params, void *stream, lb_ctx **out)
{
    std::string msg;
    if (!out) return fail(nullptr, LB_EINVAL, "out is NULL");
    *out = nullptr;
    const int v = validate(params, msg);
    if (v != LB_OK) return fail(nullptr, v, msg);
    lb_ctx *c = new lb_ctx();
    c->p = *params;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(nullptr, LB_EDEVICE, "no HIP device");
    }
    c->stream = static_cast<hipStream_t>(stream);
    const uint32_t nx = params->nx, ny = params->ny, nz = params->nz;
    c->geo.nx = nx;
    c->geo.ny = ny;
    c->geo.nz = nz;
    c->geo.nxny = nx * ny;
    c->geo.N = nx * ny * nz;
    c->geo.div_nx = make_fastdiv(nx);
    c->geo.div_ny = make_fastdiv(ny);
    c->elem = storage_bytes(params->storage);
    c->block = params->block ? params->block : 256;
    c->nblocks = (int)grid_for(c->geo.N, c->block);
    fill_collide_const(c);
    const size_t bytes = (size_t)19 * c->geo.N * c->elem;
    if (hipMalloc(&c->bufA, bytes) != hipSuccess || hipMalloc(&c->bufB, bytes) != hipSuccess ||
        hipMalloc(&c->partials, (size_t)c->nblocks * 4 * sizeof(double)) != hipSuccess ||
        hipMalloc(&c->dev_out, 64 * sizeof(double)) != hipSuccess || hipMalloc(&c->flags, sizeof(int32_t)) != hipSuccess) {
        lb_destroy(c);
        return fail(nullptr, LB_ENOMEM, "device allocation failed");
    }
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, c->stream, c->flags, 1u);
    if (hipGetLastError() != hipSuccess) {
        lb_destroy(c);
        return fail(nullptr, LB_EDEVICE, "kernel launch failed in lb_create");
    }
    *out = c;
    return LB_OK;
}

int lb_destroy(lb_ctx *c)
{
    if (!c) return LB_OK;
    use_device(c);
    (void)hipStreamSynchronize(c->stream);
    void *ptrs[] = {c->bufA, c->bufB, c->partials, c->scratch, c->dev_out, c->flags, c->force,
                    c->fmask, c->list, c->count, c->half, c->fc};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    delete c;
    return LB_OK;
}

int lb_init_equilibrium(lb_ctx *c, const double *rho, const double *u)
{
    if (!c) return LB_EINVAL;
    LB_TRY(use_device(c));
    by_storage(c->p.storage, [&](auto st) {
        hipLaunchKernelGGL((k_init_equilibrium<decltype(st)::value>), dim3(grid_for(c->geo.N, 256)), dim3(256), 0,
                           c->stream, c->bufA, c->geo, c->p.rho0, rho, u);
    });
    LB_LAUNCH_CHECK(c, "init_equilibrium");
    c->totals_valid = false;
    return LB_OK;
}

int lb_set_populations(lb_ctx *c, const void *src, int32_t dtype, int32_t shifted)
{
    if (!c) return LB_EINVAL;
    if (!src) return fail(c, LB_EINVAL, "src is NULL");
    if (dtype != LB_F64 && dtype != LB_F32) return fail(c, LB_EINVAL, "dtype must be LB_F64 or LB_F32");
    LB_TRY(use_device(c));
    by_storage(c->p.storage, [&](auto st) {
        constexpr int ST = decltype(st)::value;
        if (dtype == LB_F64)
            hipLaunchKernelGGL((k_set_pops<ST, double>), dim3(grid_for(c->geo.N, 256)), dim3(256), 0, c->stream,
                               c->bufA, c->geo, c->p.rho0, static_cast<const double *>(src), shifted);
        else
            hipLaunchKernelGGL((k_set_pops<ST, float>), dim3(grid_for(c->geo.N, 256)), dim3(256), 0, c->stream,
                               c->bufA, c->geo, c->p.rho0, static_cast<const float *>(src), shifted);
    });
    LB_LAUNCH_CHECK(c, "set_populations");
    c->totals_valid = false;
    return LB_OK;
}

int lb_get_populations(lb_ctx *c, void *dst, int32_t dtype, int32_t shifted)
{
    if (!c) return LB_EINVAL;
    if (!dst) return fail(c, LB_EINVAL, "dst is NULL");
    if (dtype != LB_F64 && dtype != LB_F32) return fail(c, LB_EINVAL, "dtype must be LB_F64 or LB_F32");
    LB_TRY(use_device(c));
    by_storage(c->p.storage, [&](auto st) {
        constexpr int ST = decltype(st)::value;
        if (dtype == LB_F64)
            hipLaunchKernelGGL((k_get_pops<ST, double>), dim3(grid_for(c->geo.N, 256)), dim3(256), 0, c->stream,
                               c->bufA, c->geo, c->p.rho0, static_cast<double *>(dst), shifted);
        else
            hipLaunchKernelGGL((k_get_pops<ST, float>), dim3(grid_for(c->geo.N, 256)), dim3(256), 0, c->stream,
                               c->bufA, c->geo, c->p.rho0, static_cast<float *>(dst), shifted);
    });
    LB_LAUNCH_CHECK(c, "get_populations");
    return LB_OK;
}

int lb_step(lb_ctx *c, int32_t nsteps)
{
    if (!c) return LB_EINVAL;
    if (nsteps < 0) return fail(c, LB_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return LB_OK;
    if (c->step + (uint64_t)nsteps > 0xffffffffull) return fail(c, LB_EINVAL, "step counter would exceed 2^32");
    LB_TRY(use_device(c));
    const bool tot = c->p.track_totals != 0;
    for (int32_t t = 0; t < nsteps; ++t) {
        StepArgs a;
        a.src = c->bufA;
        a.dst = c->bufB;
        for (int i = 0; i < 19; ++i) {
            a.srcp[i] = static_cast<const char *>(c->bufA) + (size_t)i * c->geo.N * c->elem;
            a.dstp[i] = static_cast<char *>(c->bufB) + (size_t)i * c->geo.N * c->elem;
        }
        a.geo = c->geo;
        a.cc = c->cc;
        a.step = (uint32_t)c->step;
        a.xcd_remap = 1;
        a.partials = c->partials;
        a.flags = c->flags;
        a.fmask = c->fmask;
        a.force = c->force;
        const bool frc = c->pending_force;
        by_storage(c->p.storage, [&](auto st) { launch_step_st<decltype(st)::value>(c, a, tot, frc); });
        LB_LAUNCH_CHECK(c, "stream_collide");
        if (frc) {
            hipLaunchKernelGGL(k_clear_touched, dim3(grid_for((size_t)c->pending_rows, 256)), dim3(256), 0, c->stream,
                               c->force, c->fmask, c->list, c->count, c->pending_rows, c->geo.N);
            LB_LAUNCH_CHECK(c, "clear_touched");
            c->pending_force = false;
        }
        std::swap(c->bufA, c->bufB);
        ++c->step;
        c->totals_valid = tot;
    }
    return LB_OK;
}

int lb_couple(lb_ctx *c, const lb_beads *b)
{
    if (!c) return LB_EINVAL;
    if (!b) return fail(c, LB_EINVAL, "beads is NULL");
    if (b->n < 0 || b->nbonds < 0) return fail(c, LB_EINVAL, "bead and bond counts must be >= 0");
    if (b->n > (1 << 26)) return fail(c, LB_EINVAL, "too many beads");
    if (c->pending_force) return fail(c, LB_ESTATE, "lb_couple called twice without lb_step");
    if (b->n == 0) return LB_OK;
    if (!b->pos || !b->mom || !b->mass || !b->zeta || (b->nbonds > 0 && !b->bonds))
        return fail(c, LB_EINVAL, "bead arrays must be non-NULL");
    if (!std::isfinite(b->k_bond) || !std::isfinite(b->r0)) return fail(c, LB_EINVAL, "bond parameters must be finite");
    LB_TRY(use_device(c));
    LB_TRY(ensure_bead_buffers(c, b->n));
    CoupleArgs a;
    a.pop = c->bufA;
    a.geo = c->geo;
    a.rho0 = c->p.rho0;
    for (int k = 0; k < 3; ++k) a.g[k] = c->p.body_force[k];
    a.kT = c->p.kT;
    a.key0 = c->cc.key0;
    a.key1 = c->cc.key1;
    a.box = c->cc.box;
    a.step = (uint32_t)c->step;
    a.n = b->n;
    a.pos = b->pos;
    a.mom = b->mom;
    a.mass = b->mass;
    a.zeta = b->zeta;
    a.half = c->half;
    a.fc = c->fc;
    a.force = c->force;
    a.fmask = c->fmask;
    a.list = c->list;
    a.count = c->count;
    const unsigned gb = grid_for((size_t)b->n, 256);
    hipLaunchKernelGGL(k_bead_half, dim3(gb), dim3(256), 0, c->stream, a);
    if (b->nbonds > 0)
        hipLaunchKernelGGL(k_bonds, dim3(grid_for((size_t)b->nbonds, 256)), dim3(256), 0, c->stream, c->half, c->fc,
                           b->bonds, b->nbonds, b->k_bond, b->r0, b->n);
    by_storage(c->p.storage, [&](auto st) {
        hipLaunchKernelGGL((k_bead_update<decltype(st)::value>), dim3(grid_for(8 * (size_t)b->n, 256)), dim3(256), 0,
                           c->stream, a);
    });
    LB_LAUNCH_CHECK(c, "couple");
    c->pending_force = true;
    c->pending_rows = 8 * b->n;
    return LB_OK;
}

int lb_moments(lb_ctx *c, double *rho, double *u)
{
    if (!c) return LB_EINVAL;
    if (!rho && !u) return LB_OK;
    LB_TRY(use_device(c));
    by_storage(c->p.storage, [&](auto st) {
        hipLaunchKernelGGL((k_moments<decltype(st)::value>), dim3(grid_for(c->geo.N, 256)), dim3(256), 0, c->stream,
                           c->bufA, c->geo, c->p.rho0, c->p.body_force[0], c->p.body_force[1], c->p.body_force[2],
                           rho, u);
    });
    LB_LAUNCH_CHECK(c, "moments");
    return LB_OK;
}

static int totals_from_partials(lb_ctx *c, const double *partials, int rows, double out[4])
{
    hipLaunchKernelGGL(k_reduce_cols, dim3(4), dim3(256), 0, c->stream, partials, rows, 4, c->dev_out);
    LB_LAUNCH_CHECK(c, "reduce totals");
    double h[4] = {0, 0, 0, 0};
    LB_TRY(check(c, hipMemcpyAsync(h, c->dev_out, sizeof(h), hipMemcpyDeviceToHost, c->stream), "totals copy"));
    LB_TRY(read_flags(c));
    const double N = (double)c->geo.N;
    out[0] = N * c->p.rho0 + h[0];
    out[1] = h[1];
    out[2] = h[2];
    out[3] = h[3];
    return LB_OK;
}

int lb_totals_exact(lb_ctx *c, double out[4])
{
    if (!c || !out) return LB_EINVAL;
    LB_TRY(use_device(c));
    const int nb = 2048;
    LB_TRY(ensure_scratch(c, (size_t)nb * 4 * sizeof(double)));
    by_storage(c->p.storage, [&](auto st) {
        hipLaunchKernelGGL((k_totals_exact<decltype(st)::value>), dim3(nb), dim3(256), 0, c->stream, c->bufA, c->geo,
                           c->scratch);
    });
    LB_LAUNCH_CHECK(c, "totals_exact");
    return totals_from_partials(c, c->scratch, nb, out);
}

int lb_totals(lb_ctx *c, double out[4])
{
    if (!c || !out) return LB_EINVAL;
    if (!c->totals_valid) return lb_totals_exact(c, out);
    LB_TRY(use_device(c));
    return totals_from_partials(c, c->partials, c->nblocks, out);
}

int lb_mode_stats(lb_ctx *c, double var[19])
{
    if (!c || !var) return LB_EINVAL;
    LB_TRY(use_device(c));
    const int nb = 1024;
    LB_TRY(ensure_scratch(c, (size_t)nb * 38 * sizeof(double)));
    by_storage(c->p.storage, [&](auto st) {
        hipLaunchKernelGGL((k_mode_stats<decltype(st)::value>), dim3(nb), dim3(256), 0, c->stream, c->bufA, c->geo,
                           c->p.rho0, c->scratch);
    });
    hipLaunchKernelGGL(k_reduce_cols, dim3(38), dim3(256), 0, c->stream, c->scratch, nb, 38, c->dev_out);
    LB_LAUNCH_CHECK(c, "mode_stats");
    double h[38];
    LB_TRY(check(c, hipMemcpyAsync(h, c->dev_out, sizeof(h), hipMemcpyDeviceToHost, c->stream), "mode stats copy"));
    LB_TRY(read_flags(c));
    const double N = (double)c->geo.N;
    for (int k = 0; k < 19; ++k) {
        const double mean = h[k] / N;
        var[k] = h[19 + k] / N - mean * mean;
    }
    return LB_OK;
}

int lb_noise_sample(lb_ctx *c, uint32_t site0, uint32_t count, uint32_t step, float *out)
{
    if (!c) return LB_EINVAL;
    if (!out) return fail(c, LB_EINVAL, "out is NULL");
    if ((uint64_t)site0 + count > c->geo.N) return fail(c, LB_EINVAL, "site range beyond N");
    if (count == 0) return LB_OK;
    LB_TRY(use_device(c));
    hipLaunchKernelGGL(k_noise_sample, dim3(grid_for(count, 256)), dim3(256), 0, c->stream, site0, count, step, c->cc,
                       out);
    LB_LAUNCH_CHECK(c, "noise_sample");
    return LB_OK;
}

int lb_sync(lb_ctx *c)
{
    if (!c) return LB_EINVAL;
    LB_TRY(use_device(c));
    return read_flags(c);
}

uint64_t lb_step_count(const lb_ctx *c) { return c ? c->step : 0; }

int lb_set_step_count(lb_ctx *c, uint64_t step)
{
    if (!c) return LB_EINVAL;
    if (step > 0xffffffffull) return fail(c, LB_EINVAL, "step counter must be < 2^32");
    c->step = step;
    return LB_OK;
}

const char *lb_last_error(const lb_ctx *c) { return c ? c->err.c_str() : g_create_error.c_str(); }

}  // extern "C"
