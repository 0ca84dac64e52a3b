// liblbmi: host side of the C ABI declared in include/lb.h.
//
// Owns the two population buffers of a periodic box, enqueues the fused
// stream-collide kernel and the coupling kernels on the caller's stream, and
// keeps the step counter that keys the noise.  No CPU fallback exists: every
// numerical step runs in the HIP kernels of this directory.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <functional>
#include <cmath>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#include <limits>

#include "../../include/lb.h"

#include "adjoint.h"
#include "bead_adjoint.h"
#include "batch.h"
#include "couple.h"
#include "fused.h"

using namespace lbmi;

#ifndef LBMI_XCD_REMAP
#define LBMI_XCD_REMAP 0
#endif

struct lb_ctx {
    lb_params p;
    int device = 0;
    hipStream_t stream = nullptr;       // stream all work of this context is enqueued on
    hipStream_t user_stream = nullptr;  // caller's stream (differs from `stream` for a batch)
    void *buf0 = nullptr;               // first allocated population buffer (graph parity)
    Geom geo{};
    CollideConst cc{};
    size_t elem = 4;
    // bufA holds the state, bufB is free for the next step's output.  While a
    // tape records, bufA may point into the segment buffer; own[] are the
    // two state buffers the context allocated, and bufB is always one of
    // them
    void *bufA = nullptr;
    void *bufB = nullptr;
    void *own[2] = {nullptr, nullptr};
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
    bool full_relax = false;         // every non-conserved gamma_k is 0
    // bead coupling (allocated on first lb_couple)
    long long *force = nullptr;      // [3][N] fixed point (kForceScale)
    uint32_t *fmask = nullptr;       // [ceil(N/32)] bit per site: bead force present
    double *half = nullptr;
    double *fc = nullptr;
    double *fb2 = nullptr;           // [2][cap][3] bond-force accumulators, used by alternate calls
    double *fp = nullptr;            // [cap][3] WCA pair forces
    int fb_par = 0;                  // accumulator of the next call
    int bead_cap = 0;
    bool pending_force = false;
    // WCA cell list (allocated on the first lb_couple with wca_epsilon > 0)
    int32_t *cell_head = nullptr;    // [cell_cap] first bead of each cell's list (-1 at rest)
    size_t cell_cap = 0;             // cells allocated
    int32_t *cell_next = nullptr;    // [n] next bead in the same cell
    int32_t *cell_of = nullptr;      // [n] cell of each bead
    int pair_cap = 0;
    // fused coupled steps (allocated on the first lb_coupled_steps that fuses)
    double *bead_pp = nullptr;       // [2][2][cap][3] alternate bead states (pos, mom) between launches
    int bead_pp_cap = 0;
    uint32_t *fmask_f = nullptr;     // [ceil(N/32)] second bitmap: the next step's nodes
    uint32_t *arrive = nullptr;      // count of finished particle blocks (all launches)
    uint32_t arrive_count = 0;       // its value once every enqueued launch has finished
    int32_t *partner = nullptr;      // [n][deg] bond partners of each bead
    size_t partner_cap = 0;
    int32_t *flist = nullptr;        // fused WCA: three cell lists, [3][cap] heads then [3][n] next, [3][n] cell_of
    size_t flist_cells = 0;
    int flist_n = 0;
    float *moments = nullptr;        // reverse sweep: [slots][z][4][y][x] moments of the recomputed states
    size_t moments_slots = 0;
    bool tuned = false;              // launch configuration chosen (autotune done or fixed)
    uint32_t xcd_remap = LBMI_XCD_REMAP;  // step kernel: consecutive tiles on one XCD (if the grid allows)
    // single box: launch configuration of the step kernel without / with a
    // pending bead force (the two variants differ in register use), each
    // searched on its first use when block = -1
    bool search = false;
    bool tuned_f[2] = {false, false};
    int block_f[2] = {256, 256};
    uint32_t remap_f[2] = {LBMI_XCD_REMAP, LBMI_XCD_REMAP};
    // batched replicas
    bool batch = false;
    int nbox = 0;
    std::vector<BoxDesc> boxes_h;
    BoxDesc *boxes_d = nullptr;
    uint32_t *tile_box = nullptr;    // [ntiles]
    uint32_t ntiles = 0;
    uint32_t chunk = 1;              // tiles per block
    uint64_t total_sites = 0;
    hipStream_t bstream = nullptr;   // private stream of a batch (graph capture)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    uint32_t *dstep = nullptr;       // [2]: device step counter, VACF sample count
    float *amp = nullptr;            // [tiles][12] VACF partial sums per tile (sized for 64-site tiles)
    float *ring = nullptr;           // [nbox][R][12]
    double *corr = nullptr;          // [nbox][R]
    hipGraphExec_t graph_exec[2] = {nullptr, nullptr};  // per buffer parity
    // differentiation (tape of checkpoints)
    bool taping = false;
    int tape_k = 0;
    uint64_t tape_step0 = 0;
    std::vector<void *> checkpoints;  // A-buffer copies at tape_step0 + s * tape_k
    void *seg = nullptr;              // tape_k step buffers of one segment
    size_t seg_bytes = 0;
    // the taped forward writes its step buffers into seg, so slots 1.. of the
    // last segment hold them until a reverse sweep recomputes over them
    bool seg_fwd = false;
    // checkpoint_every = 0: no checkpoints; every taped step writes its input
    // state's moments (rho - rho0, j: [z][4][y][x] FP32, 16 B per site) into
    // a slot of mom_chunks (mom_chunk_steps slots per chunk), and the reverse
    // sweep recomputes nothing
    bool tape_mom = false;
    std::vector<float *> mom_chunks;
    size_t mom_chunk_steps = 0;
    float *lamA = nullptr, *lamB = nullptr;
    double *gbar_d = nullptr;
    double *adj_partials = nullptr;
    // particle halves of the taped coupled steps: slot per taped step (-1:
    // no bead force), the bead configuration of each slot and its record in
    // tape_bead at byte offset tape_off[slot] (TapeSlot)
    std::vector<int32_t> tape_slot;
    std::vector<lb_beads> tape_beads;
    std::vector<void *> ckpt_ready;   // checkpoint buffers allocated ahead of the steps that fill them
    std::vector<size_t> tape_off;
    int pending_slot = -1;
    int tape_nb = 0;
    char *tape_bead = nullptr;
    size_t tape_bead_bytes = 0;       // allocated
    size_t tape_bead_used = 0;
    // backward scratch of the particle adjoint
    double *bead_work = nullptr;      // [5][n][3]: half_bar, fc_bar, p_bar, pos_bar, mom_bar
    int bead_work_n = 0;
    float *fbar = nullptr;            // [2][3][N] adjoint of the spread force by step parity (zero outside touched nodes)
    long long *force2 = nullptr;      // the reverse sweep's second force field and bitmap (step parity)
    uint32_t *fmask2 = nullptr;
    std::string err;
};

static std::string g_create_error;

// Static scratch of lb_step_noalloc (for callers that cannot allocate): the
// step kernel's per-block FP64 totals rows, then one word for its device
// error flag.  Each device holds its own copy from module load until the
// process ends; host code uses the address hipGetSymbolAddress returns for
// the current device (g_noalloc_scratch), never the array's name, which is a
// host-side stand-in.
constexpr size_t kNoallocRows = size_t(1) << 19;  // 16 MiB of totals rows
static __device__ __align__(256) double scratch[4 * kNoallocRows + 32];
constexpr int kMaxDevices = 64;
static double *g_noalloc_scratch[kMaxDevices] = {};
static std::mutex g_noalloc_mu;

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

// hipMalloc that leaves no error behind when it fails: the runtime keeps a
// refused allocation as the last error, which the next launch check
// (hipGetLastError) would then report as a failed launch, although the
// caller was given LB_ENOMEM and the context stays usable.
template <typename P>
bool dev_alloc(P **p, size_t bytes)
{
    if (hipMalloc(reinterpret_cast<void **>(p), bytes) == hipSuccess) return true;
    *p = nullptr;
    (void)hipGetLastError();
    return false;
}

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

// Planes per layer (single box) or per box (batch) of a population buffer:
// FP32 storage adds the rest population's residual plane (kRestLo).
uint32_t state_planes(int st) { return st == LB_F32 ? 20u : 19u; }

// Blocks of a single-box step launch: every z-layer is cut into
// ceil(nxny / block) tiles (a layer's last tile may be partial).
unsigned step_blocks(const lb_ctx *c, int block)
{
    return c->geo.nz * (unsigned)((c->geo.nxny + (uint32_t)block - 1u) / (uint32_t)block);
}

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
    if (p->rounding != LB_ROUND_NEAREST && p->rounding != LB_ROUND_STOCHASTIC) {
        msg = "rounding must be LB_ROUND_NEAREST or LB_ROUND_STOCHASTIC";
        return LB_EINVAL;
    }
    if (p->rounding == LB_ROUND_STOCHASTIC && p->storage == LB_F32) {
        msg = "stochastic rounding applies to 16-bit storage only";
        return LB_EINVAL;
    }
    if (p->walls != 0 && p->walls != 1) { msg = "walls must be 0 or 1"; return LB_EINVAL; }
    if (p->block != 0 && p->block != -1 && (p->block < 64 || p->block > 1024 || (p->block % 64) != 0)) {
        msg = "block must be 0, -1 or a multiple of 64 in [64, 1024]";
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
        c->cc.sigw[k] = (k >= 4) ? (float)(std::sqrt(wk[k] * mu * (1.0 - gam[k] * gam[k])) / wk[k]) : 0.f;
    }
    c->cc.rho0 = (float)p.rho0;
    c->cc.sqrt_rho0 = (float)std::sqrt(p.rho0);
    for (int a = 0; a < 3; ++a) c->cc.g[a] = (float)p.body_force[a];
    c->cc.key0 = (uint32_t)(p.seed & 0xffffffffu);
    c->cc.key1 = (uint32_t)(p.seed >> 32);
    c->cc.box = (uint32_t)p.box_id;
    c->cc.noise_rho0 = p.noise_rho0 ? 1 : 0;
    c->thermal = p.kT > 0.0;
    c->full_relax = true;
    for (int k = 4; k < 19; ++k) c->full_relax = c->full_relax && gam[k] == 0.0;
}

template <int ST, bool TH, bool TOT, bool FRC, bool FULL>
void launch_step_w(lb_ctx *c, const StepArgs &a)
{
    const size_t lds = TOT ? (size_t)kTotalsLds * (size_t)c->block : 0;  // block_sum_totals
    if (c->geo.walls)
        hipLaunchKernelGGL((k_stream_collide<ST, TH, TOT, FRC, true, FULL>), dim3(c->nblocks), dim3(c->block), lds,
                           c->stream, a);
    else
        hipLaunchKernelGGL((k_stream_collide<ST, TH, TOT, FRC, false, FULL>), dim3(c->nblocks), dim3(c->block), lds,
                           c->stream, a);
}

// The complete-relaxation variant serves thermal runs whose non-conserved
// rates are all 0 (it saves arithmetic where the 16-bit kernels are bound by
// it; without noise the step is bound by memory either way).
template <int ST, bool TH, bool TOT, bool FRC>
void launch_step_t(lb_ctx *c, const StepArgs &a)
{
    if (TH && c->full_relax) launch_step_w<ST, TH, TOT, FRC, TH>(c, a);
    else launch_step_w<ST, TH, TOT, FRC, false>(c, a);
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

// Dispatch on the interpolation kernel width: F(integral_constant<int, W>) for
// W in {2, 3, 4} (0 selects 2).
template <typename F>
void by_stencil(int w, F &&fn)
{
    switch (w) {
    case 3: fn(std::integral_constant<int, 3>{}); break;
    case 4: fn(std::integral_constant<int, 4>{}); break;
    default: fn(std::integral_constant<int, 2>{}); break;
    }
}

// Storage template of the step kernels: the storage type, or 4 / 5 for BF16 /
// FP16 stores with stochastic rounding.  Every other kernel only loads or
// converts once and uses the plain storage type.
template <class F>
void by_step_storage(const lb_params &p, F &&fn)
{
    if (p.rounding == LB_ROUND_STOCHASTIC) {
        if (p.storage == LB_BF16) fn(std::integral_constant<int, 4>{});
        else fn(std::integral_constant<int, 5>{});
    } else {
        by_storage(p.storage, fn);
    }
}

int ensure_scratch(lb_ctx *c, size_t bytes)
{
    if (c->scratch_bytes >= bytes) return LB_OK;
    if (c->scratch) (void)hipFree(c->scratch);
    c->scratch = nullptr;
    c->scratch_bytes = 0;
    if (!dev_alloc(&c->scratch, bytes)) return fail(c, LB_ENOMEM, "scratch allocation failed");
    c->scratch_bytes = bytes;
    return LB_OK;
}

// Device address of the static scratch on the current device, resolved once
// per device (with that device current).
int noalloc_scratch(double **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail(nullptr, LB_EDEVICE, "lb_step_noalloc: no usable current HIP device");
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(nullptr, LB_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_noalloc_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_noalloc_scratch[dev];
    return LB_OK;
}

int read_flags(lb_ctx *c)
{
    int32_t h = 0;
    LB_TRY(check(c, hipMemcpyAsync(&h, c->flags, sizeof(h), hipMemcpyDeviceToHost, c->stream), "flags copy"));
    LB_TRY(check(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize"));
    if (h & 2) return fail(c, LB_ENONFINITE, "a FENE bond was stretched to r >= r0 (bead momentum is NaN)");
    if (h & 4) return fail(c, LB_ENONFINITE, "a bead's spread force was not finite (not applied)");
    if (h & 1) return fail(c, LB_ENONFINITE, "non-finite population encountered on the device");
    if (h & 8) return fail(c, LB_EDEVICE, "a fused coupled step's site blocks stopped waiting for its particle blocks");
    return LB_OK;
}

int ensure_bead_buffers(lb_ctx *c, int n)
{
    const size_t N = c->geo.N;
    const size_t nwords = (N + 31) / 32;
    if (!c->force || !c->fmask) {
        auto release = [&]() {
            (void)hipFree(c->force);
            (void)hipFree(c->fmask);
            c->force = nullptr;
            c->fmask = nullptr;
        };
        release();
        if (!dev_alloc(&c->force, 3 * N * sizeof(long long)) ||
            !dev_alloc(&c->fmask, nwords * sizeof(uint32_t))) {
            release();
            return fail(c, LB_ENOMEM, "bead force field allocation failed");
        }
        hipLaunchKernelGGL(k_zero_f32, dim3(1024), dim3(256), 0, c->stream, reinterpret_cast<float *>(c->force),
                           6 * N);
        hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(nwords, 256)), dim3(256), 0, c->stream,
                           reinterpret_cast<int32_t *>(c->fmask), (uint32_t)nwords);
        LB_LAUNCH_CHECK(c, "zero force field");
    }
    if (n > c->bead_cap) {
        (void)hipFree(c->half);
        (void)hipFree(c->fc);
        (void)hipFree(c->fb2);
        (void)hipFree(c->fp);
        c->half = c->fc = c->fb2 = c->fp = nullptr;
        c->bead_cap = 0;
        const int cap = n < 64 ? 64 : n;
        if (!dev_alloc(&c->half, 3 * (size_t)cap * sizeof(double)) ||
            !dev_alloc(&c->fc, 3 * (size_t)cap * sizeof(double)) ||
            !dev_alloc(&c->fb2, 6 * (size_t)cap * sizeof(double)) ||
            !dev_alloc(&c->fp, 3 * (size_t)cap * sizeof(double)))
            return fail(c, LB_ENOMEM, "bead scratch allocation failed");
        // both bond accumulators start at zero; each call zeroes the other one
        hipLaunchKernelGGL(k_zero_f32, dim3(grid_for(12 * (size_t)cap, 256)), dim3(256), 0, c->stream,
                           reinterpret_cast<float *>(c->fb2), 12 * (size_t)cap);
        LB_LAUNCH_CHECK(c, "zero bond accumulators");
        c->fb_par = 0;
        c->bead_cap = cap;
    }
    return LB_OK;
}



// ---------------------------------------------------------------------------
// differentiation: checkpoints and the adjoint sweep
// ---------------------------------------------------------------------------

size_t state_bytes(const lb_ctx *c) { return (size_t)c->geo.planes * c->geo.N * c->elem; }

// Moments tape: the slot of taped step t.
float *mom_slot(const lb_ctx *c, uint64_t t)
{
    return c->mom_chunks[t / c->mom_chunk_steps] + (size_t)(t % c->mom_chunk_steps) * 4 * (size_t)c->geo.N;
}

// The checkpoints (or, on a moments tape, the moment slots) that the next
// nsteps taped steps will fill, allocated before their first launch (an
// allocation between the launches of a run would stall the queue).
int reserve_checkpoints(lb_ctx *c, int32_t nsteps)
{
    if (!c->taping) return LB_OK;
    if (c->tape_mom) {
        // chunks of up to 64 slots and about 1 GiB
        const size_t per = 4 * sizeof(float) * (size_t)c->geo.N;
        if (c->mom_chunk_steps == 0) c->mom_chunk_steps = std::max<size_t>(1, std::min<size_t>(64, ((size_t)1 << 30) / per));
        const uint64_t need = c->step - c->tape_step0 + (uint64_t)nsteps;
        while ((uint64_t)c->mom_chunks.size() * c->mom_chunk_steps < need) {
            float *p = nullptr;
            if (!dev_alloc(&p, c->mom_chunk_steps * per)) return fail(c, LB_ENOMEM, "moments tape allocation failed");
            c->mom_chunks.push_back(p);
        }
        return LB_OK;
    }
    const uint64_t s0 = c->step - c->tape_step0, K = (uint64_t)c->tape_k;
    const size_t count = (size_t)((s0 + (uint64_t)nsteps) / K - s0 / K);
    while (c->ckpt_ready.size() < count) {
        void *p = nullptr;
        if (!dev_alloc(&p, state_bytes(c))) return fail(c, LB_ENOMEM, "checkpoint allocation failed");
        c->ckpt_ready.push_back(p);
    }
    return LB_OK;
}

int push_checkpoint(lb_ctx *c)
{
    void *p = nullptr;
    if (!c->ckpt_ready.empty()) {
        p = c->ckpt_ready.back();
        c->ckpt_ready.pop_back();
    } else if (!dev_alloc(&p, state_bytes(c))) {
        return fail(c, LB_ENOMEM, "checkpoint allocation failed");
    }
    c->checkpoints.push_back(p);
    return check(c, hipMemcpyAsync(p, c->bufA, state_bytes(c), hipMemcpyDeviceToDevice, c->stream), "checkpoint copy");
}

// Put a state that sits in a slot of the segment buffer back into one of
// the context's own buffers (both are free then).
int settle_state(lb_ctx *c)
{
    if (c->bufA == c->own[0] || c->bufA == c->own[1]) return LB_OK;
    LB_TRY(check(c, hipMemcpyAsync(c->own[0], c->bufA, state_bytes(c), hipMemcpyDeviceToDevice, c->stream),
                 "state copy"));
    c->bufA = c->own[0];
    c->bufB = c->own[1];
    return LB_OK;
}

void free_tape(lb_ctx *c);

// A call that replaces the state or the step counter ends a tape: the
// state it sets is not the end of the taped trajectory.  The state leaves
// the segment buffer first (the taped steps may have left it in a slot).
int end_tape(lb_ctx *c)
{
    if (!c->taping) return LB_OK;
    LB_TRY(settle_state(c));
    free_tape(c);
    return LB_OK;
}

void free_tape(lb_ctx *c)
{
    for (void *p : c->checkpoints) (void)hipFree(p);
    c->checkpoints.clear();
    for (void *p : c->ckpt_ready) (void)hipFree(p);
    c->ckpt_ready.clear();
    for (float *p : c->mom_chunks) (void)hipFree(p);
    c->mom_chunks.clear();
    c->mom_chunk_steps = 0;
    c->tape_mom = false;
    c->taping = false;
    c->seg_fwd = false;
    c->tape_slot.clear();
    c->tape_beads.clear();
    c->tape_off.clear();
    c->tape_bead_used = 0;
    c->pending_slot = -1;
    c->tape_nb = 0;
}

// Cell grid of the WCA pair search for n beads: cells no narrower than
// r_c, at most about 512 n cells and 128 per axis (the heads cost 4 bytes
// per cell; dilute chains cluster, so cells much wider than r_c would give
// long candidate lists), an axis with fewer than 3 cells folded into one.
CellGrid cell_grid(const lb_ctx *c, const lb_beads *b)
{
    CellGrid cg;
    const double sig2 = b->wca_sigma * b->wca_sigma;
    cg.rc2 = std::cbrt(2.0) * sig2;
    cg.sig2 = sig2;
    cg.eps24 = 24.0 * b->wca_epsilon;
    const double rc = std::sqrt(cg.rc2);
    const int cap = std::min(128, std::max(3, (int)std::ceil(std::cbrt(512.0 * (double)b->n))));
    const int32_t ext[3] = {c->p.nx, c->p.ny, c->p.nz};
    for (int a = 0; a < 3; ++a) {
        cg.periodic[a] = (a == 2 && c->p.walls) ? 0 : 1;
        cg.L[a] = (double)ext[a];
        int nc = (int)std::floor(cg.L[a] / rc);
        nc = std::min(nc, cap);
        if (nc < 3) nc = 1;
        cg.nc[a] = nc;
        cg.inv_w[a] = (double)nc / cg.L[a];
    }
    return cg;
}

int ensure_pair_buffers(lb_ctx *c, int n, size_t ncell)
{
    if (ncell > c->cell_cap) {
        (void)hipFree(c->cell_head);
        c->cell_head = nullptr;
        c->cell_cap = 0;
        if (!dev_alloc(&c->cell_head, ncell * sizeof(int32_t)))
            return fail(c, LB_ENOMEM, "cell list allocation failed");
        c->cell_cap = ncell;
        // every head starts at -1 (all bits set); each use puts back the heads it set
        hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(ncell, 256)), dim3(256), 0, c->stream,
                           reinterpret_cast<uint32_t *>(c->cell_head), (uint32_t)ncell, 0xffffffffu);
        LB_LAUNCH_CHECK(c, "reset cell heads");
    }
    if (n > c->pair_cap) {
        (void)hipFree(c->cell_next);
        (void)hipFree(c->cell_of);
        c->cell_next = c->cell_of = nullptr;
        c->pair_cap = 0;
        if (!dev_alloc(&c->cell_next, (size_t)n * sizeof(int32_t)) ||
            !dev_alloc(&c->cell_of, (size_t)n * sizeof(int32_t)))
            return fail(c, LB_ENOMEM, "cell list allocation failed");
        c->pair_cap = n;
    }
    return LB_OK;
}

// WCA forces at the positions `half` (linked into the cell list by
// k_bead_half) into c->fp.
void launch_wca(lb_ctx *c, const lb_beads *b, const double *half, const CellGrid &cg)
{
    hipLaunchKernelGGL(k_wca, dim3(grid_for((size_t)kPairLanes * b->n, 256)), dim3(256), 0, c->stream, half, b->n,
                       cg, c->cell_of, c->cell_head, c->cell_next, c->fp);
}

// Adjoint of the WCA forces at the positions `half`: half_bar += J (fc_bar_i -
// fc_bar_j).  Links the cell list; k_bead_adjoint_finish puts the heads back.
int launch_wca_adjoint(lb_ctx *c, const lb_beads *b, const double *half, const double *fc_bar, double *half_bar)
{
    const CellGrid cg = cell_grid(c, b);
    if (!c->cell_head || !c->cell_of || !c->cell_next || c->pair_cap < b->n ||
        c->cell_cap < (size_t)cg.nc[0] * cg.nc[1] * cg.nc[2])
        return fail(c, LB_EDEVICE, "the pair adjoint needs the context's cell list, which no coupled step allocated");
    hipLaunchKernelGGL(k_cell_link, dim3(grid_for((size_t)b->n, 256)), dim3(256), 0, c->stream, half, b->n, cg,
                       c->cell_of, c->cell_head, c->cell_next);
    hipLaunchKernelGGL(k_wca_adjoint, dim3(grid_for((size_t)kPairLanes * b->n, 256)), dim3(256), 0, c->stream, half,
                       b->n, cg, c->cell_of, c->cell_head, c->cell_next, fc_bar, half_bar);
    return LB_OK;
}

// Threads per block of the per-bead stencil kernels: one wave, so that a few
// thousand beads spread over many CUs (the kernels are latency-bound).
constexpr int kBeadBlock = 64;

// Record of one taped coupled step in the bead tape: P at the start, R',
// F^c and P'' ([n][3] FP64 each), then the spread contributions, one entry
// of four int64 (node or -1, three fixed-point values) per bead and
// stencil lane.
struct TapeSlot {
    double *mom0, *half, *fc, *momn;
    long long *contrib;
    int entries;
};

int stencil_width(const lb_beads *b) { return (b->stencil == 3 || b->stencil == 4) ? b->stencil : 2; }

int stencil_lanes(int W) { return W == 4 ? StencilLanes<4>::value : W == 3 ? StencilLanes<3>::value : StencilLanes<2>::value; }

size_t tape_slot_bytes(const lb_beads *b)
{
    return 12 * (size_t)b->n * sizeof(double) + 4 * (size_t)stencil_lanes(stencil_width(b)) * b->n * sizeof(long long);
}

TapeSlot tape_slot_at(const lb_ctx *c, int slot)
{
    const lb_beads &b = c->tape_beads[slot];
    const size_t n3 = 3 * (size_t)b.n;
    TapeSlot t;
    t.mom0 = reinterpret_cast<double *>(c->tape_bead + c->tape_off[slot]);
    t.half = t.mom0 + n3;
    t.fc = t.half + n3;
    t.momn = t.fc + n3;
    t.contrib = reinterpret_cast<long long *>(t.momn + n3);
    t.entries = stencil_lanes(stencil_width(&b)) * b.n;
    return t;
}

// The particle half of one coupled step (k_bead_half with the bonds, the WCA
// pair search, k_bead_update) on the populations `pop`: (pos_in, mom_in) ->
// (pos, mom) (the same arrays for lb_couple), spreading into the force field
// and its bitmap, with R' and F^c in c->half, c->fc, or, for a taped step, in
// its tape slot together with P, P'' and the contributions.
void launch_couple(lb_ctx *c, const void *pop, const lb_beads *b, const double *pos_in, const double *mom_in,
                   double *pos, double *mom, uint32_t step, const TapeSlot *tape = nullptr)
{
    CoupleArgs a;
    a.pop = pop;
    a.geo = c->geo;
    a.rho0 = c->p.rho0;
    for (int k = 0; k < 3; ++k) a.g[k] = c->p.body_force[k];
    a.kT = c->p.kT;
    a.key0 = c->cc.key0;
    a.key1 = c->cc.key1;
    a.box = c->cc.box;
    a.step = step;
    a.n = b->n;
    a.pos_in = pos_in;
    a.mom_in = mom_in;
    a.pos = pos;
    a.mom = mom;
    a.mass = b->mass;
    a.zeta = b->zeta;
    a.half = tape ? tape->half : c->half;
    a.fc = tape ? tape->fc : c->fc;
    const size_t n3cap = 3 * (size_t)c->bead_cap;
    a.fb = c->fb2 + (size_t)c->fb_par * n3cap;
    a.fb_next = c->fb2 + (size_t)(c->fb_par ^ 1) * n3cap;
    c->fb_par ^= 1;
    a.cap = c->bead_cap;
    const bool wca = b->wca_epsilon > 0.0;
    a.fp = wca ? c->fp : nullptr;
    a.fext = b->fext;
    a.bonds = b->bonds;
    a.nbonds = b->nbonds;
    a.fene = (int32_t)(b->bond == LB_BOND_FENE);
    a.three_point = (int32_t)(b->noise == LB_NOISE_THREE_POINT);
    a.kb = b->k_bond;
    a.r0 = b->r0;
    a.flags = c->flags;
    a.force = c->force;
    a.fmask = c->fmask;
    a.tape_mom0 = tape ? tape->mom0 : nullptr;
    a.tape_momn = tape ? tape->momn : nullptr;
    a.tape_contrib = tape ? tape->contrib : nullptr;
    a.cell_head = wca ? c->cell_head : nullptr;
    a.cell_next = c->cell_next;
    a.cell_of = c->cell_of;
    if (wca) a.cg = cell_grid(c, b);
    const size_t roles = std::max<size_t>({(size_t)b->n, (size_t)b->nbonds, (size_t)c->bead_cap});
    hipLaunchKernelGGL(k_bead_half, dim3(grid_for(roles, 256)), dim3(256), 0, c->stream, a);
    if (wca) launch_wca(c, b, a.half, a.cg);
    by_storage(c->p.storage, [&](auto st) {
        constexpr int ST = decltype(st)::value;
        by_stencil(b->stencil, [&](auto w) {
            constexpr int W = decltype(w)::value;
            hipLaunchKernelGGL((k_bead_update<ST, W>),
                               dim3(grid_for(StencilLanes<W>::value * (size_t)b->n, kBeadBlock)), dim3(kBeadBlock), 0,
                               c->stream, a);
        });
    });
}

// Reserves the tape slot of a taped coupled step (the particle half's
// kernels fill it).
// Room in the bead tape for `slots` more records of b (at most one
// reallocation, which waits for the stream: a run of taped steps asks for
// all of its slots before its first launch).
int tape_grow(lb_ctx *c, const lb_beads *b, size_t slots)
{
    const size_t need = slots * tape_slot_bytes(b);
    if (c->tape_bead_used + need > c->tape_bead_bytes) {
        const size_t cap = std::max<size_t>(16 * tape_slot_bytes(b), 2 * (c->tape_bead_used + need));
        char *p = nullptr;
        if (!dev_alloc(&p, cap)) return fail(c, LB_ENOMEM, "bead tape allocation failed");
        if (c->tape_bead && c->tape_bead_used > 0)
            LB_TRY(check(c, hipMemcpyAsync(p, c->tape_bead, c->tape_bead_used, hipMemcpyDeviceToDevice, c->stream),
                         "bead tape copy"));
        if (c->tape_bead) {
            LB_TRY(check(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize"));
            (void)hipFree(c->tape_bead);
        }
        c->tape_bead = p;
        c->tape_bead_bytes = cap;
    }
    return LB_OK;
}

int tape_reserve(lb_ctx *c, const lb_beads *b, TapeSlot *out)
{
    if (c->tape_nb == 0) c->tape_nb = b->n;
    if (b->n != c->tape_nb)
        return fail(c, LB_EUNSUPPORTED, "the bead count must stay the same over the taped steps");
    LB_TRY(tape_grow(c, b, 1));
    const size_t need = tape_slot_bytes(b);
    c->tape_off.push_back(c->tape_bead_used);
    c->tape_bead_used += need;
    c->tape_beads.push_back(*b);
    c->pending_slot = (int)c->tape_beads.size() - 1;
    *out = tape_slot_at(c, c->pending_slot);
    return LB_OK;
}

// Geometry and element size of a single box (z-major layout).
void init_single_box(lb_ctx *c, const lb_params *p)
{
    const uint32_t nx = p->nx, ny = p->ny, nz = p->nz;
    c->geo.nx = nx;
    c->geo.ny = ny;
    c->geo.nz = nz;
    c->geo.nxny = nx * ny;
    c->geo.N = nx * ny * nz;
    c->geo.div_nx = make_fastdiv(nx);
    c->geo.div_ny = make_fastdiv(ny);
    c->geo.walls = (uint32_t)p->walls;
    c->geo.zmajor = 1u;
    c->geo.planes = state_planes(p->storage);
    c->elem = storage_bytes(p->storage);
}

StepArgs plain_step_args(lb_ctx *c, const void *src, void *dst, uint32_t step)
{
    StepArgs a;
    a.src = src;
    a.dst = dst;
    a.geo = c->geo;
    a.tiles = (c->geo.nxny + (uint32_t)c->block - 1u) / (uint32_t)c->block;
    a.div_tiles = make_fastdiv(a.tiles);
    a.cc = c->cc;
    a.step = step;
    a.xcd_remap = c->xcd_remap;
    a.partials = c->partials;
    a.flags = c->flags;
    a.fmask = nullptr;
    a.force = nullptr;
    a.consume = 0u;
    a.arrive = nullptr;
    a.arrive_target = 0u;
    a.block0 = 0u;
    a.moments = nullptr;
    return a;
}

// ---------------------------------------------------------------------------
// batched replicas and launch-configuration search
// ---------------------------------------------------------------------------

// Orders the context's private stream after the caller's stream at entry and
// the caller's stream after the private stream at exit (batch contexts only).
struct Join {
    lb_ctx *c;
    explicit Join(lb_ctx *cc) : c(cc)
    {
        if (c && c->batch) {
            (void)hipEventRecord(c->ev_in, c->user_stream);
            (void)hipStreamWaitEvent(c->stream, c->ev_in, 0);
        }
    }
    ~Join()
    {
        if (c && c->batch) {
            (void)hipEventRecord(c->ev_out, c->stream);
            (void)hipStreamWaitEvent(c->user_stream, c->ev_out, 0);
        }
    }
};

int batch_build_tiles(lb_ctx *c, int block)
{
    std::vector<uint32_t> tiles;
    uint32_t first = 0;
    for (int b = 0; b < c->nbox; ++b) {
        BoxDesc &d = c->boxes_h[b];
        const uint32_t nt = (d.geo.N + block - 1) / block;
        d.first_tile = first;
        for (uint32_t t = 0; t < nt; ++t) tiles.push_back((uint32_t)b);
        first += nt;
    }
    c->ntiles = first;
    (void)hipFree(c->tile_box);
    c->tile_box = nullptr;
    if (!dev_alloc(&c->tile_box, tiles.size() * sizeof(uint32_t)))
        return fail(c, LB_ENOMEM, "tile table allocation failed");
    LB_TRY(check(c, hipMemcpyAsync(c->tile_box, tiles.data(), tiles.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                                   c->stream), "tile table upload"));
    LB_TRY(check(c, hipMemcpyAsync(c->boxes_d, c->boxes_h.data(), c->boxes_h.size() * sizeof(BoxDesc),
                                   hipMemcpyHostToDevice, c->stream), "box table upload"));
    LB_TRY(check(c, hipStreamSynchronize(c->stream), "tile table sync"));
    c->block = block;
    return LB_OK;
}

template <int ST, bool TH, bool VA>
void batch_launch_t(lb_ctx *c, const BatchArgs &a, unsigned grid)
{
    if (TH && c->full_relax)
        hipLaunchKernelGGL((k_batch_step<ST, TH, VA, TH>), dim3(grid), dim3(c->block), 0, c->stream, a);
    else
        hipLaunchKernelGGL((k_batch_step<ST, TH, VA, false>), dim3(grid), dim3(c->block), 0, c->stream, a);
}

void batch_launch_step(lb_ctx *c, const void *src, void *dst, bool vacf)
{
    BatchArgs a;
    a.src = src;
    a.dst = dst;
    a.boxes = c->boxes_d;
    a.tile_box = c->tile_box;
    a.ntiles = c->ntiles;
    a.chunk = c->chunk;
    a.cc = c->cc;
    a.step_ptr = c->dstep;
    a.amp = c->amp;
    a.flags = c->flags;
    const unsigned grid = (c->ntiles + c->chunk - 1) / c->chunk;
    c->nblocks = (int)grid;
    by_step_storage(c->p, [&](auto st) {
        constexpr int ST = decltype(st)::value;
        if (c->thermal) {
            if (vacf) batch_launch_t<ST, true, true>(c, a, grid);
            else batch_launch_t<ST, true, false>(c, a, grid);
        } else {
            if (vacf) batch_launch_t<ST, false, true>(c, a, grid);
            else batch_launch_t<ST, false, false>(c, a, grid);
        }
    });
}

// One batched time step: fused step kernel, VACF sample, counter advance.
void batch_enqueue_step(lb_ctx *c, const void *src, void *dst)
{
    const bool vacf = c->p.vacf_lags > 0;
    batch_launch_step(c, src, dst, vacf);
    if (vacf) {
        const int R = c->p.vacf_lags;
        hipLaunchKernelGGL(k_vacf_update, dim3(c->nbox), dim3(std::max(R, 64)), 0, c->stream, c->amp, c->boxes_d,
                           (uint32_t)c->block, c->ring, c->corr, R, c->dstep + 1);
    }
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, c->stream, c->dstep, c->dstep + 1, vacf ? 1 : 0);
}

// Mean duration of one launch: a warm-up launch, one timed launch to size the
// repetition count, then at least `reps` launches and about 2 ms in total.
float time_launches(lb_ctx *c, int reps, const std::function<void()> &launch)
{
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    auto timed = [&](int n) {
        (void)hipEventRecord(e0, c->stream);
        for (int r = 0; r < n; ++r) launch();
        (void)hipEventRecord(e1, c->stream);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        return ms / n;
    };
    launch();  // warm-up
    const float first = timed(1);
    // about 8 ms per measurement: a few launches of a large box differ by
    // several per cent from run to run, more than the candidates differ
    const int n = std::max(reps, std::min(400, (int)(8.0f / std::max(first, 1e-3f))));
    const float ms = timed(n);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
}

// Launch-configuration search of a batch: each candidate (threads per block x
// blocks per step) runs the step kernel from A into B (the state and the step
// counter are not advanced) and the fastest is kept.
int autotune(lb_ctx *c)
{
    if (c->batch) {
        // blocks per CU of the persistent launch; 0 = one tile per block (no
        // tile loop, the hardware deals tiles out); with the VACF the
        // candidates run the VACF variant of the kernel
        // Two passes over the candidates, each candidate's better time
        // counts (one pass of a few launches has picked a configuration
        // several per cent slower than the best).
        const int blocks[] = {128, 256, 512, 1024};
        const int per_cu[] = {2, 4, 8, 16, 0};
        float t[4][5];
        float best = 1e30f;
        int bb = 256;
        uint32_t bc = 1;
        for (int pass = 0; pass < 2; ++pass)
            for (int ib = 0; ib < 4; ++ib) {
                LB_TRY(batch_build_tiles(c, blocks[ib]));
                for (int ip = 0; ip < 5; ++ip) {
                    const int pc = per_cu[ip];
                    const uint32_t grid = pc > 0 ? 256u * (uint32_t)pc : c->ntiles;
                    c->chunk = std::max<uint32_t>(1u, (c->ntiles + grid - 1) / grid);
                    const float ms =
                        time_launches(c, 3, [&] { batch_launch_step(c, c->bufA, c->bufB, c->p.vacf_lags > 0); });
                    LB_LAUNCH_CHECK(c, "autotune batch");
                    t[ib][ip] = pass == 0 ? ms : std::min(t[ib][ip], ms);
                    if (pass == 1 && t[ib][ip] < best) {
                        best = t[ib][ip];
                        bb = blocks[ib];
                        bc = c->chunk;
                    }
                }
            }
        LB_TRY(batch_build_tiles(c, bb));
        c->chunk = bc;
        c->nblocks = (int)((c->ntiles + c->chunk - 1) / c->chunk);
    }
    c->tuned = true;
    return LB_OK;
}

// Single box: search threads per block x XCD remap for the step kernel
// variant with or without bead force; each candidate runs the kernel from A
// into B without advancing the state (with a pending force the force buffers
// hold this step's force and are only read).
int autotune_single(lb_ctx *c, bool frc)
{
    const int blocks[] = {64, 128, 256, 512, 1024};
    float best = 1e30f;
    const int k = frc ? 1 : 0;
    // two passes over the candidates, each candidate's better time counts
    float t[10];
    for (int pass = 0; pass < 2; ++pass)
    for (int cand = 0; cand < 10; ++cand) {
        c->block = blocks[cand >> 1];
        c->xcd_remap = (uint32_t)(cand & 1);
        c->nblocks = (int)step_blocks(c, c->block);
        StepArgs a = plain_step_args(c, c->bufA, c->bufB, (uint32_t)c->step);
        if (frc) {
            a.fmask = c->fmask;
            a.force = c->force;
        }
        const bool tot = c->p.track_totals != 0;
        const float ms = time_launches(c, 3, [&] {
            by_step_storage(c->p, [&](auto st) { launch_step_st<decltype(st)::value>(c, a, tot, frc); });
        });
        LB_LAUNCH_CHECK(c, "autotune");
        t[cand] = pass == 0 ? ms : std::min(t[cand], ms);
        if (pass == 1 && t[cand] < best) {
            best = t[cand];
            c->block_f[k] = c->block;
            c->remap_f[k] = c->xcd_remap;
        }
    }
    c->tuned_f[k] = true;
    return LB_OK;
}

// Launch configuration of the next single-box step launch.
int select_launch(lb_ctx *c, bool frc)
{
    const int k = frc ? 1 : 0;
    if (c->search && !c->tuned_f[k]) LB_TRY(autotune_single(c, frc));
    c->block = c->block_f[k];
    c->xcd_remap = c->remap_f[k];
    c->nblocks = (int)step_blocks(c, c->block);
    return LB_OK;
}


int batch_step(lb_ctx *c, int32_t nsteps)
{
    if (!c->tuned) LB_TRY(autotune(c));
    const int G = c->p.graph_steps;
    int32_t done = 0;
    if (G > 0) {
        while (nsteps - done >= G) {
            const int par = (c->bufA == c->buf0) ? 0 : 1;
            if (!c->graph_exec[par]) {
                hipGraph_t g = nullptr;
                LB_TRY(check(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal), "begin capture"));
                void *A = c->bufA, *B = c->bufB;
                for (int k = 0; k < G; ++k) {
                    batch_enqueue_step(c, A, B);
                    std::swap(A, B);
                }
                LB_TRY(check(c, hipStreamEndCapture(c->stream, &g), "end capture"));
                LB_TRY(check(c, hipGraphInstantiate(&c->graph_exec[par], g, nullptr, nullptr, 0), "instantiate"));
                (void)hipGraphDestroy(g);
            }
            LB_TRY(check(c, hipGraphLaunch(c->graph_exec[par], c->stream), "graph launch"));
            // G is even: the buffers are back in the same roles
            done += G;
            c->step += (uint64_t)G;
        }
    }
    for (; done < nsteps; ++done) {
        batch_enqueue_step(c, c->bufA, c->bufB);
        LB_LAUNCH_CHECK(c, "batch step");
        std::swap(c->bufA, c->bufB);
        ++c->step;
    }
    c->totals_valid = false;
    return LB_OK;
}

// Output buffer of the next single-box step: bufB; while taping, for the
// step that ends a segment a new checkpoint buffer (*ckpt = true: the step
// writes the checkpoint itself, which then holds the state until the next
// step reads it; nothing writes into it afterwards, and a call that replaces
// the state in place first moves it to an own buffer, settle_state), and
// inside a segment the segment buffer's next slot (the step buffer the
// reverse sweep would otherwise recompute).
int step_dst(lb_ctx *c, void **dst, bool *ckpt)
{
    *dst = c->bufB;
    *ckpt = false;
    if (!c->taping || c->tape_mom) return LB_OK;
    const uint64_t k = (c->step - c->tape_step0) % (uint64_t)c->tape_k;
    if (k + 1 == (uint64_t)c->tape_k) {
        if (!c->ckpt_ready.empty()) {
            *dst = c->ckpt_ready.back();
            c->ckpt_ready.pop_back();
        } else if (!dev_alloc(dst, state_bytes(c))) {
            return fail(c, LB_ENOMEM, "checkpoint allocation failed");
        }
        *ckpt = true;
    } else if (c->seg_fwd) {
        *dst = static_cast<char *>(c->seg) + (size_t)(k + 1) * state_bytes(c);
    }
    return LB_OK;
}

// Bookkeeping after a single-box step launch that wrote the state to dst
// (ckpt: dst is the checkpoint of the segment the step ended).
int step_done(lb_ctx *c, void *dst, bool tot, bool ckpt)
{
    // the state moves to dst; bufB becomes an own buffer that does not hold it
    c->bufB = (c->bufA == c->own[0] || c->bufA == c->own[1]) ? c->bufA : (dst == c->own[0] ? c->own[1] : c->own[0]);
    c->bufA = dst;
    ++c->step;
    c->totals_valid = tot;
    if (ckpt) c->checkpoints.push_back(dst);
    return LB_OK;
}

// Argument checks of lb_couple and lb_coupled_steps (LB_OK: go on).
int couple_check(lb_ctx *c, const lb_beads *b)
{
    if (c->batch) return fail(c, LB_EUNSUPPORTED, "bead coupling is not available on a batch context");
    if (!b) return fail(c, LB_EINVAL, "beads is NULL");
    if (b->n < 0 || b->nbonds < 0) return fail(c, LB_EINVAL, "bead and bond counts must be >= 0");
    if (b->n > (1 << 26)) return fail(c, LB_EINVAL, "too many beads");
    if (c->pending_force) return fail(c, LB_ESTATE, "lb_couple called twice without lb_step");
    if (b->n == 0) return LB_OK;
    if (!b->pos || !b->mom || !b->mass || !b->zeta || (b->nbonds > 0 && !b->bonds))
        return fail(c, LB_EINVAL, "bead arrays must be non-NULL");
    if (!std::isfinite(b->k_bond) || !std::isfinite(b->r0)) return fail(c, LB_EINVAL, "bond parameters must be finite");
    if (b->stencil != 0 && b->stencil != 2 && b->stencil != 3 && b->stencil != 4)
        return fail(c, LB_EINVAL, "stencil must be 0, 2, 3 or 4");
    if (b->bond != LB_BOND_HARMONIC && b->bond != LB_BOND_FENE) return fail(c, LB_EINVAL, "unknown bond kind");
    if (b->noise != LB_NOISE_GAUSSIAN && b->noise != LB_NOISE_THREE_POINT)
        return fail(c, LB_EINVAL, "unknown bead noise distribution");
    if (b->bond == LB_BOND_FENE && b->nbonds > 0 && !(b->r0 > 0.0 && b->k_bond >= 0.0))
        return fail(c, LB_EINVAL, "FENE bonds need r0 > 0 and k_bond >= 0");
    if (!(std::isfinite(b->wca_epsilon) && b->wca_epsilon >= 0.0))
        return fail(c, LB_EINVAL, "wca_epsilon must be finite and >= 0");
    const bool wca = b->wca_epsilon > 0.0;
    if (wca) {
        if (!(std::isfinite(b->wca_sigma) && b->wca_sigma > 0.0))
            return fail(c, LB_EINVAL, "wca_sigma must be finite and > 0");
        const double rc = std::cbrt(std::sqrt(2.0)) * b->wca_sigma;
        const int32_t lmin = std::min(c->p.nx, c->p.walls ? c->p.ny : std::min(c->p.ny, c->p.nz));
        if (!(2.0 * rc < (double)lmin))
            return fail(c, LB_EINVAL, "the WCA cutoff 2^(1/6) sigma must be below half of every periodic box extent");
    }
    return LB_OK;
}

// Bond partners of each bead for the fused coupled step: table [n][deg] in
// bond-list order, -1 padded (bonds with an index outside [0, n) are
// skipped, as bond_force does).  *deg = 0 without bonds; *ok = false if the
// largest degree exceeds kMaxFusedDegree (those runs take separate launches).
constexpr int kMaxFusedDegree = 64;

int build_partners(lb_ctx *c, const lb_beads *b, int *deg, bool *ok)
{
    *deg = 0;
    *ok = true;
    if (b->nbonds == 0) return LB_OK;
    std::vector<int32_t> bonds(2 * (size_t)b->nbonds);
    LB_TRY(check(c, hipMemcpyAsync(bonds.data(), b->bonds, bonds.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                                   c->stream), "bond list copy"));
    LB_TRY(check(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize"));
    const int n = b->n;
    std::vector<int32_t> cnt((size_t)n, 0);
    auto valid = [&](size_t q) {
        const int32_t ia = bonds[2 * q], ib = bonds[2 * q + 1];
        return ia >= 0 && ib >= 0 && ia < n && ib < n;
    };
    for (size_t q = 0; q < (size_t)b->nbonds; ++q)
        if (valid(q)) {
            ++cnt[bonds[2 * q]];
            ++cnt[bonds[2 * q + 1]];
        }
    int d = 0;
    for (int v : cnt) d = std::max(d, v);
    if (d > kMaxFusedDegree) {
        *ok = false;
        return LB_OK;
    }
    *deg = d;
    if (d == 0) return LB_OK;
    std::vector<int32_t> tab((size_t)n * d, -1);
    std::fill(cnt.begin(), cnt.end(), 0);
    for (size_t q = 0; q < (size_t)b->nbonds; ++q)
        if (valid(q)) {
            const int32_t ia = bonds[2 * q], ib = bonds[2 * q + 1];
            tab[(size_t)ia * d + cnt[ia]++] = ib;
            tab[(size_t)ib * d + cnt[ib]++] = ia;
        }
    if (c->partner_cap < tab.size()) {
        (void)hipFree(c->partner);
        c->partner = nullptr;
        c->partner_cap = 0;
        if (!dev_alloc(&c->partner, tab.size() * sizeof(int32_t)))
            return fail(c, LB_ENOMEM, "bond partner table allocation failed");
        c->partner_cap = tab.size();
    }
    // synchronous: the host table goes out of scope
    LB_TRY(check(c, hipMemcpyAsync(c->partner, tab.data(), tab.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                   c->stream), "bond partner table upload"));
    return check(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
}

// Buffers of the fused coupled step: the alternate bead states, the second
// bitmap and the particle block counter.
int ensure_fused_buffers(lb_ctx *c, int n)
{
    if (!c->fmask_f || !c->arrive) {
        const size_t nwords = ((size_t)c->geo.N + 31) / 32;
        if (!dev_alloc(&c->fmask_f, nwords * sizeof(uint32_t)) ||
            !dev_alloc(&c->arrive, sizeof(uint32_t)))
            return fail(c, LB_ENOMEM, "fused step buffers allocation failed");
        hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(nwords, 256)), dim3(256), 0, c->stream,
                           reinterpret_cast<int32_t *>(c->fmask_f), (uint32_t)nwords);
        hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, c->stream, reinterpret_cast<int32_t *>(c->arrive), 1u);
        LB_LAUNCH_CHECK(c, "zero fused step buffers");
        c->arrive_count = 0;
    }
    if (n > c->bead_pp_cap) {
        (void)hipFree(c->bead_pp);
        c->bead_pp = nullptr;
        c->bead_pp_cap = 0;
        if (!dev_alloc(&c->bead_pp, 12 * (size_t)n * sizeof(double)))
            return fail(c, LB_ENOMEM, "fused step bead buffers allocation failed");
        c->bead_pp_cap = n;
    }
    return LB_OK;
}

// The three rotating cell lists of fused steps with WCA pairs: heads all -1
// on entry and after every call.
int ensure_fused_lists(lb_ctx *c, int n, size_t ncell)
{
    if (c->flist && c->flist_cells >= ncell && c->flist_n >= n) return LB_OK;
    (void)hipFree(c->flist);
    c->flist = nullptr;
    c->flist_cells = 0;
    c->flist_n = 0;
    const size_t words = 3 * ncell + 6 * (size_t)n;
    if (!dev_alloc(&c->flist, words * sizeof(int32_t)))
        return fail(c, LB_ENOMEM, "fused cell lists allocation failed");
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(3 * ncell, 256)), dim3(256), 0, c->stream,
                       reinterpret_cast<uint32_t *>(c->flist), (uint32_t)(3 * ncell), 0xffffffffu);
    LB_LAUNCH_CHECK(c, "fused cell lists");
    c->flist_cells = ncell;
    c->flist_n = n;
    return LB_OK;
}

template <int ST, bool TH, bool TOT, int W, bool PAIRS, bool MOM = false>
void launch_fused_t(lb_ctx *c, const StepArgs &a, const ParticleArgs &p, unsigned grid)
{
    const size_t lds = TOT ? (size_t)kTotalsLds * (size_t)c->block : 0;  // block_sum_totals
    if (TH && c->full_relax)
        hipLaunchKernelGGL((k_coupled_step<ST, TH, TOT, TH, W, PAIRS, MOM>), dim3(grid), dim3(c->block), lds, c->stream,
                           a, p);
    else
        hipLaunchKernelGGL((k_coupled_step<ST, TH, TOT, false, W, PAIRS, MOM>), dim3(grid), dim3(c->block), lds,
                           c->stream, a, p);
}

// mom: a step of a moments tape (no fused totals; phi_2 only, the caller
// takes the separate launches for the wider kernels)
template <int ST, int W, bool PAIRS>
void launch_fused_st(lb_ctx *c, const StepArgs &a, const ParticleArgs &p, unsigned grid, bool tot, bool mom)
{
    if constexpr (W == 2) {
        if (mom) {
            if (c->thermal) launch_fused_t<ST, true, false, W, PAIRS, true>(c, a, p, grid);
            else launch_fused_t<ST, false, false, W, PAIRS, true>(c, a, p, grid);
            return;
        }
    }
    if (c->thermal) {
        if (tot) launch_fused_t<ST, true, true, W, PAIRS>(c, a, p, grid);
        else launch_fused_t<ST, true, false, W, PAIRS>(c, a, p, grid);
    } else {
        if (tot) launch_fused_t<ST, false, true, W, PAIRS>(c, a, p, grid);
        else launch_fused_t<ST, false, false, W, PAIRS>(c, a, p, grid);
    }
}

// The step kernel of the reverse sweep's recompute and of a moments tape's
// forward (k_recompute_step): with frc the bead force of a.force, with mom
// the input state's moments written to a.moments (one of the two at least),
// and in extra blocks the recorded force of the next taped coupled step put
// back (entries > 0).  site_blocks blocks of `block` threads take the sites,
// the tile of block b being b (a.xcd_remap = 0).
void launch_recompute(lb_ctx *c, const StepArgs &a, int block, uint32_t site_blocks, bool frc, bool mom,
                      const long long *contrib, int entries, long long *force_next, uint32_t *fmask_next)
{
    const unsigned grid = site_blocks + (entries > 0 ? grid_for((size_t)entries, block) : 0u);
    by_step_storage(c->p, [&](auto st) {
        constexpr int ST = decltype(st)::value;
        auto go = [&](auto th, auto walls, auto full) {
            constexpr bool TH = decltype(th)::value, WL = decltype(walls)::value, FU = decltype(full)::value;
            // (force, moments): (yes, yes), (yes, no), (no, yes)
            if (frc && mom)
                hipLaunchKernelGGL((k_recompute_step<ST, TH, WL, FU, true, true>), dim3(grid), dim3(block), 0,
                                   c->stream, a, site_blocks, contrib, entries, force_next, fmask_next);
            else if (frc)
                hipLaunchKernelGGL((k_recompute_step<ST, TH, WL, FU, true, false>), dim3(grid), dim3(block), 0,
                                   c->stream, a, site_blocks, contrib, entries, force_next, fmask_next);
            else
                hipLaunchKernelGGL((k_recompute_step<ST, TH, WL, FU, false, true>), dim3(grid), dim3(block), 0,
                                   c->stream, a, site_blocks, contrib, entries, force_next, fmask_next);
        };
        using T_ = std::true_type;
        using F_ = std::false_type;
        const bool full = c->thermal && c->full_relax;
        if (c->geo.walls) {
            if (!c->thermal) go(F_{}, T_{}, F_{});
            else if (full) go(T_{}, T_{}, T_{});
            else go(T_{}, T_{}, F_{});
        } else {
            if (!c->thermal) go(F_{}, F_{}, F_{});
            else if (full) go(T_{}, F_{}, T_{});
            else go(T_{}, F_{}, F_{});
        }
    });
}

}  // namespace

// A ROCTX range around each entry point (named after it): a profiler run
// with marker tracing shows the host-side span of every library call.
struct CallRange {
    explicit CallRange(const char *name) { roctxRangePushA(name); }
    ~CallRange() { roctxRangePop(); }
    CallRange(const CallRange &) = delete;
    CallRange &operator=(const CallRange &) = delete;
};
#define LB_RANGE() CallRange lb_call_range_(__func__)

extern "C" {

int lb_params_two_rate(double gamma_e, double magic, lb_params *params)
{
    if (!params) return fail(nullptr, LB_EINVAL, "params is NULL");
    if (!(std::fabs(gamma_e) < 1.0)) return fail(nullptr, LB_EINVAL, "two-rate relaxation needs |gamma_e| < 1");
    if (!(magic > 0.0) || !std::isfinite(magic)) return fail(nullptr, LB_EINVAL, "magic must be finite and > 0");
    // relaxation times tau = 1 / (1 - gamma); Lambda = (tau_e - 1/2)(tau_o - 1/2)
    const double tau_e = 1.0 / (1.0 - gamma_e);
    const double tau_o = 0.5 + magic / (tau_e - 0.5);
    const double gamma_o = 1.0 - 1.0 / tau_o;
    params->gamma_shear = params->gamma_bulk = params->gamma_4a = params->gamma_4b = gamma_e;
    params->gamma_3a = params->gamma_3b = gamma_o;
    return LB_OK;
}

int lb_create(const lb_params *params, void *stream, lb_ctx **out)
{
    LB_RANGE();
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
    c->user_stream = c->stream;
    init_single_box(c, params);
    c->block = params->block > 0 ? params->block : 256;
    c->tuned = true;
    c->search = params->block == -1;
    c->block_f[0] = c->block_f[1] = c->block;
    c->nblocks = (int)step_blocks(c, c->block);
    fill_collide_const(c);
    const size_t bytes = state_bytes(c);
    // per-block totals rows: the most blocks any block size gives (64 threads)
    const size_t rows = std::max<size_t>(grid_for(c->geo.N, 64), step_blocks(c, 64));
    if (!dev_alloc(&c->bufA, bytes) || !dev_alloc(&c->bufB, bytes) ||
        !dev_alloc(&c->partials, rows * 4 * sizeof(double)) ||
        !dev_alloc(&c->dev_out, 64 * sizeof(double)) || !dev_alloc(&c->flags, sizeof(int32_t))) {
        lb_destroy(c);
        return fail(nullptr, LB_ENOMEM, "device allocation failed");
    }
    c->buf0 = c->bufA;
    c->own[0] = c->bufA;
    c->own[1] = c->bufB;
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, c->stream, c->flags, 1u);
    if (hipGetLastError() != hipSuccess) {
        lb_destroy(c);
        return fail(nullptr, LB_EDEVICE, "kernel launch failed in lb_create");
    }
    *out = c;
    return LB_OK;
}

int lb_create_batch(const lb_params *params, int32_t nbox, const int32_t *dims, void *stream, lb_ctx **out)
{
    LB_RANGE();
    std::string msg;
    if (!out) return fail(nullptr, LB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!params || !dims || nbox < 1) return fail(nullptr, LB_EINVAL, "need params, dims and nbox >= 1");
    lb_params p = *params;
    p.nx = dims[0];
    p.ny = dims[1];
    p.nz = dims[2];
    const int v = validate(&p, msg);
    if (v != LB_OK) return fail(nullptr, v, msg);
    if (p.graph_steps < 0 || (p.graph_steps & 1)) return fail(nullptr, LB_EINVAL, "graph_steps must be even and >= 0");
    if (p.walls) return fail(nullptr, LB_EUNSUPPORTED, "walls are available for a single box only");
    if (p.vacf_lags < 0 || p.vacf_lags > 1024) return fail(nullptr, LB_EINVAL, "vacf_lags must be in [0, 1024]");
    // every box's extents before any device call
    uint64_t total = 0;
    for (int b = 0; b < nbox; ++b) {
        const int32_t *e = dims + 3 * b;
        if (e[0] < 2 || e[1] < 2 || e[2] < 2) return fail(nullptr, LB_EINVAL, "every box extent must be >= 2");
        const uint64_t Nb = (uint64_t)e[0] * e[1] * e[2];
        if (Nb >= (1ull << 30)) return fail(nullptr, LB_EINVAL, "box site count must be < 2^30");
        total += Nb;
    }
    if (total >= (1ull << 31)) return fail(nullptr, LB_EINVAL, "total site count must be < 2^31");
    lb_ctx *c = new lb_ctx();
    c->p = p;
    c->batch = true;
    c->nbox = nbox;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(nullptr, LB_EDEVICE, "no HIP device");
    }
    uint64_t off = 0;
    for (int b = 0; b < nbox; ++b) {
        const int32_t *e = dims + 3 * b;
        const uint64_t Nb = (uint64_t)e[0] * e[1] * e[2];
        BoxDesc d{};
        d.geo.nx = e[0];
        d.geo.ny = e[1];
        d.geo.nz = e[2];
        d.geo.nxny = (uint32_t)(e[0] * e[1]);
        d.geo.N = (uint32_t)Nb;
        d.geo.div_nx = make_fastdiv(e[0]);
        d.geo.div_ny = make_fastdiv(e[1]);
        d.geo.planes = state_planes(p.storage);
        d.off = off;
        d.box_id = (uint32_t)(p.box_id + b);
        d.inv_L[0] = 1.0f / (float)e[0];
        d.inv_L[1] = 1.0f / (float)e[1];
        d.inv_L[2] = 1.0f / (float)e[2];
        c->boxes_h.push_back(d);
        off += (uint64_t)d.geo.planes * Nb;
        c->total_sites += Nb;
    }
    c->geo = c->boxes_h[0].geo;  // first box (diagnostic helpers loop over all boxes)
    c->elem = storage_bytes(p.storage);
    fill_collide_const(c);
    c->user_stream = static_cast<hipStream_t>(stream);
    const size_t bytes = (size_t)off * c->elem;
    const int R = p.vacf_lags;
    // VACF rows: one per tile of the smallest tile (64 sites) any launch uses
    size_t amp_rows = 0;
    for (const BoxDesc &d : c->boxes_h) amp_rows += (d.geo.N + 63u) / 64u;
    bool ok = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) == hipSuccess;
    ok = ok && dev_alloc(&c->bufA, bytes) && dev_alloc(&c->bufB, bytes) &&
         dev_alloc(&c->boxes_d, nbox * sizeof(BoxDesc)) &&
         dev_alloc(&c->dstep, 2 * sizeof(uint32_t)) &&
         dev_alloc(&c->dev_out, 64 * sizeof(double)) && dev_alloc(&c->flags, sizeof(int32_t));
    if (ok && R > 0)
        ok = dev_alloc(&c->amp, amp_rows * 12 * sizeof(float)) &&
             dev_alloc(&c->ring, (size_t)nbox * R * 12 * sizeof(float)) &&
             dev_alloc(&c->corr, (size_t)nbox * R * sizeof(double));
    if (!ok) {
        lb_destroy(c);
        return fail(nullptr, LB_ENOMEM, "batch allocation failed");
    }
    c->buf0 = c->bufA;
    c->own[0] = c->bufA;
    c->own[1] = c->bufB;
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, c->stream, c->flags, 1u);
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, c->stream, reinterpret_cast<int32_t *>(c->dstep), 2u);
    if (R > 0) {
        hipLaunchKernelGGL(k_zero_f32, dim3(256), dim3(256), 0, c->stream, reinterpret_cast<float *>(c->corr),
                           (size_t)nbox * R * 2);
    }
    c->block = p.block > 0 ? p.block : 256;
    c->tuned = p.block > 0;
    if (batch_build_tiles(c, c->block) != LB_OK || hipGetLastError() != hipSuccess) {
        const std::string e = c->err;
        lb_destroy(c);
        return fail(nullptr, LB_EDEVICE, "batch set-up failed: " + e);
    }
    c->chunk = std::max<uint32_t>(1u, (c->ntiles + 2047u) / 2048u);
    c->nblocks = (int)((c->ntiles + c->chunk - 1) / c->chunk);
    *out = c;
    return LB_OK;
}

int lb_destroy(lb_ctx *c)
{
    LB_RANGE();
    if (!c) return LB_OK;
    use_device(c);
    (void)hipStreamSynchronize(c->stream);
    void *ptrs[] = {c->own[0] ? c->own[0] : c->bufA,
                    c->own[1] ? c->own[1] : c->bufB,
                    c->partials,  c->scratch,   c->dev_out,   c->flags,
                    c->force,      c->fmask,     c->half,      c->fc,
                    c->boxes_d,    c->tile_box,  c->dstep,     c->amp,       c->ring,      c->corr,
                    c->cell_head,  c->cell_next,  c->cell_of,   c->fb2,       c->fp};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    for (int k = 0; k < 2; ++k)
        if (c->graph_exec[k]) (void)hipGraphExecDestroy(c->graph_exec[k]);
    free_tape(c);
    void *adj[] = {c->seg,       c->lamA, c->lamB,   c->gbar_d, c->adj_partials, c->tape_bead,
                   c->bead_work, c->fbar, c->force2, c->fmask2};
    for (void *q : adj)
        if (q) (void)hipFree(q);
    void *fused[] = {c->bead_pp, c->fmask_f, c->arrive, c->partner, c->moments, c->flist};
    for (void *q : fused)
        if (q) (void)hipFree(q);
    if (c->batch) {
        if (c->ev_in) (void)hipEventDestroy(c->ev_in);
        if (c->ev_out) (void)hipEventDestroy(c->ev_out);
        if (c->stream) (void)hipStreamDestroy(c->stream);
    }
    delete c;
    return LB_OK;
}

int lb_init_equilibrium(lb_ctx *c, const double *rho, const double *u)
{
    LB_RANGE();
    if (!c) return LB_EINVAL;
    LB_TRY(use_device(c));
    Join j(c);
    if (c->batch) {
        uint64_t site0 = 0;
        for (const BoxDesc &d : c->boxes_h) {
            by_storage(c->p.storage, [&](auto st) {
                hipLaunchKernelGGL((k_init_equilibrium<decltype(st)::value>), dim3(grid_for(d.geo.N, 256)), dim3(256), 0,
                                   c->stream, static_cast<char *>(c->bufA) + d.off * c->elem, d.geo, c->p.rho0,
                                   rho ? rho + site0 : nullptr, u ? u + 3 * site0 : nullptr);
            });
            site0 += d.geo.N;
        }
        LB_LAUNCH_CHECK(c, "init_equilibrium");
        return LB_OK;
    }
    LB_TRY(end_tape(c));
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
    LB_RANGE();
    if (!c) return LB_EINVAL;
    if (!src) return fail(c, LB_EINVAL, "src is NULL");
    if (dtype != LB_F64 && dtype != LB_F32) return fail(c, LB_EINVAL, "dtype must be LB_F64 or LB_F32");
    LB_TRY(use_device(c));
    Join j(c);
    const size_t isz = dtype == LB_F64 ? 8 : 4;
    auto one = [&](void *buf, const Geom &g, const void *sp) {
        by_storage(c->p.storage, [&](auto st) {
            constexpr int ST = decltype(st)::value;
            if (dtype == LB_F64)
                hipLaunchKernelGGL((k_set_pops<ST, double>), dim3(grid_for(g.N, 256)), dim3(256), 0, c->stream, buf, g,
                                   c->p.rho0, static_cast<const double *>(sp), shifted);
            else
                hipLaunchKernelGGL((k_set_pops<ST, float>), dim3(grid_for(g.N, 256)), dim3(256), 0, c->stream, buf, g,
                                   c->p.rho0, static_cast<const float *>(sp), shifted);
        });
    };
    if (c->batch) {
        uint64_t site0 = 0;  // the caller's array holds [19][N_b] per box, box after box
        for (const BoxDesc &d : c->boxes_h) {
            one(static_cast<char *>(c->bufA) + d.off * c->elem, d.geo, static_cast<const char *>(src) + 19 * site0 * isz);
            site0 += d.geo.N;
        }
    } else {
        LB_TRY(end_tape(c));
        one(c->bufA, c->geo, src);
    }
    LB_LAUNCH_CHECK(c, "set_populations");
    c->totals_valid = false;
    return LB_OK;
}

int lb_get_populations(lb_ctx *c, void *dst, int32_t dtype, int32_t shifted)
{
    LB_RANGE();
    if (!c) return LB_EINVAL;
    if (!dst) return fail(c, LB_EINVAL, "dst is NULL");
    if (dtype != LB_F64 && dtype != LB_F32) return fail(c, LB_EINVAL, "dtype must be LB_F64 or LB_F32");
    LB_TRY(use_device(c));
    Join j(c);
    const size_t isz = dtype == LB_F64 ? 8 : 4;
    auto one = [&](const void *buf, const Geom &g, void *dp) {
        by_storage(c->p.storage, [&](auto st) {
            constexpr int ST = decltype(st)::value;
            if (dtype == LB_F64)
                hipLaunchKernelGGL((k_get_pops<ST, double>), dim3(grid_for(g.N, 256)), dim3(256), 0, c->stream, buf, g,
                                   c->p.rho0, static_cast<double *>(dp), shifted);
            else
                hipLaunchKernelGGL((k_get_pops<ST, float>), dim3(grid_for(g.N, 256)), dim3(256), 0, c->stream, buf, g,
                                   c->p.rho0, static_cast<float *>(dp), shifted);
        });
    };
    if (c->batch) {
        uint64_t site0 = 0;  // the caller's array holds [19][N_b] per box, box after box
        for (const BoxDesc &d : c->boxes_h) {
            one(static_cast<const char *>(c->bufA) + d.off * c->elem, d.geo, static_cast<char *>(dst) + 19 * site0 * isz);
            site0 += d.geo.N;
        }
    } else {
        one(c->bufA, c->geo, dst);
    }
    LB_LAUNCH_CHECK(c, "get_populations");
    return LB_OK;
}

int lb_step(lb_ctx *c, int32_t nsteps)
{
    LB_RANGE();
    if (!c) return LB_EINVAL;
    if (nsteps < 0) return fail(c, LB_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return LB_OK;
    if (c->step + (uint64_t)nsteps > 0xffffffffull) return fail(c, LB_EINVAL, "step counter would exceed 2^32");
    LB_TRY(use_device(c));
    if (c->batch) {
        Join j(c);
        return batch_step(c, nsteps);
    }
    const bool tot = c->p.track_totals != 0;
    LB_TRY(reserve_checkpoints(c, nsteps));
    for (int32_t t = 0; t < nsteps; ++t) {
        const bool frc = c->pending_force;
        LB_TRY(select_launch(c, frc));
        if (c->taping) c->tape_slot.push_back(frc ? c->pending_slot : -1);
        void *dst = nullptr;
        bool ckpt = false;
        LB_TRY(step_dst(c, &dst, &ckpt));
        StepArgs a = plain_step_args(c, c->bufA, dst, (uint32_t)c->step);
        if (frc) {
            // the step reads the bead force and leaves the field and its bitmap zero
            a.fmask = c->fmask;
            a.force = c->force;
            a.consume = 1u;
        }
        // a step of a moments tape also writes its input state's moments
        // (no fused totals then: lb_totals forms them from the state)
        const bool mom = c->taping && c->tape_mom;
        if (mom) {
            a.xcd_remap = 0u;
            a.moments = mom_slot(c, c->step - c->tape_step0);
            launch_recompute(c, a, c->block, (uint32_t)c->nblocks, frc, true, nullptr, 0, nullptr, nullptr);
        } else {
            by_step_storage(c->p, [&](auto st) { launch_step_st<decltype(st)::value>(c, a, tot, frc); });
        }
        LB_LAUNCH_CHECK(c, "stream_collide");
        if (frc) {
            c->pending_force = false;
            c->pending_slot = -1;
        }
        LB_TRY(step_done(c, dst, tot && !mom, ckpt));
    }
    return LB_OK;
}

int lb_step_noalloc(const lb_params *params, const void *src, void *dst, uint64_t step, double *totals, void *stream)
{
    LB_RANGE();
    std::string msg;
    const int v = validate(params, msg);
    if (v != LB_OK) return fail(nullptr, v, msg);
    if (params->block == -1) return fail(nullptr, LB_EINVAL, "lb_step_noalloc needs block 0 or 64..1024 (no launch search)");
    if (!src || !dst) return fail(nullptr, LB_EINVAL, "src and dst must be non-NULL");
    if (step > 0xffffffffull) return fail(nullptr, LB_EINVAL, "step must be < 2^32");
    lb_ctx c;  // host bookkeeping only: no device memory is attached to it
    c.p = *params;
    c.stream = static_cast<hipStream_t>(stream);
    init_single_box(&c, params);
    const uintptr_t bytes = (uintptr_t)state_bytes(&c);
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(src), b0 = reinterpret_cast<uintptr_t>(dst);
    if (a0 < b0 + bytes && b0 < a0 + bytes) return fail(nullptr, LB_EINVAL, "src and dst overlap");
    c.block = params->block > 0 ? params->block : 256;
    c.nblocks = (int)step_blocks(&c, c.block);
    if ((size_t)c.nblocks > kNoallocRows)
        return fail(nullptr, LB_EINVAL,
                    "the step needs " + std::to_string(c.nblocks) + " blocks; the static scratch holds totals for " +
                        std::to_string(kNoallocRows) + " (use a larger block)");
    double *scr = nullptr;
    LB_TRY(noalloc_scratch(&scr));
    c.partials = scr;
    c.flags = reinterpret_cast<int32_t *>(scr + 4 * kNoallocRows);
    fill_collide_const(&c);
    const StepArgs a = plain_step_args(&c, src, dst, (uint32_t)step);
    const bool tot = totals != nullptr;
    by_step_storage(c.p, [&](auto st) { launch_step_st<decltype(st)::value>(&c, a, tot, false); });
    if (hipGetLastError() != hipSuccess) return fail(nullptr, LB_EDEVICE, "lb_step_noalloc: step launch failed");
    if (tot) {
        // same reduction order as lb_totals: column sums of the partial rows,
        // mass + N rho0 in FP64
        hipLaunchKernelGGL(k_reduce_cols, dim3(4), dim3(256), 0, c.stream, scr, c.nblocks, 4, totals,
                           (double)c.geo.N * params->rho0);
        if (hipGetLastError() != hipSuccess) return fail(nullptr, LB_EDEVICE, "lb_step_noalloc: totals launch failed");
    }
    return LB_OK;
}

int lb_couple(lb_ctx *c, const lb_beads *b)
{
    LB_RANGE();
    if (!c) return LB_EINVAL;
    LB_TRY(couple_check(c, b));
    if (b->n == 0) return LB_OK;
    const bool wca = b->wca_epsilon > 0.0;
    LB_TRY(use_device(c));
    LB_TRY(ensure_bead_buffers(c, b->n));
    if (wca) {
        const CellGrid cg = cell_grid(c, b);
        LB_TRY(ensure_pair_buffers(c, b->n, (size_t)cg.nc[0] * cg.nc[1] * cg.nc[2]));
    }
    c->pending_slot = -1;
    TapeSlot slot;
    if (c->taping) LB_TRY(tape_reserve(c, b, &slot));
    launch_couple(c, c->bufA, b, b->pos, b->mom, b->pos, b->mom, (uint32_t)c->step, c->taping ? &slot : nullptr);
    LB_LAUNCH_CHECK(c, "couple");
    c->pending_force = true;
    return LB_OK;
}

int lb_coupled_steps(lb_ctx *c, const lb_beads *b, int32_t nsteps)
{
    LB_RANGE();
    if (!c) return LB_EINVAL;
    if (nsteps < 0) return fail(c, LB_EINVAL, "nsteps must be >= 0");
    LB_TRY(couple_check(c, b));
    if (nsteps == 0) return LB_OK;
    if (c->step + (uint64_t)nsteps > 0xffffffffull) return fail(c, LB_EINVAL, "step counter would exceed 2^32");
    LB_TRY(use_device(c));
    // one launch per step without walls (WCA pairs, and the steps of a
    // moments tape, with phi_2 only); everything else (and a single step: its
    // bead state would be read and written by the same launch) takes the
    // separate launches
    const bool wca = b->wca_epsilon > 0.0;
    const bool mom_tape = c->taping && c->tape_mom;
    bool fused = nsteps >= 2 && b->n > 0 && !c->geo.walls && ((!wca && !mom_tape) || stencil_width(b) == 2);
    int deg = 0;
    if (fused) LB_TRY(build_partners(c, b, &deg, &fused));
    if (!fused) {
        for (int32_t k = 0; k < nsteps; ++k) {
            LB_TRY(lb_couple(c, b));
            LB_TRY(lb_step(c, 1));
        }
        return LB_OK;
    }
    const int n = b->n;
    const int LANES = stencil_lanes(stencil_width(b));
    const int PLANES = wca ? std::max(LANES, kPairLanes) : LANES;  // lanes per bead of the particle blocks
    LB_TRY(ensure_bead_buffers(c, n));
    LB_TRY(ensure_fused_buffers(c, n));
    CellGrid cg{};
    size_t ncell = 0;
    int32_t *lh[3] = {nullptr, nullptr, nullptr}, *ln[3] = {nullptr, nullptr, nullptr},
            *lc[3] = {nullptr, nullptr, nullptr};
    if (wca) {
        cg = cell_grid(c, b);
        ncell = (size_t)cg.nc[0] * cg.nc[1] * cg.nc[2];
        LB_TRY(ensure_fused_lists(c, n, ncell));
        // the context's own cell list too: the reverse sweep's pair Jacobians use it
        LB_TRY(ensure_pair_buffers(c, n, ncell));
        for (int r = 0; r < 3; ++r) {
            lh[r] = c->flist + (size_t)r * c->flist_cells;
            ln[r] = c->flist + 3 * c->flist_cells + (size_t)r * c->flist_n;
            lc[r] = c->flist + 3 * c->flist_cells + 3 * (size_t)c->flist_n + (size_t)r * c->flist_n;
        }
    }
    if (c->taping) {
        if (c->tape_nb == 0) c->tape_nb = n;
        if (n != c->tape_nb) return fail(c, LB_EUNSUPPORTED, "the bead count must stay the same over the taped steps");
        LB_TRY(tape_grow(c, b, (size_t)nsteps));
        LB_TRY(reserve_checkpoints(c, nsteps));
    }
    uint32_t *const bm[2] = {c->fmask, c->fmask_f};
    by_stencil(b->stencil, [&](auto w) {
        hipLaunchKernelGGL(k_bead_nodes<decltype(w)::value>, dim3(grid_for((size_t)LANES * n, 256)), dim3(256), 0,
                           c->stream, b->pos, b->mom, b->mass, n, c->geo, bm[0], cg, lh[0], ln[0], lc[0]);
    });
    LB_LAUNCH_CHECK(c, "bead nodes");
    const bool tot = c->p.track_totals != 0 && !mom_tape;  // a moments tape's steps: no fused totals
    const size_t n3 = 3 * (size_t)n;
    const double *pos_in = b->pos, *mom_in = b->mom;
    for (int32_t k = 0; k < nsteps; ++k) {
        // the last step writes the caller's arrays, the others alternate
        // between two private states
        double *pos = k + 1 == nsteps ? b->pos : c->bead_pp + (size_t)(k & 1) * 2 * n3;
        double *mom = k + 1 == nsteps ? b->mom : pos + n3;
        c->pending_slot = -1;
        TapeSlot slot;
        if (c->taping) LB_TRY(tape_reserve(c, b, &slot));
        LB_TRY(select_launch(c, true));
        if (c->taping) c->tape_slot.push_back(c->pending_slot);
        void *dst = nullptr;
        bool ckpt = false;
        LB_TRY(step_dst(c, &dst, &ckpt));
        StepArgs a = plain_step_args(c, c->bufA, dst, (uint32_t)c->step);
        a.fmask = bm[k & 1];
        a.force = c->force;
        if (mom_tape) a.moments = mom_slot(c, c->step - c->tape_step0);
        a.consume = 1u;
        const uint32_t pblocks = (uint32_t)((grid_for((size_t)PLANES * n, (unsigned)c->block) + 7) / 8 * 8);
        // the counter's value once this launch's particle blocks are counted
        // (taken over only once the launch is enqueued)
        const uint32_t target = c->arrive_count + pblocks;
        a.arrive = c->arrive;
        a.arrive_target = target;
        a.block0 = pblocks;
        ParticleArgs p;
        p.pop = c->bufA;
        p.geo = c->geo;
        p.rho0 = c->p.rho0;
        for (int q = 0; q < 3; ++q) p.g[q] = c->p.body_force[q];
        p.kT = c->p.kT;
        p.key0 = c->cc.key0;
        p.key1 = c->cc.key1;
        p.box = c->cc.box;
        p.step = (uint32_t)c->step;
        p.n = n;
        p.pos_in = pos_in;
        p.mom_in = mom_in;
        p.pos = pos;
        p.mom = mom;
        p.mass = b->mass;
        p.zeta = b->zeta;
        p.fext = b->fext;
        p.partner = c->partner;
        p.deg = deg;
        p.fene = (int32_t)(b->bond == LB_BOND_FENE);
        p.three_point = (int32_t)(b->noise == LB_NOISE_THREE_POINT);
        p.kb = b->k_bond;
        p.r0 = b->r0;
        p.flags = c->flags;
        p.force = c->force;
        p.fmask_next = k + 1 < nsteps ? bm[(k + 1) & 1] : nullptr;
        p.half = c->taping ? slot.half : c->half;
        p.fc = c->taping ? slot.fc : c->fc;
        p.tape_mom0 = c->taping ? slot.mom0 : nullptr;
        p.tape_momn = c->taping ? slot.momn : nullptr;
        p.tape_contrib = c->taping ? slot.contrib : nullptr;
        p.arrive = c->arrive;
        // the cell lists of steps k - 1, k, k + 1 (distinct: k mod 3 rotates)
        p.cg = cg;
        p.head = lh[k % 3];
        p.next = ln[k % 3];
        p.cell_of = lc[k % 3];
        p.head_reset = (wca && k >= 1) ? lh[(k + 2) % 3] : nullptr;
        p.cell_of_reset = lc[(k + 2) % 3];
        p.head_build = (wca && k + 1 < nsteps) ? lh[(k + 1) % 3] : nullptr;
        p.next_build = ln[(k + 1) % 3];
        p.cell_of_build = lc[(k + 1) % 3];
        const unsigned grid = pblocks + (unsigned)c->nblocks;
        by_step_storage(c->p, [&](auto st) {
            constexpr int ST = decltype(st)::value;
            if (wca)
                launch_fused_st<ST, 2, true>(c, a, p, grid, tot, mom_tape);
            else
                by_stencil(b->stencil,
                           [&](auto w) { launch_fused_st<ST, decltype(w)::value, false>(c, a, p, grid, tot, mom_tape); });
        });
        LB_LAUNCH_CHECK(c, "coupled step");
        c->arrive_count = target;
        c->pending_slot = -1;
        LB_TRY(step_done(c, dst, tot, ckpt));
        pos_in = pos;
        mom_in = mom;
    }
    if (wca) {
        // the last step's list back to -1 (the one before it the last launch reset)
        hipLaunchKernelGGL(k_cell_unlink, dim3(grid_for((size_t)n, 256)), dim3(256), 0, c->stream, lc[(nsteps - 1) % 3],
                           n, lh[(nsteps - 1) % 3]);
        LB_LAUNCH_CHECK(c, "cell list reset");
    }
    return LB_OK;
}

int lb_moments(lb_ctx *c, double *rho, double *u)
{
    LB_RANGE();
    if (!c) return LB_EINVAL;
    if (!rho && !u) return LB_OK;
    LB_TRY(use_device(c));
    Join j(c);
    auto one = [&](const void *buf, const Geom &g, double *r, double *uu) {
        by_storage(c->p.storage, [&](auto st) {
            hipLaunchKernelGGL((k_moments<decltype(st)::value>), dim3(grid_for(g.N, 256)), dim3(256), 0, c->stream, buf,
                               g, c->p.rho0, c->p.body_force[0], c->p.body_force[1], c->p.body_force[2], r, uu);
        });
    };
    if (c->batch) {
        uint64_t site0 = 0;
        for (const BoxDesc &d : c->boxes_h) {
            one(static_cast<const char *>(c->bufA) + d.off * c->elem, d.geo, rho ? rho + site0 : nullptr,
                u ? u + 3 * site0 : nullptr);
            site0 += d.geo.N;
        }
    } else {
        one(c->bufA, c->geo, rho, u);
    }
    LB_LAUNCH_CHECK(c, "moments");
    return LB_OK;
}

static int totals_from_partials(lb_ctx *c, const double *partials, int rows, double out[4])
{
    hipLaunchKernelGGL(k_reduce_cols, dim3(4), dim3(256), 0, c->stream, partials, rows, 4, c->dev_out, 0.0);
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

int lb_negative_count(lb_ctx *c, uint64_t *sites, double *min_pop)
{
    LB_RANGE();
    if (!c) return LB_EINVAL;
    if (!sites && !min_pop) return LB_OK;
    LB_TRY(use_device(c));
    Join j(c);
    const int nb = 1024;
    const int nbox = c->batch ? c->nbox : 1;
    LB_TRY(ensure_scratch(c, (size_t)nbox * nb * 2 * sizeof(double)));
    for (int k = 0; k < nbox; ++k) {
        const char *buf = static_cast<const char *>(c->bufA) + (c->batch ? c->boxes_h[k].off * c->elem : 0);
        const Geom &g = c->batch ? c->boxes_h[k].geo : c->geo;
        by_storage(c->p.storage, [&](auto st) {
            hipLaunchKernelGGL((k_negative_scan<decltype(st)::value>), dim3(nb), dim3(256), 0, c->stream, buf, g,
                               c->p.rho0, c->scratch + (size_t)k * nb * 2);
        });
    }
    LB_LAUNCH_CHECK(c, "negative scan");
    std::vector<double> h((size_t)nbox * nb * 2);
    LB_TRY(check(c, hipMemcpyAsync(h.data(), c->scratch, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream),
                 "negative scan copy"));
    LB_TRY(check(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize"));
    double cnt = 0.0, mn = std::numeric_limits<double>::infinity();
    for (size_t r = 0; r < h.size() / 2; ++r) {
        cnt += h[2 * r];
        mn = std::min(mn, h[2 * r + 1]);
    }
    if (sites) *sites = (uint64_t)cnt;
    if (min_pop) *min_pop = mn;
    return LB_OK;
}

int lb_totals_exact(lb_ctx *c, double out[4])
{
    LB_RANGE();
    if (!c || !out) return LB_EINVAL;
    LB_TRY(use_device(c));
    Join j(c);
    if (c->batch) {
        const int nbper = 64;
        LB_TRY(ensure_scratch(c, (size_t)c->nbox * nbper * 4 * sizeof(double)));
        for (int b = 0; b < c->nbox; ++b) {
            const BoxDesc &d = c->boxes_h[b];
            by_storage(c->p.storage, [&](auto st) {
                hipLaunchKernelGGL((k_totals_exact<decltype(st)::value>), dim3(nbper), dim3(256), 0, c->stream,
                                   static_cast<const char *>(c->bufA) + d.off * c->elem, d.geo,
                                   c->scratch + (size_t)b * nbper * 4);
            });
        }
        LB_LAUNCH_CHECK(c, "totals_exact");
        LB_TRY(totals_from_partials(c, c->scratch, c->nbox * nbper, out));
        out[0] += ((double)c->total_sites - (double)c->geo.N) * c->p.rho0;
        return LB_OK;
    }
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
    LB_RANGE();
    if (!c || !out) return LB_EINVAL;
    if (c->batch || !c->totals_valid) return lb_totals_exact(c, out);
    LB_TRY(use_device(c));
    return totals_from_partials(c, c->partials, c->nblocks, out);
}

int lb_mode_stats(lb_ctx *c, double var[19])
{
    LB_RANGE();
    if (!c || !var) return LB_EINVAL;
    LB_TRY(use_device(c));
    Join j(c);
    int rows = 1024;
    if (c->batch) {
        const int nbper = 32;
        rows = c->nbox * nbper;
        LB_TRY(ensure_scratch(c, (size_t)rows * 38 * sizeof(double)));
        for (int b = 0; b < c->nbox; ++b) {
            const BoxDesc &d = c->boxes_h[b];
            by_storage(c->p.storage, [&](auto st) {
                hipLaunchKernelGGL((k_mode_stats<decltype(st)::value>), dim3(nbper), dim3(256), 0, c->stream,
                                   static_cast<const char *>(c->bufA) + d.off * c->elem, d.geo, c->p.rho0,
                                   c->scratch + (size_t)b * nbper * 38);
            });
        }
    } else {
        LB_TRY(ensure_scratch(c, (size_t)rows * 38 * sizeof(double)));
        by_storage(c->p.storage, [&](auto st) {
            hipLaunchKernelGGL((k_mode_stats<decltype(st)::value>), dim3(rows), dim3(256), 0, c->stream, c->bufA,
                               c->geo, c->p.rho0, c->scratch);
        });
    }
    hipLaunchKernelGGL(k_reduce_cols, dim3(38), dim3(256), 0, c->stream, c->scratch, rows, 38, c->dev_out, 0.0);
    LB_LAUNCH_CHECK(c, "mode_stats");
    double h[38];
    LB_TRY(check(c, hipMemcpyAsync(h, c->dev_out, sizeof(h), hipMemcpyDeviceToHost, c->stream), "mode stats copy"));
    LB_TRY(read_flags(c));
    const double N = c->batch ? (double)c->total_sites : (double)c->geo.N;
    for (int k = 0; k < 19; ++k) {
        const double mean = h[k] / N;
        var[k] = h[19 + k] / N - mean * mean;
    }
    return LB_OK;
}

int lb_noise_sample(lb_ctx *c, uint32_t site0, uint32_t count, uint32_t step, float *out)
{
    LB_RANGE();
    if (!c) return LB_EINVAL;
    if (c->batch) return fail(c, LB_EUNSUPPORTED, "noise sampling is per single box");
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
    LB_RANGE();
    if (!c) return LB_EINVAL;
    LB_TRY(use_device(c));
    return read_flags(c);
}

int lb_tape_reserve(lb_ctx *c, int32_t nsteps, const lb_beads *b)
{
    LB_RANGE();
    if (!c) return LB_EINVAL;
    if (nsteps < 0) return fail(c, LB_EINVAL, "nsteps must be >= 0");
    if (!c->taping) return fail(c, LB_ESTATE, "no tape is recording");
    LB_TRY(use_device(c));
    LB_TRY(reserve_checkpoints(c, nsteps));
    if (b && b->n > 0) {
        LB_TRY(couple_check(c, b));
        if (c->tape_nb == 0) c->tape_nb = b->n;
        if (b->n != c->tape_nb)
            return fail(c, LB_EUNSUPPORTED, "the bead count must stay the same over the taped steps");
        LB_TRY(tape_grow(c, b, (size_t)nsteps));
        // the coupled steps' own device buffers (force field, bitmaps, bond
        // partner table, cell lists), which their first call would allocate
        LB_TRY(ensure_bead_buffers(c, b->n));
        LB_TRY(ensure_fused_buffers(c, b->n));
        if (b->wca_epsilon > 0.0) {
            const CellGrid cg = cell_grid(c, b);
            const size_t ncell = (size_t)cg.nc[0] * cg.nc[1] * cg.nc[2];
            LB_TRY(ensure_pair_buffers(c, b->n, ncell));
            LB_TRY(ensure_fused_lists(c, b->n, ncell));
        }
        int deg = 0;
        bool ok = true;
        LB_TRY(build_partners(c, b, &deg, &ok));
    }
    return LB_OK;
}

int lb_tape_begin(lb_ctx *c, int32_t checkpoint_every)
{
    LB_RANGE();
    if (!c) return LB_EINVAL;
    if (c->batch) return fail(c, LB_EUNSUPPORTED, "differentiation is per single box");
    if (checkpoint_every < 0) return fail(c, LB_EINVAL, "checkpoint_every must be >= 0");
    if (c->pending_force) return fail(c, LB_ESTATE, "lb_tape_begin between lb_couple and lb_step");
    LB_TRY(use_device(c));
    LB_TRY(settle_state(c));
    free_tape(c);
    if (checkpoint_every == 0) {
        // moments tape: slots are reserved by the steps (or lb_tape_reserve)
        c->tape_mom = true;
        c->tape_k = 0;
        c->tape_step0 = c->step;
        c->taping = true;
        return LB_OK;
    }
    // the forward writes each segment's step buffers straight into the
    // segment buffer, so the reverse sweep recomputes no step of the last
    // segment (none at all when checkpoint_every covers the whole run); if
    // the buffer does not fit, the sweep recomputes every segment
    // The buffer is taken up front only while it leaves at least half of the
    // device's free memory to the checkpoints, the backward buffers and the
    // caller (T is not known yet); otherwise the reverse sweep allocates it
    // and recomputes every segment.
    bool fits = (size_t)checkpoint_every <= SIZE_MAX / state_bytes(c);
    const size_t need = fits ? (size_t)checkpoint_every * state_bytes(c) : SIZE_MAX;
    if (fits && c->seg_bytes < need) {
        size_t free_b = 0, total_b = 0;
        fits = hipMemGetInfo(&free_b, &total_b) == hipSuccess && need <= (free_b + c->seg_bytes) / 2;
    }
    if (fits && c->seg_bytes < need) {
        (void)hipFree(c->seg);
        c->seg = nullptr;
        c->seg_bytes = 0;
        if (dev_alloc(&c->seg, need)) c->seg_bytes = need;  // one that did not fit is no error here
    }
    c->seg_fwd = c->seg_bytes >= need;
    c->tape_k = checkpoint_every;
    c->tape_step0 = c->step;
    c->taping = true;
    // a refused first checkpoint leaves no tape behind
    const int rc = push_checkpoint(c);
    if (rc != LB_OK) free_tape(c);
    return rc;
}

// Reverse sweep over the tape.  Per segment: restore its checkpoint and
// recompute its step buffers with the forward step kernel, except for the
// last segment, whose buffers the taped forward left in place (a coupled step's
// bead force is put back from the contributions its particle half recorded,
// k_respread; the bead kernels do not run again); then, from the last step
// of the segment back, the adjoint step: for a coupled step the force is put
// back once more, the fluid adjoint (FORCE variant) also writes the adjoint
// of the spread force at the flagged sites, and the particle adjoint
// (k_bead_adjoint, the bond and pair Jacobians, k_bead_adjoint_finish)
// carries the bead adjoints back from the taped R', F^c, P and P'' and adds
// the interpolation's share to lambda and gbar.
static int backward_impl(lb_ctx *c, const void *dL_dn_T, int32_t dtype, const double *dR_T, const double *dP_T,
                         void *dL_dn_0, double dL_dg[3], double *dR_0, double *dP_0)
{
    if (!c) return LB_EINVAL;
    if (!c->taping) return fail(c, LB_ESTATE, "lb_backward needs lb_tape_begin before the steps");
    if (c->pending_force) return fail(c, LB_ESTATE, "lb_backward between lb_couple and lb_step");
    if (!dL_dn_T || !dL_dn_0) return fail(c, LB_EINVAL, "gradient arrays must be non-NULL");
    if (dtype != LB_F64 && dtype != LB_F32) return fail(c, LB_EINVAL, "dtype must be LB_F64 or LB_F32");
    LB_TRY(use_device(c));
    const size_t N = c->geo.N, n19 = 19 * N;
    if (c->step < c->tape_step0 || (!c->tape_mom && c->tape_k < 1))
        return fail(c, LB_ESTATE, "the tape does not match the step counter");
    const uint64_t T = c->step - c->tape_step0;
    // one slot per taped step; one checkpoint at the start and after every K
    // steps, or (moments tape) one moment slot per step, the whole run being
    // one segment whose states are never needed
    if (T != (uint64_t)c->tape_slot.size())
        return fail(c, LB_ESTATE, "the tape does not match the steps taken since lb_tape_begin");
    if (c->tape_mom) {
        if (T > (uint64_t)INT32_MAX || (uint64_t)c->mom_chunks.size() * c->mom_chunk_steps < T)
            return fail(c, LB_ESTATE, "the moments tape does not cover the steps taken since lb_tape_begin");
    } else if ((uint64_t)c->checkpoints.size() != 1 + T / (uint64_t)c->tape_k) {
        return fail(c, LB_ESTATE, "the tape does not match the steps taken since lb_tape_begin");
    }
    const int K = c->tape_mom ? (int)std::max<uint64_t>(T, 1) : c->tape_k;
    const size_t sb = state_bytes(c);
    const int nbd = c->tape_nb;
    const bool coupled = !c->tape_beads.empty();
    LB_TRY(settle_state(c));  // the sweep may overwrite the segment buffer
    // a segment holds at most min(K, T) step buffers (none on a moments tape)
    const uint64_t slots = c->tape_mom ? 0 : std::min<uint64_t>((uint64_t)K, T);
    if (slots > SIZE_MAX / sb) return fail(c, LB_ENOMEM, "segment buffer too large");
    if (c->seg_bytes < slots * sb) {
        (void)hipFree(c->seg);
        c->seg = nullptr;
        c->seg_bytes = 0;
        c->seg_fwd = false;
        if (!dev_alloc(&c->seg, slots * sb)) return fail(c, LB_ENOMEM, "segment buffer allocation failed");
        c->seg_bytes = slots * sb;
    }
    // the moments (rho - rho0, j) of the recomputed states, 16 B per site
    // and state (the adjoint step reads them instead of the 19 pulled
    // values): taken when a segment is recomputed at all and the buffer
    // leaves half of the free memory; otherwise the adjoint reads the states
    const size_t mom_stride = 4 * N;
    const bool recompute = !c->tape_mom && (T > (uint64_t)K || !c->seg_fwd);
    if (recompute && slots >= 2 && c->moments_slots < slots - 1) {
        (void)hipFree(c->moments);
        c->moments = nullptr;
        c->moments_slots = 0;
        const size_t need = (size_t)(slots - 1) * mom_stride * sizeof(float);
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && need <= free_b / 2) {
            // if it is refused, the states serve instead
            if (dev_alloc(&c->moments, need)) c->moments_slots = (size_t)(slots - 1);
        }
    }
    // the adjoint step's blocks, dealt out layer by layer (256 threads)
    const unsigned nb = step_blocks(c, 256);
    const uint32_t adj_tiles = (c->geo.nxny + 255u) / 256u;
    if (!c->lamA || !c->lamB || !c->gbar_d || !c->adj_partials) {
        auto release = [&]() {
            (void)hipFree(c->lamA);
            (void)hipFree(c->lamB);
            (void)hipFree(c->gbar_d);
            (void)hipFree(c->adj_partials);
            c->lamA = c->lamB = nullptr;
            c->gbar_d = c->adj_partials = nullptr;
        };
        release();
        if (!dev_alloc(&c->lamA, n19 * sizeof(float)) || !dev_alloc(&c->lamB, n19 * sizeof(float)) ||
            !dev_alloc(&c->gbar_d, 3 * sizeof(double)) ||
            !dev_alloc(&c->adj_partials, (size_t)nb * 3 * sizeof(double))) {
            release();
            return fail(c, LB_ENOMEM, "adjoint buffers allocation failed");
        }
    }
    double *half_bar = nullptr, *fc_bar = nullptr, *p_bar = nullptr;
    double *pos_bar = nullptr, *mom_bar = nullptr;
    if (coupled) {
        if (c->bead_work_n < nbd) {
            (void)hipFree(c->bead_work);
            c->bead_work = nullptr;
            c->bead_work_n = 0;
            if (!dev_alloc(&c->bead_work, 15 * (size_t)nbd * sizeof(double)))
                return fail(c, LB_ENOMEM, "bead adjoint buffers allocation failed");
            c->bead_work_n = nbd;
        }
        if (!c->fbar || !c->force2 || !c->fmask2) {
            const size_t nwords = (N + 31) / 32;
            auto release = [&]() {
                (void)hipFree(c->fbar);
                (void)hipFree(c->force2);
                (void)hipFree(c->fmask2);
                c->fbar = nullptr;
                c->force2 = nullptr;
                c->fmask2 = nullptr;
            };
            release();
            if (!dev_alloc(&c->fbar, 6 * N * sizeof(float)) ||
                !dev_alloc(&c->force2, 3 * N * sizeof(long long)) ||
                !dev_alloc(&c->fmask2, nwords * sizeof(uint32_t))) {
                release();
                return fail(c, LB_ENOMEM, "force adjoint allocation failed");
            }
            hipLaunchKernelGGL(k_zero_f32, dim3(1024), dim3(256), 0, c->stream, c->fbar, 6 * N);
            hipLaunchKernelGGL(k_zero_f32, dim3(1024), dim3(256), 0, c->stream, reinterpret_cast<float *>(c->force2),
                               6 * N);
            hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(nwords, 256)), dim3(256), 0, c->stream,
                               reinterpret_cast<int32_t *>(c->fmask2), (uint32_t)nwords);
        }
        const size_t n3 = 3 * (size_t)nbd;
        half_bar = c->bead_work;
        fc_bar = half_bar + n3;
        p_bar = fc_bar + n3;
        pos_bar = p_bar + n3;
        mom_bar = pos_bar + n3;
        if (dR_T)
            LB_TRY(check(c, hipMemcpyAsync(pos_bar, dR_T, n3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream),
                         "bead gradient copy"));
        else
            hipLaunchKernelGGL(k_zero_f32, dim3(grid_for(2 * n3, 256)), dim3(256), 0, c->stream,
                               reinterpret_cast<float *>(pos_bar), 2 * n3);
        if (dP_T)
            LB_TRY(check(c, hipMemcpyAsync(mom_bar, dP_T, n3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream),
                         "bead gradient copy"));
        else
            hipLaunchKernelGGL(k_zero_f32, dim3(grid_for(2 * n3, 256)), dim3(256), 0, c->stream,
                               reinterpret_cast<float *>(mom_bar), 2 * n3);
    }
    if (dtype == LB_F64)
        hipLaunchKernelGGL(k_to_lam<double>, dim3(1024), dim3(256), 0, c->stream, static_cast<const double *>(dL_dn_T),
                           c->lamA, c->geo);
    else
        hipLaunchKernelGGL(k_to_lam<float>, dim3(1024), dim3(256), 0, c->stream, static_cast<const float *>(dL_dn_T),
                           c->lamA, c->geo);
    hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, c->stream, reinterpret_cast<float *>(c->gbar_d), (size_t)6);
    // the adjoint steps add their block sums of dL/dg into adj_partials; one
    // reduction at the end of the sweep
    hipLaunchKernelGGL(k_zero_f32, dim3(grid_for(6 * (size_t)nb, 256)), dim3(256), 0, c->stream,
                       reinterpret_cast<float *>(c->adj_partials), 6 * (size_t)nb);
    LB_LAUNCH_CHECK(c, "backward set-up");

    // Put the spread force of taped step t (coupled) back into a (zero) field.
    auto respread = [&](uint64_t t, long long *force, uint32_t *fmask) {
        const TapeSlot ts = tape_slot_at(c, c->tape_slot[t]);
        hipLaunchKernelGGL(k_respread, dim3(grid_for((size_t)ts.entries, 256)), dim3(256), 0, c->stream, ts.contrib,
                           ts.entries, c->geo.N, force, fmask);
    };
    auto coupled_at = [&](uint64_t t) { return c->tape_slot[t] >= 0; };
    // The reverse sweep alternates two force fields and two fbar halves by
    // the parity of the tape index, so that the extra blocks of each adjoint
    // step can put the next step's force back and clear the fbar of the
    // coupled step before it while the step reads its own.  A coupled step's
    // particle adjoint is finished late: its bond Jacobians run in those extra
    // blocks, its pair Jacobians after that kernel, and R'bar -> (Rbar, Pbar)
    // inside the next coupled step's k_bead_adjoint (or k_bead_adjoint_finish
    // after the last one).
    long long *const fpar[2] = {c->force, c->force2};
    uint32_t *const mpar[2] = {c->fmask, c->fmask2};
    float *const fbpar[2] = {c->fbar, c->fbar ? c->fbar + 3 * N : nullptr};
    int64_t pending = -1;  // tape index of the coupled step whose particle adjoint is not finished
    bool pending_jac = false;  // ... and whose bond and pair Jacobians are still to come
    // a refused pair adjoint (no cell list: not expected, the buffers are
    // checked before the sweep) leaves its error for the end of the sweep
    int pair_rc = LB_OK;
    auto pair_jacobians = [&](int64_t t) {
        const lb_beads &bp = c->tape_beads[c->tape_slot[t]];
        if (bp.wca_epsilon > 0.0 && pair_rc == LB_OK)
            pair_rc = launch_wca_adjoint(c, &bp, tape_slot_at(c, c->tape_slot[t]).half, fc_bar, half_bar);
    };
    // the pair adjoint relinks the context's cell list at each taped R'
    for (const lb_beads &bp : c->tape_beads) {
        if (!(bp.wca_epsilon > 0.0)) continue;
        const CellGrid cg = cell_grid(c, &bp);
        if (!c->cell_head || !c->cell_of || !c->cell_next || c->pair_cap < bp.n ||
            c->cell_cap < (size_t)cg.nc[0] * cg.nc[1] * cg.nc[2])
            return fail(c, LB_EDEVICE, "the pair adjoint needs the context's cell list, which no coupled step allocated");
    }

    const unsigned saved_blocks = c->nblocks;
    const int saved_block = c->block;
    c->block = 256;
    c->nblocks = (int)step_blocks(c, 256);
    const int nseg = (int)((T + K - 1) / K);
    // the state at step k of segment sg: the segment's checkpoint itself for
    // k = 0 (read in place, never written), then the segment buffer's slots
    auto state_at = [&](int sg, int k) -> char * {
        return k == 0 ? static_cast<char *>(c->checkpoints[sg]) : static_cast<char *>(c->seg) + (size_t)k * sb;
    };
    int rc = LB_OK;
    for (int sg = nseg - 1; sg >= 0 && rc == LB_OK; --sg) {
        const uint64_t t0 = (uint64_t)sg * K;
        const int len = (int)std::min<uint64_t>((uint64_t)K, T - t0);
        char *seg = static_cast<char *>(c->seg);
        // the last segment's step buffers 1 .. len-1 are still those the
        // forward wrote, unless an earlier sweep recomputed over them
        const bool kept = c->tape_mom || (c->seg_fwd && sg == nseg - 1);
        if (!kept) c->seg_fwd = false;
        // recompute steps 0 .. len-2 of the segment; the force fields
        // alternate by step parity, and a coupled step's launch puts the
        // next recomputed coupled step's force back in its last blocks.  Each
        // recompute step also writes its input state's moments, which the
        // adjoint step of that state reads instead of the state itself.
        const bool mom = !kept && len >= 2 && c->moments && (size_t)(len - 1) <= c->moments_slots;
        if (!kept && len >= 2 && coupled_at(t0)) respread(t0, fpar[t0 & 1u], mpar[t0 & 1u]);
        for (int k = 0; !kept && k + 1 < len; ++k) {
            const uint64_t t = t0 + k;
            const uint32_t step = (uint32_t)(c->tape_step0 + t);
            StepArgs a = plain_step_args(c, state_at(sg, k), seg + (size_t)(k + 1) * sb, step);
            const bool next = k + 2 < len && coupled_at(t + 1);
            const bool frc = coupled_at(t);
            if (mom || frc) {
                if (frc) {
                    a.fmask = mpar[t & 1u];
                    a.force = fpar[t & 1u];
                    a.consume = 1u;
                    // the force variant reads the bitmap at every site
                    if (!a.fmask || !a.force) {
                        rc = fail(c, LB_EDEVICE, "backward recompute: a coupled step without its force field");
                        break;
                    }
                }
                a.xcd_remap = 0u;  // the side blocks follow the step's own grid
                a.moments = mom ? c->moments + (size_t)k * mom_stride : nullptr;
                const TapeSlot tn = next ? tape_slot_at(c, c->tape_slot[t + 1]) : TapeSlot{};
                launch_recompute(c, a, 256, (uint32_t)c->nblocks, frc, mom, next ? tn.contrib : nullptr,
                                 next ? tn.entries : 0, fpar[(t + 1) & 1u], mpar[(t + 1) & 1u]);
            } else {
                if (next) respread(t + 1, fpar[(t + 1) & 1u], mpar[(t + 1) & 1u]);
                by_step_storage(c->p, [&](auto st) { launch_step_st<decltype(st)::value>(c, a, false, false); });
            }
        }
        if (rc != LB_OK) break;
        if ((rc = hipGetLastError() == hipSuccess ? LB_OK : fail(c, LB_EDEVICE, "backward recompute")) != LB_OK) break;
        // adjoint steps len-1 .. 0
        if (coupled_at(t0 + len - 1)) respread(t0 + len - 1, fpar[(t0 + len - 1) & 1u], mpar[(t0 + len - 1) & 1u]);
        for (int k = len - 1; k >= 0; --k) {
            const uint64_t t = t0 + k;
            const int q = (int)(t & 1u);
            const uint32_t step = (uint32_t)(c->tape_step0 + t);
            const int slot = c->tape_slot[t];
            // the step's input state, or on a moments tape its moments only
            const void *pop = c->tape_mom ? nullptr : state_at(sg, k);
            float *const tmom = c->tape_mom ? mom_slot(c, t) : nullptr;
            AdjArgs aa;
            aa.moments = c->tape_mom ? tmom : (mom && k + 1 < len) ? c->moments + (size_t)k * mom_stride : nullptr;
            aa.state = pop;
            aa.lam_in = c->lamA;
            aa.lam_out = c->lamB;
            aa.geo = c->geo;
            aa.cc = c->cc;
            aa.step = step;
            aa.partials = c->adj_partials;
            aa.force = fpar[q];
            aa.fmask = mpar[q];
            aa.fbar = fbpar[q];
            aa.tiles = adj_tiles;
            aa.div_tiles = make_fastdiv(adj_tiles);
            aa.main_blocks = nb;
            AdjSide &sd = aa.side;
            sd = AdjSide{};
            if (k >= 1 && coupled_at(t - 1)) {
                const TapeSlot tn = tape_slot_at(c, c->tape_slot[t - 1]);
                sd.put_contrib = tn.contrib;
                sd.put_entries = tn.entries;
                sd.put_force = fpar[(t - 1) & 1u];
                sd.put_fmask = mpar[(t - 1) & 1u];
            }
            if (pending >= 0 && pending_jac) {
                const lb_beads &bp = c->tape_beads[c->tape_slot[pending]];
                const TapeSlot tp = tape_slot_at(c, c->tape_slot[pending]);
                sd.half = tp.half;
                sd.fc_bar = fc_bar;
                sd.half_bar = half_bar;
                sd.bonds = bp.bonds;
                sd.nbonds = bp.nbonds;
                sd.nbeads = nbd;
                sd.fene = (int)(bp.bond == LB_BOND_FENE);
                sd.kb = bp.k_bond;
                sd.r0 = bp.r0;
                sd.clear_fbar = fbpar[pending & 1];
                sd.clear_contrib = tp.contrib;
                sd.clear_entries = tp.entries;
            }
            const int side_jobs = std::max({sd.put_entries, sd.nbonds, sd.clear_entries});
            const unsigned grid = nb + (side_jobs > 0 ? grid_for((size_t)side_jobs, 256) : 0u);
            by_storage(c->p.storage, [&](auto st) {
                constexpr int ST = decltype(st)::value;
                auto go = [&](auto th, auto frc) {
                    constexpr bool TH = decltype(th)::value, FRC = decltype(frc)::value;
                    if (c->geo.walls)
                        hipLaunchKernelGGL((k_adjoint_step<ST, TH, FRC, true>), dim3(grid), dim3(256), 0, c->stream,
                                           aa);
                    else
                        hipLaunchKernelGGL((k_adjoint_step<ST, TH, FRC, false>), dim3(grid), dim3(256), 0, c->stream,
                                           aa);
                };
                using T_ = std::true_type;
                using F_ = std::false_type;
                if (slot >= 0) {
                    if (c->thermal) go(T_{}, T_{});
                    else go(F_{}, T_{});
                } else {
                    if (c->thermal) go(T_{}, F_{});
                    else go(F_{}, F_{});
                }
            });
            if (pending >= 0 && pending_jac) {
                pair_jacobians(pending);
                pending_jac = false;
            }
            if (slot >= 0) {
                const lb_beads &bc = c->tape_beads[slot];
                const TapeSlot ts = tape_slot_at(c, slot);
                BeadAdjArgs ba;
                ba.pop = pop;
                ba.moments = tmom;
                ba.geo = c->geo;
                ba.rho0 = c->p.rho0;
                for (int r = 0; r < 3; ++r) ba.g[r] = c->p.body_force[r];
                ba.n = nbd;
                ba.mom0 = ts.mom0;
                ba.mom1 = ts.momn;
                ba.mass = bc.mass;
                ba.zeta = bc.zeta;
                ba.half = ts.half;
                ba.fc = ts.fc;
                ba.fbar = fbpar[q];
                ba.pos_bar = pos_bar;
                ba.mom_bar = mom_bar;
                ba.half_bar = half_bar;
                ba.fc_bar = fc_bar;
                ba.p_bar = p_bar;
                ba.lam = c->lamB;
                ba.gbar = c->gbar_d;
                ba.fold = pending >= 0 ? 1 : 0;
                ba.fold_mass = nullptr;
                ba.fold_cell_head = nullptr;
                ba.fold_cell_of = c->cell_of;
                if (pending >= 0) {
                    const lb_beads &bp = c->tape_beads[c->tape_slot[pending]];
                    ba.fold_mass = bp.mass;
                    ba.fold_cell_head = bp.wca_epsilon > 0.0 ? c->cell_head : nullptr;
                }
                by_storage(c->p.storage, [&](auto st) {
                    constexpr int ST = decltype(st)::value;
                    by_stencil(bc.stencil, [&](auto w) {
                        constexpr int W = decltype(w)::value;
                        hipLaunchKernelGGL((k_bead_adjoint<ST, W>),
                                           dim3(grid_for(StencilLanes<W>::value * (size_t)nbd, kBeadBlock)),
                                           dim3(kBeadBlock), 0,
                                           c->stream, ba);
                    });
                });
                pending = (int64_t)t;
                pending_jac = true;
            }
            std::swap(c->lamA, c->lamB);
        }
        if (hipGetLastError() != hipSuccess) rc = fail(c, LB_EDEVICE, "adjoint step");
    }
    if (rc == LB_OK && pending >= 0) {
        // the earliest coupled step: bond and pair Jacobians, then the finish
        const lb_beads &bp = c->tape_beads[c->tape_slot[pending]];
        const TapeSlot tp = tape_slot_at(c, c->tape_slot[pending]);
        if (pending_jac) {
            if (bp.nbonds > 0)
                hipLaunchKernelGGL(k_bonds_adjoint, dim3(grid_for((size_t)bp.nbonds, 256)), dim3(256), 0, c->stream,
                                   tp.half, fc_bar, half_bar, bp.bonds, bp.nbonds, bp.k_bond, bp.r0, nbd,
                                   (int)(bp.bond == LB_BOND_FENE));
            pair_jacobians(pending);
        }
        hipLaunchKernelGGL(k_bead_adjoint_finish, dim3(grid_for(std::max<size_t>((size_t)nbd, (size_t)tp.entries), 256)),
                           dim3(256), 0, c->stream, nbd, bp.mass, half_bar, p_bar, pos_bar, mom_bar,
                           fbpar[pending & 1], tp.contrib, tp.entries, c->geo.N,
                           bp.wca_epsilon > 0.0 ? c->cell_head : nullptr, c->cell_of);
        if (hipGetLastError() != hipSuccess) rc = fail(c, LB_EDEVICE, "bead adjoint");
    }
    c->block = saved_block;
    c->nblocks = (int)saved_blocks;
    if (rc == LB_OK && pair_rc != LB_OK) rc = pair_rc;
    if (rc != LB_OK) {
        // a sweep that stopped part way may leave WCA cell heads linked: put
        // them all back so that the next particle half starts from empty lists
        if (c->cell_head)
            hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(c->cell_cap, 256)), dim3(256), 0, c->stream,
                               reinterpret_cast<uint32_t *>(c->cell_head), (uint32_t)c->cell_cap, 0xffffffffu);
        return rc;
    }
    hipLaunchKernelGGL(k_accumulate_cols, dim3(3), dim3(256), 0, c->stream, c->adj_partials, (int)nb, 3, c->gbar_d);
    if (dtype == LB_F64)
        hipLaunchKernelGGL(k_from_lam<double>, dim3(1024), dim3(256), 0, c->stream, c->lamA,
                           static_cast<double *>(dL_dn_0), c->geo);
    else
        hipLaunchKernelGGL(k_from_lam<float>, dim3(1024), dim3(256), 0, c->stream, c->lamA,
                           static_cast<float *>(dL_dn_0), c->geo);
    LB_LAUNCH_CHECK(c, "backward output");
    if (coupled) {
        const size_t n3 = 3 * (size_t)nbd;
        if (dR_0)
            LB_TRY(check(c, hipMemcpyAsync(dR_0, pos_bar, n3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream),
                         "bead gradient copy"));
        if (dP_0)
            LB_TRY(check(c, hipMemcpyAsync(dP_0, mom_bar, n3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream),
                         "bead gradient copy"));
    }
    double h[3] = {0, 0, 0};
    LB_TRY(check(c, hipMemcpyAsync(h, c->gbar_d, sizeof(h), hipMemcpyDeviceToHost, c->stream), "gbar copy"));
    LB_TRY(read_flags(c));
    if (dL_dg)
        for (int k = 0; k < 3; ++k) dL_dg[k] = h[k];
    return LB_OK;
}

int lb_backward(lb_ctx *c, const void *dL_dn_T, int32_t dtype, void *dL_dn_0, double dL_dg[3])
{
    LB_RANGE();
    return backward_impl(c, dL_dn_T, dtype, nullptr, nullptr, dL_dn_0, dL_dg, nullptr, nullptr);
}

int lb_backward_coupled(lb_ctx *c, const void *dL_dn_T, int32_t dtype, const double *dL_dR_T, const double *dL_dP_T,
                        void *dL_dn_0, double dL_dg[3], double *dL_dR_0, double *dL_dP_0)
{
    LB_RANGE();
    return backward_impl(c, dL_dn_T, dtype, dL_dR_T, dL_dP_T, dL_dn_0, dL_dg, dL_dR_0, dL_dP_0);
}

int lb_vacf(lb_ctx *c, double *out, int64_t *nsamples)
{
    LB_RANGE();
    if (!c || !out) return LB_EINVAL;
    if (!c->batch || c->p.vacf_lags <= 0) return fail(c, LB_EINVAL, "context has no VACF (batch with vacf_lags > 0)");
    LB_TRY(use_device(c));
    const int R = c->p.vacf_lags;
    std::vector<double> h((size_t)c->nbox * R);
    uint32_t ns = 0;
    LB_TRY(check(c, hipMemcpyAsync(h.data(), c->corr, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream),
                 "vacf copy"));
    LB_TRY(check(c, hipMemcpyAsync(&ns, c->dstep + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream),
                 "vacf count copy"));
    LB_TRY(read_flags(c));
    const double kT = c->p.kT > 0.0 ? c->p.kT : 1.0;
    for (int b = 0; b < c->nbox; ++b) {
        const double norm = 6.0 * (double)c->boxes_h[b].geo.N * kT * c->p.rho0;
        for (int t = 0; t < R; ++t) {
            const double cnt = (double)ns - (double)t;
            out[(size_t)b * R + t] = cnt > 0 ? h[(size_t)b * R + t] / (cnt * norm) : 0.0;
        }
    }
    if (nsamples) *nsamples = ns;
    return LB_OK;
}

int lb_launch_config(lb_ctx *c, int32_t force, int32_t out[4])
{
    LB_RANGE();
    if (!c || !out) return LB_EINVAL;
    if (c->batch) {
        out[0] = c->block;
        out[1] = (int32_t)((c->ntiles + c->chunk - 1) / c->chunk);
        out[2] = (int32_t)c->chunk;
        out[3] = 0;
        return LB_OK;
    }
    const int k = force ? 1 : 0;
    out[0] = c->block_f[k];
    out[1] = (int32_t)grid_for(c->geo.N, c->block_f[k]);
    out[2] = 1;
    out[3] = (int32_t)c->remap_f[k];
    return LB_OK;
}

uint64_t lb_step_count(const lb_ctx *c) { return c ? c->step : 0; }

int lb_set_step_count(lb_ctx *c, uint64_t step)
{
    LB_RANGE();
    if (!c) return LB_EINVAL;
    if (step > 0xffffffffull) return fail(c, LB_EINVAL, "step counter must be < 2^32");
    if (c->pending_force) return fail(c, LB_ESTATE, "lb_set_step_count between lb_couple and lb_step");
    if (!c->batch) {
        LB_TRY(use_device(c));
        LB_TRY(end_tape(c));
    }
    c->step = step;
    if (c->batch) {
        LB_TRY(use_device(c));
        Join j(c);
        hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(64), 0, c->stream, c->dstep, (uint32_t)step);
        LB_LAUNCH_CHECK(c, "set step");
    }
    return LB_OK;
}

// Checkpoint file: this header, the box extents (int32 [nbox][3]), then the
// stored populations of every box (buffer A, box after box, [19][N_b] in the
// storage type), as they are in device memory.
struct SaveHeader {
    char magic[8];          // "LBMICKP1"
    uint32_t version;       // 1
    uint32_t header_bytes;  // sizeof(SaveHeader)
    lb_params params;
    int32_t nbox;           // 1 for a single box
    int32_t elem;           // bytes per stored population
    uint64_t step;
    uint64_t total_sites;
};
static const char kSaveMagic[8] = {'L', 'B', 'M', 'I', 'C', 'K', 'P', '1'};
// version 3: single-box populations in the z-major layout (pop_index), FP32
// storage with the rest residual plane
static const uint32_t kSaveVersion = 3;

static void ctx_dims(const lb_ctx *c, std::vector<int32_t> &dims)
{
    dims.clear();
    if (c->batch) {
        for (const BoxDesc &d : c->boxes_h) {
            dims.push_back((int32_t)d.geo.nx);
            dims.push_back((int32_t)d.geo.ny);
            dims.push_back((int32_t)d.geo.nz);
        }
    } else {
        dims = {(int32_t)c->geo.nx, (int32_t)c->geo.ny, (int32_t)c->geo.nz};
    }
}

static size_t ctx_sites(const lb_ctx *c) { return c->batch ? (size_t)c->total_sites : (size_t)c->geo.N; }

// Bytes of the stored populations of every box (the state lb_save writes).
static size_t ctx_state_bytes(const lb_ctx *c) { return (size_t)state_planes(c->p.storage) * ctx_sites(c) * c->elem; }

int lb_save(lb_ctx *c, const char *path)
{
    LB_RANGE();
    if (!c) return LB_EINVAL;
    if (!path) return fail(c, LB_EINVAL, "path is NULL");
    if (c->pending_force) return fail(c, LB_ESTATE, "lb_save between lb_couple and lb_step");
    LB_TRY(use_device(c));
    std::vector<int32_t> dims;
    ctx_dims(c, dims);
    SaveHeader h{};
    std::memcpy(h.magic, kSaveMagic, 8);
    h.version = kSaveVersion;
    h.header_bytes = (uint32_t)sizeof(SaveHeader);
    h.params = c->p;
    h.nbox = c->batch ? c->nbox : 1;
    h.elem = (int32_t)c->elem;
    h.step = c->step;
    h.total_sites = ctx_sites(c);
    const size_t bytes = ctx_state_bytes(c);
    std::vector<char> host(bytes);
    {
        Join j(c);
        LB_TRY(check(c, hipMemcpyAsync(host.data(), c->bufA, bytes, hipMemcpyDeviceToHost, c->stream), "state copy"));
        LB_TRY(check(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize"));
    }
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(c, LB_EIO, std::string("cannot open for writing: ") + path);
    bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1 &&
              std::fwrite(dims.data(), sizeof(int32_t), dims.size(), f) == dims.size() &&
              std::fwrite(host.data(), 1, bytes, f) == bytes;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return fail(c, LB_EIO, std::string("write failed: ") + path);
    return LB_OK;
}

int lb_load(lb_ctx *c, const char *path)
{
    LB_RANGE();
    if (!c) return LB_EINVAL;
    if (!path) return fail(c, LB_EINVAL, "path is NULL");
    if (c->pending_force) return fail(c, LB_ESTATE, "lb_load between lb_couple and lb_step");
    LB_TRY(use_device(c));
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(c, LB_EIO, std::string("cannot open for reading: ") + path);
    SaveHeader h{};
    std::vector<int32_t> dims, want;
    ctx_dims(c, want);
    const size_t bytes = ctx_state_bytes(c);
    std::vector<char> host;
    std::string why;
    if (std::fread(&h, sizeof(h), 1, f) != 1 || std::memcmp(h.magic, kSaveMagic, 8) != 0 || h.version != kSaveVersion ||
        h.header_bytes != sizeof(SaveHeader)) {
        why = "not a checkpoint of this library";
    } else if (h.nbox != (c->batch ? c->nbox : 1) || h.params.storage != c->p.storage || h.elem != (int32_t)c->elem ||
               h.total_sites != ctx_sites(c)) {
        why = "checkpoint layout (boxes, storage, sites) differs from the context";
    } else {
        dims.resize(want.size());
        host.resize(bytes);
        if (std::fread(dims.data(), sizeof(int32_t), dims.size(), f) != dims.size() || dims != want)
            why = "checkpoint box extents differ from the context";
        else if (std::fread(host.data(), 1, bytes, f) != bytes)
            why = "checkpoint file is truncated";
    }
    std::fclose(f);
    if (!why.empty()) return fail(c, LB_EIO, why + ": " + path);
    if (h.step > 0xffffffffull) return fail(c, LB_EIO, "checkpoint step counter out of range");
    if (!c->batch) LB_TRY(end_tape(c));
    {
        Join j(c);
        LB_TRY(check(c, hipMemcpyAsync(c->bufA, host.data(), bytes, hipMemcpyHostToDevice, c->stream), "state copy"));
        LB_TRY(check(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize"));
    }
    c->totals_valid = false;
    return lb_set_step_count(c, h.step);
}

const char *lb_last_error(const lb_ctx *c) { return c ? c->err.c_str() : g_create_error.c_str(); }

}  // extern "C"
