// m2c_api.hip -- host runtime behind the C ABI of include/m2c.h.
//
// One context owns one grid's device buffers and stream.  A time step is
// enqueued as a fixed kernel sequence with no host round trip:
//   count (+ previous step's phase update) -> scan (+ close the previous
//   step, open this one: dt) -> scatter -> [FIVER, stage] x 2
// with the last step's phase update and closing after the loop.  Every
// kernel returns at once when an earlier one has reported an error, so the
// last good state is the start-of-step buffer of the failing step (the two
// full states alternate between W[0] and W[1]).  The host reads the device
// scalars once per m2c_step call.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/m2c.h"
#include "m2c_internal.h"
#include "m2c_kernels.h"
#include "m2c_mlp.h"
#include "m2c_reinit.h"

using namespace m2c;

const MlpDev* m2c_mlp_dev(const m2c_mlp* m);   // m2c_learned.hip

static_assert(M2C_LIM_MC == LIM_MC && M2C_LIM_VAN_ALBADA == LIM_VA && M2C_LIM_VAN_ALBADA_MOD == LIM_VA_MOD &&
                  M2C_FLUX_HLLC == FLUX_HLLC && M2C_FLUX_LLF == FLUX_LLF,
              "option values shared by the ABI and the kernels");

constexpr int EV_STRIDE = 8;        // events per timed step (up to three RK stages)

struct m2c_ctx {
    m2c_config cfg;
    Grid g;
    int device = 0;
    hipStream_t stream = nullptr;
    double* W[2] = {nullptr, nullptr};
    double* W1 = nullptr;           // stage-1 state; also scratch for host transfers
    uint8_t* chi[2] = {nullptr, nullptr};
    int32_t* queue = nullptr;
    int32_t* fslot = nullptr;
    double* fluxF = nullptr;
    double* star = nullptr;
    int32_t* flips = nullptr;
    int32_t* blockcnt = nullptr;
    DevScalars* sc = nullptr;       // device
    DevScalars* hsc = nullptr;      // pinned host mirror
    long long qcap = 0;
    int nblk_compact = 0;
    int cur = 0;                    // index of the current state
    bool has_state = false;
    bool lam_valid = false;
    int tx = 32, ty = 8, kz = 8;
    int tiles[3] = {1, 1, 1};
    bool profiling = false;
    int prof_every = 1;             // profiling: time one step in prof_every
    long long prof_seq = 0;         // steps enqueued since profiling was switched on
    MlpDev mlp{};                   // context copy of the learned guess (null: acoustic)
    bool use_mlp = false;
    std::vector<hipEvent_t> evpool;  // profiling: EV_STRIDE events per timed step
    int ev_steps = 0;               // steps recorded in the pool, not yet harvested
    double ms_stage = 0, ms_fiver = 0, ms_other = 0;
    long long stage_launches = 0, fiver_launches = 0;
    long long steps_base = 0;       // steps_done at the last stats reset
    char err[256] = {0};
};

namespace {

int set_err(m2c_ctx* c, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int set_err(m2c_ctx* c, int code, const char* fmt, ...)
{
    if (c) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(c->err, sizeof(c->err), fmt, ap);
        va_end(ap);
    }
    return code;
}

#define HIPCHK(ctx, expr)                                                                       \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return set_err((ctx), M2C_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

bool valid_config(const m2c_config* c, char* why, size_t n)
{
    if (!c) return snprintf(why, n, "null config"), false;
    if (c->struct_size != sizeof(m2c_config))
        return snprintf(why, n, "struct_size %u != %zu", c->struct_size, sizeof(m2c_config)), false;
    if (c->nx < 1 || c->ny < 1 || c->nz < 1) return snprintf(why, n, "grid extents must be >= 1"), false;
    const long long N = (long long)c->nx * c->ny * c->nz;
    if (N > (1ll << 29)) return snprintf(why, n, "grid larger than 2^29 cells"), false;
    for (int d = 0; d < 3; ++d) {
        if (!(c->hi[d] > c->lo[d])) return snprintf(why, n, "empty box along axis %d", d), false;
        const bool plo = c->bc[2 * d] == M2C_BC_PERIODIC, phi = c->bc[2 * d + 1] == M2C_BC_PERIODIC;
        if (plo != phi) return snprintf(why, n, "periodic boundaries must pair up (axis %d)", d), false;
        for (int s = 0; s < 2; ++s)
            if (c->bc[2 * d + s] < 0 || c->bc[2 * d + s] > 2) return snprintf(why, n, "bad bc"), false;
    }
    if (c->eos_general != 0 && c->eos_general != 1) return snprintf(why, n, "eos_general must be 0 or 1"), false;
    if (c->eos_general) {
        eos::EosTable t;
        if (!eos::prepare(2, c->eos, t)) return snprintf(why, n, "invalid general EOS parameters"), false;
        if (c->precision != M2C_PREC_FP64) return snprintf(why, n, "general EOS runs in FP64 only"), false;
        if (!(c->riemann_ds == 0.0 || (c->riemann_ds >= 1e-3 && c->riemann_ds <= 0.5)))
            return snprintf(why, n, "riemann_ds must be 0 or in [1e-3, 0.5]"), false;
        if ((c->tile_x || c->tile_y) && !stage_tile_supported_eos(c->tile_x, c->tile_y))
            return snprintf(why, n, "general EOS: stage tile must be 16x15 or 64x2"), false;
    } else {
        for (int m = 0; m < 2; ++m)
            if (!(c->gamma[m] > 1.0) || !(c->pc[m] >= 0.0) || !std::isfinite(c->pc[m]))
                return snprintf(why, n, "material %d needs gamma > 1 and p_c >= 0", m), false;
    }
    if (!(c->limiter_alpha >= 0.0 && c->limiter_alpha <= 2.0))
        return snprintf(why, n, "limiter alpha must lie in [0, 2]"), false;
    if (c->limiter < M2C_LIM_MC || c->limiter > M2C_LIM_VAN_ALBADA_MOD) return snprintf(why, n, "bad limiter"), false;
    if (c->limiter != M2C_LIM_MC && (c->limiter_k < 2 || c->limiter_k > 8 || c->limiter_k % 2 != 0))
        return snprintf(why, n, "Van Albada exponent k must be even, 2..8"), false;
    if (c->flux != M2C_FLUX_HLLC && c->flux != M2C_FLUX_LLF) return snprintf(why, n, "bad flux"), false;
    if (!(c->ls_band >= 0.0) || !std::isfinite(c->ls_band)) return snprintf(why, n, "ls_band must be >= 0"), false;
    if (c->rk_order < 1 || c->rk_order > 3)
        return snprintf(why, n, "rk_order must be 1 (forward Euler), 2 or 3 (TVD-RK)"), false;
    if (!(c->dt_fixed > 0.0) && !(c->cfl > 0.0)) return snprintf(why, n, "cfl must be > 0"), false;
    if (c->precision != M2C_PREC_FP64 && c->precision != M2C_PREC_MIXED)
        return snprintf(why, n, "bad precision"), false;
    if (c->guess != M2C_GUESS_ACOUSTIC) return snprintf(why, n, "only the acoustic guess is built"), false;
    if (!(c->riemann_rtol > 0.0) || c->riemann_maxit < 1) return snprintf(why, n, "bad Riemann tolerance"), false;
    if ((c->tile_x || c->tile_y) && !stage_tile_supported(c->tile_x, c->tile_y))
        return snprintf(why, n, "unsupported stage tile %dx%d", c->tile_x, c->tile_y), false;
    if (c->tile_z < 0) return snprintf(why, n, "tile_z must be >= 0"), false;
    return true;
}

void fill_grid(Grid& g, const m2c_config& c)
{
    memset(&g, 0, sizeof(g));
    g.nx = c.nx;
    g.ny = c.ny;
    g.nz = c.nz;
    g.N = (long long)c.nx * c.ny * c.nz;
    const int nd[3] = {c.nx, c.ny, c.nz};
    for (int d = 0; d < 3; ++d) {
        g.act[d] = nd[d] > 1;
        g.h[d] = (c.hi[d] - c.lo[d]) / nd[d];
        g.rh[d] = 1.0 / g.h[d];
        g.rh6[d] = 1.0 / (6.0 * g.h[d]);
    }
    for (int f = 0; f < 6; ++f) g.bc[f] = c.bc[f];
    for (int m = 0; m < 2; ++m) {
        g.gamma[m] = c.gamma[m];
        g.pc[m] = c.pc[m];
        g.gpc[m] = c.gamma[m] * c.pc[m];
        g.inv_gm1[m] = 1.0 / (c.gamma[m] - 1.0);
    }
    g.alpha = c.limiter_alpha;
    g.cfl = c.cfl;
    g.dt_fixed = c.dt_fixed;
    g.rtol = c.riemann_rtol;
    g.maxit = c.riemann_maxit;
    g.guess = c.guess;
    g.rk_stages = c.rk_order;
    g.limiter = c.limiter;
    g.limk = c.limiter_k;
    g.flux = c.flux;
    g.ls_band = c.ls_band;
    g.eosg = c.eos_general;
    g.rds = c.riemann_ds > 0.0 ? c.riemann_ds : 0.01;
    if (c.eos_general) {
        eos::EosTable t;
        if (eos::prepare(2, c.eos, t)) {
            g.ek[0] = t.m[0];
            g.ek[1] = t.m[1];
        }
        // the stiffened-gas fields stay valid numbers (unused)
        for (int m = 0; m < 2; ++m) {
            g.gamma[m] = 1.4;
            g.pc[m] = g.gpc[m] = 0.0;
            g.inv_gm1[m] = 2.5;
        }
    }
}

// Reset the error state of the device scalars (host mirror -> device).
int clear_error(m2c_ctx* c)
{
    c->hsc->err = 0;
    c->hsc->err_cell = LLONG_MAX;
    HIPCHK(c, hipMemcpyAsync(&c->sc->err, &c->hsc->err, sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(&c->sc->err_cell, &c->hsc->err_cell, sizeof(long long), hipMemcpyHostToDevice,
                             c->stream));
    return M2C_OK;
}

// The next step rebuilds the interface queue (the state, and with it the
// material ids, was replaced outside the stepping).
int invalidate_queue(m2c_ctx* c)
{
    c->hsc->qvalid = 0;
    HIPCHK(c, hipMemcpyAsync(&c->sc->qvalid, &c->hsc->qvalid, sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    return M2C_OK;
}

int pull_scalars(m2c_ctx* c)
{
    HIPCHK(c, hipMemcpyAsync(c->hsc, c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return M2C_OK;
}

IfaceArgs iface_args(m2c_ctx* c, const double* Win)
{
    IfaceArgs a;
    a.g = c->g;
    a.Win = Win;
    a.chi = c->chi[c->cur];
    a.queue = c->queue;
    a.fslot = c->fslot;
    a.fluxF = c->fluxF;
    a.star = c->star;
    a.blockcnt = c->blockcnt;
    a.qcap = c->qcap;
    a.nblk = c->nblk_compact;
    a.sc = c->sc;
    return a;
}

const char* status_name(int s)
{
    switch (s) {
    case M2C_OK: return "ok";
    case M2C_ERR_ARG: return "invalid argument";
    case M2C_ERR_NONPHYSICAL: return "non-physical state (rho <= 0, p + p_c <= 0 or non-finite)";
    case M2C_ERR_RIEMANN: return "interface Riemann problem without admissible star pressure";
    case M2C_ERR_DEVICE: return "HIP runtime failure";
    case M2C_ERR_STATE: return "call out of order";
    case M2C_ERR_UNIMPLEMENTED: return "not implemented";
    case M2C_ERR_NOMEM: return "out of memory or work-queue capacity";
    default: return "unknown status";
    }
}

// Accumulate the kernel-class times of the steps recorded in the event pool
// (synchronises on the last recorded event).
int harvest_events(m2c_ctx* c)
{
    if (c->ev_steps == 0) return M2C_OK;
    // per timed step: e[0] before the compaction, e[1 + 2k] before the
    // FIVER launch of stage k, e[2 + 2k] before its stage kernel, e[1 + 2S]
    // after the last stage kernel
    const int S = c->cfg.rk_order;
    HIPCHK(c, hipEventSynchronize(c->evpool[(size_t)(c->ev_steps - 1) * EV_STRIDE + 1 + 2 * S]));
    for (int k = 0; k < c->ev_steps; ++k) {
        hipEvent_t* e = c->evpool.data() + (size_t)k * EV_STRIDE;
        float t;
        HIPCHK(c, hipEventElapsedTime(&t, e[0], e[1]));
        c->ms_other += t;
        for (int j = 0; j < S; ++j) {
            HIPCHK(c, hipEventElapsedTime(&t, e[1 + 2 * j], e[2 + 2 * j]));
            c->ms_fiver += t;
            HIPCHK(c, hipEventElapsedTime(&t, e[2 + 2 * j], e[3 + 2 * j]));
            c->ms_stage += t;
        }
        c->stage_launches += S;
        c->fiver_launches += S;
    }
    c->ev_steps = 0;
    return M2C_OK;
}

// Enqueue one full time step with state parity p (reads W[p], writes
// W[1-p]).  prev (nullable): the phase update of the previous step of this
// call, still pending; it runs in this step's count kernel, and this step's
// scan kernel closes that step.  The step's own phase update is returned in
// *phase, pending.
int enqueue_step(m2c_ctx* c, int p, double dt_imposed, const PhaseArgs* prev, PhaseArgs* phase)
{
    hipStream_t s = c->stream;
    const int q = 1 - p;
    const bool mixed = c->cfg.precision == M2C_PREC_MIXED;
    hipEvent_t* ev = nullptr;
    if (c->profiling && c->prof_seq++ % c->prof_every == 0) {
        if ((size_t)(c->ev_steps + 1) * EV_STRIDE > c->evpool.size()) {
            int rc = harvest_events(c);
            if (rc) return rc;
        }
        ev = c->evpool.data() + (size_t)c->ev_steps * EV_STRIDE;
    }
    if (ev) HIPCHK(c, hipEventRecord(ev[0], s));
    IfaceArgs ia = iface_args(c, c->W[p]);
    ia.chi = c->chi[p];
    HIPCHK(c, launch_compact(ia, prev, prev != nullptr, true, dt_imposed, s));

    StageArgs sa;
    sa.g = c->g;
    sa.chi = c->chi[p];
    sa.chi_next = c->chi[q];
    sa.flips = c->flips;
    sa.fslot = c->fslot;
    sa.fluxF = c->fluxF;
    sa.qcap = c->qcap;
    sa.sc = c->sc;
    sa.tiles_x = c->tiles[0];
    sa.tiles_y = c->tiles[1];
    sa.tiles_z = c->tiles[2];
    sa.kz = c->kz;

    // Runge-Kutta stages (section "Time integration"): stage s reads Win,
    // writes Wout = c0 W^n + c1 (Win + dt R(Win)); the FIVER fluxes of each
    // stage come from its own input state, and the last stage keeps the
    // star states for the phase update.  Buffers: W[p] = W^n, W[q] = W^{n+1},
    // W1 = the intermediate state (RK3 passes its first stage through W[q]).
    struct Stage {
        int kind;
        const double* win;
        double* wout;
        double c0, c1;
    };
    Stage st[3];
    const int S = c->cfg.rk_order;
    if (S == 1) {
        st[0] = {4, c->W[p], c->W[q], 0.0, 1.0};                 // forward Euler
    } else if (S == 2) {
        st[0] = {1, c->W[p], c->W1, 0.0, 1.0};                   // W(1) = W^n + dt R(W^n)
        st[1] = {2, c->W1, c->W[q], 0.5, 0.5};                   // 1/2 W^n + 1/2 (W(1) + dt R)
    } else {
        st[0] = {1, c->W[p], c->W[q], 0.0, 1.0};
        st[1] = {3, c->W[q], c->W1, 0.75, 0.25};                 // 3/4 W^n + 1/4 (W(1) + dt R)
        st[2] = {2, c->W1, c->W[q], 1.0 / 3.0, 2.0 / 3.0};       // 1/3 W^n + 2/3 (W(2) + dt R)
    }
    for (int k = 0; k < S; ++k) {
        if (ev) HIPCHK(c, hipEventRecord(ev[1 + 2 * k], s));
        ia.Win = st[k].win;
        HIPCHK(c, launch_fiver(ia, k == S - 1, c->use_mlp ? &c->mlp : nullptr, s));
        if (ev) HIPCHK(c, hipEventRecord(ev[2 + 2 * k], s));
        sa.Win = st[k].win;
        sa.W0 = c->W[p];
        sa.Wout = st[k].wout;
        sa.c0 = st[k].c0;
        sa.c1 = st[k].c1;
        HIPCHK(c, launch_stage(st[k].kind, mixed, c->tx, c->ty, sa, s));
    }
    if (ev) HIPCHK(c, hipEventRecord(ev[1 + 2 * S], s));

    PhaseArgs& pa = *phase;
    pa.g = c->g;
    pa.W = c->W[q];
    pa.chi_old = c->chi[p];
    pa.chi_new = c->chi[q];
    pa.flips = c->flips;
    pa.fslot = c->fslot;
    pa.star = c->star;
    pa.qcap = c->qcap;
    pa.sc = c->sc;
    if (ev) ++c->ev_steps;
    return M2C_OK;
}

int run_steps(m2c_ctx* c, int32_t nsteps, double dt_imposed, double* t_out)
{
    if (!c) return M2C_ERR_ARG;
    if (nsteps < 0) return set_err(c, M2C_ERR_ARG, "nsteps < 0");
    if (!c->has_state) return set_err(c, M2C_ERR_STATE, "m2c_step before a state was set");
    HIPCHK(c, hipSetDevice(c->device));
    int rc = clear_error(c);
    if (rc) return rc;
    if (!c->lam_valid && !(dt_imposed > 0.0) && !(c->cfg.dt_fixed > 0.0)) {
        HIPCHK(c, launch_lambda(c->g, c->W[c->cur], c->chi[c->cur], c->sc, c->stream));
    }
    rc = pull_scalars(c);
    if (rc) return rc;
    const long long done0 = c->hsc->steps_done;
    int p = c->cur;
    PhaseArgs pend[2];
    for (int32_t k = 0; k < nsteps; ++k) {
        rc = enqueue_step(c, p, dt_imposed, k > 0 ? &pend[(k - 1) & 1] : nullptr, &pend[k & 1]);
        if (rc) return rc;
        p = 1 - p;
    }
    if (nsteps > 0) {
        HIPCHK(c, launch_phase(pend[(nsteps - 1) & 1], c->stream));
        HIPCHK(c, launch_end_step(c->sc, c->g.rk_stages, c->stream));
    }
    rc = pull_scalars(c);
    if (rc) return rc;
    rc = harvest_events(c);
    if (rc) return rc;
    const long long done = c->hsc->steps_done - done0;
    c->cur = (int)((c->cur + done) & 1);
    if (t_out) *t_out = c->hsc->t;
    if (c->hsc->err != 0) {
        c->lam_valid = false;
        if ((rc = invalidate_queue(c))) return rc;
        const int e = c->hsc->err;
        const int code = e == ST_OVERFLOW ? M2C_ERR_NOMEM : e;
        return set_err(c, code, "step %lld failed: %s (cell %lld)", c->hsc->steps_done + 1, status_name(code),
                       c->hsc->err_cell);
    }
    c->lam_valid = true;
    return M2C_OK;
}

int upload_prim(m2c_ctx* c, const double* dprim)
{
    int rc = clear_error(c);
    if (rc) return rc;
    const int q = 1 - c->cur;
    HIPCHK(c, launch_prim_to_cons(c->g, dprim, c->W[q], c->chi[q], c->sc, c->stream));
    if ((rc = invalidate_queue(c))) return rc;
    rc = pull_scalars(c);
    if (rc) return rc;
    if (c->hsc->err != 0) {
        const long long cell = c->hsc->err_cell;
        clear_error(c);
        c->hsc->err_cell = cell;
        return set_err(c, M2C_ERR_NONPHYSICAL, "set_state: inadmissible primitive state at cell %lld", cell);
    }
    c->cur = q;
    c->has_state = true;
    c->lam_valid = false;
    return M2C_OK;
}

}  // namespace

void m2c_fill_grid(Grid* g, const m2c_config* c) { fill_grid(*g, *c); }

extern "C" {

int m2c_validate_config(const m2c_config* c)
{
    char why[160];
    return valid_config(c, why, sizeof(why)) ? M2C_OK : M2C_ERR_ARG;
}

void m2c_config_default(m2c_config* c)
{
    if (!c) return;
    memset(c, 0, sizeof(*c));
    c->struct_size = sizeof(m2c_config);
    c->nx = c->ny = c->nz = 1;
    for (int d = 0; d < 3; ++d) {
        c->lo[d] = 0.0;
        c->hi[d] = 1.0;
    }
    c->gamma[0] = 1.4;
    c->pc[0] = 0.0;
    c->gamma[1] = 6.12;
    c->pc[1] = 3.43e8;
    for (int f = 0; f < 6; ++f) c->bc[f] = M2C_BC_TRANSMISSIVE;
    c->limiter_alpha = 1.2;
    c->rk_order = 2;
    c->cfl = 0.5;
    c->dt_fixed = 0.0;
    c->precision = M2C_PREC_FP64;
    c->guess = M2C_GUESS_ACOUSTIC;
    c->riemann_rtol = 1e-12;
    c->riemann_maxit = 50;
    c->limiter = M2C_LIM_MC;
    c->limiter_k = 2;
    c->flux = M2C_FLUX_HLLC;
    c->ls_band = 0.0;
    c->eos_general = 0;
    c->riemann_ds = 0.0;
}

const char* m2c_strerror(int status) { return status_name(status); }

const char* m2c_last_error(const m2c_ctx* ctx) { return ctx ? ctx->err : "null context"; }

void m2c_destroy(m2c_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (int k = 0; k < 2; ++k) {
        (void)hipFree(c->W[k]);
        (void)hipFree(c->chi[k]);
    }
    (void)hipFree(c->W1);
    (void)hipFree(c->queue);
    (void)hipFree(c->fslot);
    (void)hipFree(c->fluxF);
    (void)hipFree(c->star);
    (void)hipFree(c->flips);
    (void)hipFree(c->blockcnt);
    (void)hipFree(c->sc);
    (void)hipFree(c->mlp.master);
    (void)hipFree(c->mlp.wbf);
    if (c->hsc) (void)hipHostFree(c->hsc);
    for (auto& e : c->evpool) (void)hipEventDestroy(e);
    delete c;
}

int m2c_create(const m2c_config* cfg, m2c_ctx** out)
{
    if (!out) return M2C_ERR_ARG;
    *out = nullptr;
    char why[160];
    if (!valid_config(cfg, why, sizeof(why))) return M2C_ERR_ARG;
    m2c_ctx* c = new (std::nothrow) m2c_ctx();
    if (!c) return M2C_ERR_NOMEM;
    c->cfg = *cfg;
    fill_grid(c->g, *cfg);
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return M2C_ERR_DEVICE;
    }
    const long long N = c->g.N;
    // interface queue capacity: every face for small grids, one face per
    // cell beyond that (far above any sheet-like interface)
    c->qcap = 3 * N;
    if (c->qcap > 65536 && c->qcap > N) c->qcap = N > 65536 ? N : 65536;
    c->nblk_compact = (int)((N + COMPACT_CELLS_PER_BLOCK - 1) / COMPACT_CELLS_PER_BLOCK);

    // stage tiles: (tile_x, tile_y), else 16x15 (its 511 in-plane faces are
    // exactly two rounds of the block's 256 threads), 64x2 for quasi-1D
    // grids.  Planes per block: tile_z,
    // else the most of 32, 16 that still leaves at least 4096 blocks (16
    // rounds of two blocks per CU: the prologue of a block's march and the
    // re-read halo planes are amortised over more planes; 32 measured 1.5%
    // faster than 16 on 384^3), otherwise 8.
    c->tx = cfg->tile_x ? cfg->tile_x : 16;
    c->ty = cfg->tile_y ? cfg->tile_y : 15;
    if (!cfg->tile_x && c->g.ny == 1) {
        c->tx = 64;
        c->ty = 2;
    }
    if (cfg->tile_z) {
        c->kz = cfg->tile_z;
    } else {
        const long long txy = (long long)((c->g.nx + c->tx - 1) / c->tx) * ((c->g.ny + c->ty - 1) / c->ty);
        c->kz = txy * ((c->g.nz + 31) / 32) >= 4096 ? 32 : (txy * ((c->g.nz + 15) / 16) >= 4096 ? 16 : 8);
    }
    if (c->kz > c->g.nz) c->kz = c->g.nz;
    c->tiles[0] = (c->g.nx + c->tx - 1) / c->tx;
    c->tiles[1] = (c->g.ny + c->ty - 1) / c->ty;
    c->tiles[2] = (c->g.nz + c->kz - 1) / c->kz;

    bool ok = true;
    auto alloc = [&](void** p, size_t bytes) {
        if (ok && hipMalloc(p, bytes) != hipSuccess) {
            ok = false;
            *p = nullptr;
        }
    };
    for (int k = 0; k < 2; ++k) {
        alloc((void**)&c->W[k], 6 * N * sizeof(double));
        alloc((void**)&c->chi[k], N);
    }
    alloc((void**)&c->W1, 6 * N * sizeof(double));
    alloc((void**)&c->queue, c->qcap * sizeof(int32_t));
    alloc((void**)&c->fslot, 3 * N * sizeof(int32_t));
    alloc((void**)&c->fluxF, 10 * c->qcap * sizeof(double));
    alloc((void**)&c->star, 8 * c->qcap * sizeof(double));
    alloc((void**)&c->flips, N * sizeof(int32_t));
    alloc((void**)&c->blockcnt, (size_t)c->nblk_compact * sizeof(int32_t));
    alloc((void**)&c->sc, sizeof(DevScalars));
    if (ok && hipHostMalloc((void**)&c->hsc, sizeof(DevScalars), hipHostMallocDefault) != hipSuccess) ok = false;
    if (!ok) {
        m2c_destroy(c);
        return M2C_ERR_NOMEM;
    }
    memset(c->hsc, 0, sizeof(DevScalars));
    c->hsc->err_cell = LLONG_MAX;
    if (hipMemcpy(c->sc, c->hsc, sizeof(DevScalars), hipMemcpyHostToDevice) != hipSuccess ||
        launch_fill_i32(c->fslot, 3 * N, -1, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        m2c_destroy(c);
        return M2C_ERR_DEVICE;
    }
    *out = c;
    return M2C_OK;
}

int m2c_set_stream(m2c_ctx* c, void* s)
{
    if (!c) return M2C_ERR_ARG;
    c->stream = (hipStream_t)s;
    return M2C_OK;
}

int m2c_set_state(m2c_ctx* c, const double* prim6)
{
    if (!c || !prim6) return M2C_ERR_ARG;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpyAsync(c->W1, prim6, 6 * c->g.N * sizeof(double), hipMemcpyHostToDevice, c->stream));
    return upload_prim(c, c->W1);
}

int m2c_set_state_device(m2c_ctx* c, const double* dprim6)
{
    if (!c || !dprim6) return M2C_ERR_ARG;
    HIPCHK(c, hipSetDevice(c->device));
    return upload_prim(c, dprim6);
}

int m2c_get_state(m2c_ctx* c, double* prim6, uint8_t* id)
{
    if (!c || !prim6) return M2C_ERR_ARG;
    if (!c->has_state) return set_err(c, M2C_ERR_STATE, "no state set");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_cons_to_prim(c->g, c->W[c->cur], c->chi[c->cur], c->W1, c->stream));
    HIPCHK(c, hipMemcpyAsync(prim6, c->W1, 6 * c->g.N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (id) HIPCHK(c, hipMemcpyAsync(id, c->chi[c->cur], c->g.N, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return M2C_OK;
}

int m2c_get_state_device(m2c_ctx* c, double* dprim6)
{
    if (!c || !dprim6) return M2C_ERR_ARG;
    if (!c->has_state) return set_err(c, M2C_ERR_STATE, "no state set");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_cons_to_prim(c->g, c->W[c->cur], c->chi[c->cur], dprim6, c->stream));
    return M2C_OK;
}

int m2c_get_conserved(m2c_ctx* c, double* w6)
{
    if (!c || !w6) return M2C_ERR_ARG;
    if (!c->has_state) return set_err(c, M2C_ERR_STATE, "no state set");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpyAsync(w6, c->W[c->cur], 6 * c->g.N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return M2C_OK;
}

int m2c_set_conserved(m2c_ctx* c, const double* w6)
{
    if (!c || !w6) return M2C_ERR_ARG;
    HIPCHK(c, hipSetDevice(c->device));
    const int q = 1 - c->cur;
    HIPCHK(c, hipMemcpyAsync(c->W[q], w6, 6 * c->g.N * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_chi_from_phi(c->g, c->W[q], c->chi[q], c->stream));
    const int rc = invalidate_queue(c);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->cur = q;
    c->has_state = true;
    c->lam_valid = false;
    return M2C_OK;
}

int m2c_step(m2c_ctx* c, int32_t nsteps, double* t_out) { return run_steps(c, nsteps, 0.0, t_out); }

int m2c_reinit(m2c_ctx* c, int32_t iters, double band)
{
    if (!c) return M2C_ERR_ARG;
    if (iters < 0 || !(band >= 0.0) || !std::isfinite(band))
        return set_err(c, M2C_ERR_ARG, "iters must be >= 0 and band >= 0");
    if (!c->has_state) return set_err(c, M2C_ERR_STATE, "no state set");
    if (iters == 0) return M2C_OK;
    HIPCHK(c, hipSetDevice(c->device));
    ReinitGrid g;
    if (!reinit_grid(c->g.nx, c->g.ny, c->g.nz, c->g.h, c->cfg.bc, g)) return set_err(c, M2C_ERR_ARG, "grid");
    // the stage buffer is free between steps: S, the second iterate, block flags
    const long long N = c->g.N;
    double* phi = c->W[c->cur] + 5 * N;
    HIPCHK(c, reinit_run(g, phi, c->W1, c->W1 + N, (int32_t*)(c->W1 + 2 * N), iters, band, c->stream));
    return invalidate_queue(c);
}

int m2c_step_dt(m2c_ctx* c, int32_t nsteps, double dt, double* t_out)
{
    if (!c) return M2C_ERR_ARG;
    if (!(dt > 0.0) || !std::isfinite(dt)) return set_err(c, M2C_ERR_ARG, "dt must be positive and finite");
    return run_steps(c, nsteps, dt, t_out);
}

int m2c_get_stats(m2c_ctx* c, m2c_stats* s)
{
    if (!c || !s) return M2C_ERR_ARG;
    HIPCHK(c, hipSetDevice(c->device));
    int rc = pull_scalars(c);
    if (rc) return rc;
    const DevScalars& d = *c->hsc;
    memset(s, 0, sizeof(*s));
    s->steps = d.steps_done - c->steps_base;
    s->t = d.t;
    s->dt_last = d.dt_last;
    s->iface_faces_last = d.qlen;
    s->riemann_solves = d.solves;
    s->newton_iters = d.newton_iters;
    s->bisection_fallbacks = d.fallbacks;
    s->flips = d.flips;
    s->orphans = d.orphans;
    s->mlp_fallbacks = d.mlp_fallbacks;
    s->err_code = d.err == ST_OVERFLOW ? M2C_ERR_NOMEM : d.err;
    s->err_cell = d.err ? d.err_cell : -1;
    s->ms_stage = c->ms_stage;
    s->ms_fiver = c->ms_fiver;
    s->ms_other = c->ms_other;
    s->stage_launches = c->stage_launches;
    s->fiver_launches = c->fiver_launches;
    return M2C_OK;
}

int m2c_reset_stats(m2c_ctx* c)
{
    if (!c) return M2C_ERR_ARG;
    HIPCHK(c, hipSetDevice(c->device));
    int rc = pull_scalars(c);
    if (rc) return rc;
    DevScalars& d = *c->hsc;
    d.solves = d.newton_iters = d.fallbacks = d.flips = d.orphans = d.mlp_fallbacks = 0;
    HIPCHK(c, hipMemcpyAsync(c->sc, c->hsc, sizeof(DevScalars), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->steps_base = d.steps_done;
    c->ms_stage = c->ms_fiver = c->ms_other = 0;
    c->stage_launches = c->fiver_launches = 0;
    return M2C_OK;
}

int m2c_set_profiling(m2c_ctx* c, int every)
{
    if (!c || every < 0) return M2C_ERR_ARG;
    HIPCHK(c, hipSetDevice(c->device));
    const int on = every;
    if (on && c->evpool.empty()) {
        c->evpool.resize(EV_STRIDE * 512, nullptr);
        for (auto& e : c->evpool) HIPCHK(c, hipEventCreate(&e));
    }
    if (!on) {
        int rc = harvest_events(c);
        if (rc) return rc;
    }
    c->profiling = on != 0;
    c->prof_every = on > 0 ? on : 1;
    c->prof_seq = 0;
    return M2C_OK;
}

int m2c_interface_faces(m2c_ctx* c, int32_t* out, int64_t cap, int64_t* count)
{
    if (!c || !count || cap < 0) return M2C_ERR_ARG;
    if (!c->has_state) return set_err(c, M2C_ERR_STATE, "no state set");
    HIPCHK(c, hipSetDevice(c->device));
    int rc = clear_error(c);
    if (rc) return rc;
    IfaceArgs ia = iface_args(c, c->W[c->cur]);
    HIPCHK(c, launch_compact(ia, nullptr, false, false, 0.0, c->stream));
    rc = pull_scalars(c);
    if (rc) return rc;
    if (c->hsc->err != 0) {
        clear_error(c);
        return set_err(c, M2C_ERR_NOMEM, "interface queue capacity %lld exceeded", c->qcap);
    }
    const long long n = c->hsc->qlen;
    *count = n;
    const long long m = n < cap ? n : cap;
    if (out && m > 0) {
        HIPCHK(c, hipMemcpyAsync(out, c->queue, m * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return M2C_OK;
}

int m2c_eval_hllc(int64_t n, const double* qL, const double* qR, double gamma, double pc, int32_t prec,
                  double* F, void* hip_stream)
{
    if (n < 0 || (n > 0 && (!qL || !qR || !F))) return M2C_ERR_ARG;
    if (!(gamma > 1.0) || !(pc >= 0.0)) return M2C_ERR_ARG;
    if (prec != M2C_PREC_FP64 && prec != M2C_PREC_MIXED) return M2C_ERR_ARG;
    if (n == 0) return M2C_OK;
    if (launch_hllc_points(n, qL, qR, gamma, pc, prec == M2C_PREC_MIXED, F, (hipStream_t)hip_stream) !=
        hipSuccess)
        return M2C_ERR_DEVICE;
    return M2C_OK;
}

int m2c_riemann_solve(int64_t n, const double* in, const double* eos, int32_t guess, double rtol, int32_t maxit,
                      double* out, int32_t* iters, void* hip_stream)
{
    if (n < 0 || (n > 0 && (!in || !eos || !out))) return M2C_ERR_ARG;
    if (!(rtol > 0.0) || maxit < 1) return M2C_ERR_ARG;
    if (guess != M2C_GUESS_ACOUSTIC) return M2C_ERR_UNIMPLEMENTED;
    if (n == 0) return M2C_OK;
    hipStream_t s = (hipStream_t)hip_stream;
    int32_t* dvac = nullptr;
    if (hipMalloc((void**)&dvac, sizeof(int32_t)) != hipSuccess) return M2C_ERR_NOMEM;
    int32_t hv = 0;
    int rc = M2C_OK;
    if (hipMemsetAsync(dvac, 0, sizeof(int32_t), s) != hipSuccess ||
        launch_riemann_points(n, in, eos, nullptr, rtol, maxit, out, iters, dvac, nullptr, s) != hipSuccess ||
        hipMemcpyAsync(&hv, dvac, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        rc = M2C_ERR_DEVICE;
    (void)hipFree(dvac);
    if (rc == M2C_OK && hv > 0) rc = M2C_ERR_RIEMANN;
    return rc;
}

int m2c_autotune(m2c_ctx* c, int32_t steps, int32_t tile_out[3], float* ms_out)
{
    static const int cands_sg[][3] = {{16, 15, 8}, {16, 15, 16}, {16, 16, 8}, {16, 16, 16}, {16, 16, 4},
                                      {32, 8, 8},  {32, 7, 8},   {16, 15, 4}, {16, 15, 32}};
    static const int cands_eos[][3] = {{16, 15, 8}, {16, 15, 4}};
    if (!c || steps < 1) return M2C_ERR_ARG;
    const int(*cands)[3] = c->g.eosg ? cands_eos : cands_sg;
    const int ncand = c->g.eosg ? 2 : 9;
    if (!c->has_state) return set_err(c, M2C_ERR_STATE, "no state set");
    HIPCHK(c, hipSetDevice(c->device));
    int rc = pull_scalars(c);
    if (rc) return rc;
    const DevScalars sc0 = *c->hsc;
    const int cur0 = c->cur;
    const bool lam0 = c->lam_valid;
    const long long N = c->g.N;
    double* snapW = nullptr;
    uint8_t* snapX = nullptr;
    HIPCHK(c, hipMalloc((void**)&snapW, 6 * N * sizeof(double)));
    if (hipMalloc((void**)&snapX, N) != hipSuccess) {
        (void)hipFree(snapW);
        return set_err(c, M2C_ERR_NOMEM, "autotune snapshot");
    }
    auto restore = [&]() -> int {
        c->cur = cur0;
        c->lam_valid = lam0;
        *c->hsc = sc0;
        c->hsc->qvalid = 0;                    // the trial steps may have changed the queue
        HIPCHK(c, hipMemcpyAsync(c->W[cur0], snapW, 6 * N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->chi[cur0], snapX, N, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->sc, c->hsc, sizeof(DevScalars), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return M2C_OK;
    };
    auto set_tile = [&](int tx, int ty, int kz) {
        c->tx = tx;
        c->ty = ty;
        c->kz = kz < c->g.nz ? kz : c->g.nz;
        c->tiles[0] = (c->g.nx + tx - 1) / tx;
        c->tiles[1] = (c->g.ny + ty - 1) / ty;
        c->tiles[2] = (c->g.nz + c->kz - 1) / c->kz;
    };
    if (hipMemcpyAsync(snapW, c->W[cur0], 6 * N * sizeof(double), hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(snapX, c->chi[cur0], N, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
        rc = set_err(c, M2C_ERR_DEVICE, "autotune snapshot copy");
    const bool prof = c->profiling;
    c->profiling = false;
    int bt[3] = {c->tx, c->ty, c->kz};
    float best = -1.0f;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = set_err(c, M2C_ERR_DEVICE, "event create");
    for (int ci = 0; ci < ncand; ++ci) {
        const int* cand = cands[ci];
        if (rc) break;
        set_tile(cand[0], cand[1], cand[2]);
        if ((rc = restore()) || (rc = run_steps(c, 1, 0.0, nullptr)) || (rc = restore())) break;
        if (hipEventRecord(e0, c->stream) != hipSuccess) { rc = M2C_ERR_DEVICE; break; }
        if ((rc = run_steps(c, steps, 0.0, nullptr))) break;
        if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            rc = M2C_ERR_DEVICE;
            break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (best < 0.0f || ms < best) {
            best = ms;
            bt[0] = cand[0];
            bt[1] = cand[1];
            bt[2] = cand[2];
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    set_tile(bt[0], bt[1], bt[2]);
    const int rc2 = restore();
    c->profiling = prof;
    (void)hipFree(snapW);
    (void)hipFree(snapX);
    if (rc) return rc;
    if (rc2) return rc2;
    if (tile_out) {
        tile_out[0] = bt[0];
        tile_out[1] = bt[1];
        tile_out[2] = bt[2];
    }
    if (ms_out) *ms_out = best / steps;
    return M2C_OK;
}

int m2c_set_guess(m2c_ctx* c, const m2c_mlp* m)
{
    if (!c) return M2C_ERR_ARG;
    HIPCHK(c, hipSetDevice(c->device));
    if (!m) {
        c->use_mlp = false;
        return M2C_OK;
    }
    const MlpDev* src = m2c_mlp_dev(m);
    if (!c->mlp.master) {
        HIPCHK(c, hipMalloc((void**)&c->mlp.master, MLP_NPARAM * sizeof(float)));
        HIPCHK(c, hipMalloc((void**)&c->mlp.wbf, MLP_NBF * sizeof(uint16_t)));
    }
    HIPCHK(c, hipMemcpyAsync(c->mlp.master, src->master, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToDevice,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(c->mlp.wbf, src->wbf, MLP_NBF * sizeof(uint16_t), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->use_mlp = true;
    return M2C_OK;
}

int m2c_get_tile(const m2c_ctx* c, int32_t tile[3])
{
    if (!c || !tile) return M2C_ERR_ARG;
    tile[0] = c->tx;
    tile[1] = c->ty;
    tile[2] = c->kz;
    return M2C_OK;
}

}  // extern "C"
