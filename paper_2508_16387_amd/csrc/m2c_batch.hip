// m2c_batch.hip -- batched form and tile autotuning behind include/m2c.h.
//
// A batch holds many independent runs (uneven grids, one precision and one
// stage-tile shape for all).  Every device buffer of every run is allocated
// once; one time step of all runs is one fixed kernel sequence
//   begin -> compaction -> [FIVER, persistent stage] x 2 -> phase -> end
// over device-side run descriptors, captured once into a hipGraph and
// replayed per step.  Each run keeps its own dt, error state and state
// parity in device memory, so runs of different sizes and CFL limits (and a
// run that has failed) share the same graph.  The autotuner times every
// supported tile shape on the batch itself and keeps the fastest.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/m2c.h"
#include "m2c_internal.h"
#include "m2c_kernels.h"

using namespace m2c;

void m2c_fill_grid(Grid* g, const m2c_config* c);   // m2c_api.hip

namespace {

struct RunHost {
    m2c_config cfg;
    RunDesc d;
    bool has_state = false;
    bool lam_valid = false;
    long long steps_base = 0;
};

}  // namespace

struct m2c_batch {
    int n = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<RunHost> runs;
    RunDesc* d_runs = nullptr;
    DevScalars* d_sc = nullptr;
    DevScalars* hsc = nullptr;       // pinned mirror [n]
    int2* d_cmap = nullptr;
    int ncblocks = 0;
    int2* d_items = nullptr;
    int nitems = 0;
    int tx = 16, ty = 16, kz = 8;
    bool mixed = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    char err[256] = {0};
};

namespace {

int berr(m2c_batch* b, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int berr(m2c_batch* b, int code, const char* fmt, ...)
{
    if (b) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(b->err, sizeof(b->err), fmt, ap);
        va_end(ap);
    }
    return code;
}

#define BCHK(b, expr)                                                                            \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) return berr((b), M2C_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

__global__ void k_batch_clear_err(DevScalars* sc, int n)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    sc[r].err = 0;
    sc[r].err_cell = LLONG_MAX;
}

__global__ void k_batch_zero_lam(DevScalars* sc) { sc->lam_bits = 0ull; }

int pull(m2c_batch* b)
{
    BCHK(b, hipMemcpyAsync(b->hsc, b->d_sc, b->n * sizeof(DevScalars), hipMemcpyDeviceToHost, b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));
    return M2C_OK;
}

int push(m2c_batch* b)
{
    BCHK(b, hipMemcpyAsync(b->d_sc, b->hsc, b->n * sizeof(DevScalars), hipMemcpyHostToDevice, b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));
    return M2C_OK;
}

void drop_graph(m2c_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// (Re)build the (run, tile) work list for the current tile shape.
int build_items(m2c_batch* b)
{
    std::vector<int2> items;
    for (int r = 0; r < b->n; ++r) {
        RunDesc& d = b->runs[r].d;
        d.kz = b->kz < d.g.nz ? b->kz : d.g.nz;
        d.tiles_x = (d.g.nx + b->tx - 1) / b->tx;
        d.tiles_y = (d.g.ny + b->ty - 1) / b->ty;
        d.tiles_z = (d.g.nz + d.kz - 1) / d.kz;
        const int nt = d.tiles_x * d.tiles_y * d.tiles_z;
        for (int t = 0; t < nt; ++t) items.push_back(make_int2(r, t));
    }
    if (b->d_items) (void)hipFree(b->d_items);
    b->d_items = nullptr;
    b->nitems = (int)items.size();
    BCHK(b, hipMalloc((void**)&b->d_items, items.size() * sizeof(int2)));
    BCHK(b, hipMemcpy(b->d_items, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice));
    std::vector<RunDesc> descs(b->n);
    for (int r = 0; r < b->n; ++r) descs[r] = b->runs[r].d;
    BCHK(b, hipMemcpy(b->d_runs, descs.data(), b->n * sizeof(RunDesc), hipMemcpyHostToDevice));
    drop_graph(b);
    return M2C_OK;
}

int enqueue_batch_step(m2c_batch* b, hipStream_t s)
{
    BCHK(b, launch_begin_batch(b->d_runs, b->n, 0.0, s));
    BCHK(b, launch_compact_batch(b->d_runs, b->n, b->d_cmap, b->ncblocks, s));
    BCHK(b, launch_fiver_batch(b->d_runs, b->n, 1, s));
    BCHK(b, launch_stage_batch(1, b->mixed, b->tx, b->ty, b->d_runs, b->d_items, b->nitems, s));
    BCHK(b, launch_fiver_batch(b->d_runs, b->n, 2, s));
    BCHK(b, launch_stage_batch(2, b->mixed, b->tx, b->ty, b->d_runs, b->d_items, b->nitems, s));
    BCHK(b, launch_phase_batch(b->d_runs, b->n, s));
    BCHK(b, launch_end_batch(b->d_runs, b->n, 2, s));
    return M2C_OK;
}

int ensure_graph(m2c_batch* b)
{
    if (b->exec) return M2C_OK;
    BCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed));
    int rc = enqueue_batch_step(b, b->stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return berr(b, M2C_ERR_DEVICE, "graph capture: %s", hipGetErrorString(e));
    b->graph = g;
    BCHK(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return M2C_OK;
}

// Steps of every run; returns the first failure (run order).
int run_batch(m2c_batch* b, int32_t nsteps, std::vector<long long>* done_out)
{
    BCHK(b, hipSetDevice(b->device));
    for (int r = 0; r < b->n; ++r)
        if (!b->runs[r].has_state) return berr(b, M2C_ERR_STATE, "run %d has no state", r);
    int rc = pull(b);
    if (rc) return rc;
    hipLaunchKernelGGL(k_batch_clear_err, dim3((b->n + 63) / 64), dim3(64), 0, b->stream, b->d_sc, b->n);
    for (int r = 0; r < b->n; ++r) {
        RunHost& R = b->runs[r];
        if (!R.lam_valid && !(R.cfg.dt_fixed > 0.0)) {
            const int cur = b->hsc[r].cur;
            hipLaunchKernelGGL(k_batch_zero_lam, dim3(1), dim3(1), 0, b->stream, R.d.sc);
            BCHK(b, launch_lambda(R.d.g, R.d.W[cur], R.d.chi[cur], R.d.sc, b->stream));
        }
    }
    BCHK(b, hipGetLastError());
    rc = ensure_graph(b);
    if (rc) return rc;
    std::vector<long long> done0(b->n);
    for (int r = 0; r < b->n; ++r) done0[r] = b->hsc[r].steps_done;
    for (int32_t k = 0; k < nsteps; ++k) BCHK(b, hipGraphLaunch(b->exec, b->stream));
    rc = pull(b);
    if (rc) return rc;
    int first = M2C_OK;
    for (int r = 0; r < b->n; ++r) {
        const DevScalars& d = b->hsc[r];
        if (done_out) done_out->push_back(d.steps_done - done0[r]);
        if (d.err != 0) {
            b->runs[r].lam_valid = false;
            const int code = d.err == ST_OVERFLOW ? M2C_ERR_NOMEM : d.err;
            if (first == M2C_OK) {
                first = code;
                berr(b, code, "run %d: step %lld failed (%s) at cell %lld", r, d.steps_done + 1,
                     m2c_strerror(code), d.err_cell);
            }
        } else {
            b->runs[r].lam_valid = true;
        }
    }
    return first;
}

const int kTileCandidates[][3] = {{16, 16, 8}, {16, 16, 4}, {32, 8, 8}, {16, 15, 8}, {32, 7, 8}, {16, 15, 4}};

}  // namespace

extern "C" {

void m2c_batch_destroy(m2c_batch* b)
{
    if (!b) return;
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    for (auto& R : b->runs) {
        for (int k = 0; k < 2; ++k) {
            (void)hipFree(R.d.W[k]);
            (void)hipFree(R.d.chi[k]);
        }
        (void)hipFree(R.d.W1);
        (void)hipFree(R.d.queue);
        (void)hipFree(R.d.fslot);
        (void)hipFree(R.d.fluxF);
        (void)hipFree(R.d.star);
        (void)hipFree(R.d.flips);
        (void)hipFree(R.d.blockcnt);
    }
    (void)hipFree(b->d_runs);
    (void)hipFree(b->d_sc);
    (void)hipFree(b->d_cmap);
    (void)hipFree(b->d_items);
    if (b->hsc) (void)hipHostFree(b->hsc);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

int m2c_batch_create(int32_t n, const m2c_config* cfgs, m2c_batch** out)
{
    if (!out || n < 1 || !cfgs) return M2C_ERR_ARG;
    *out = nullptr;
    for (int r = 0; r < n; ++r) {
        if (m2c_validate_config(&cfgs[r]) != M2C_OK) return M2C_ERR_ARG;
        if (cfgs[r].precision != cfgs[0].precision) return M2C_ERR_ARG;
        if (cfgs[r].rk_order != 2) return M2C_ERR_ARG;         // the batched kernels are TVD-RK2
        if (cfgs[r].eos_general) return M2C_ERR_ARG;           // and stiffened gases
        if (cfgs[r].limiter != M2C_LIM_MC || cfgs[r].flux != M2C_FLUX_HLLC || cfgs[r].ls_band != 0.0)
            return M2C_ERR_ARG;                                 // with MC, HLLC, the whole grid
    }
    m2c_batch* b = new (std::nothrow) m2c_batch();
    if (!b) return M2C_ERR_NOMEM;
    b->n = n;
    b->mixed = cfgs[0].precision == M2C_PREC_MIXED;
    if (cfgs[0].tile_x) {
        b->tx = cfgs[0].tile_x;
        b->ty = cfgs[0].tile_y;
    }
    if (cfgs[0].tile_z) b->kz = cfgs[0].tile_z;
    b->runs.resize(n);
    bool ok = hipGetDevice(&b->device) == hipSuccess &&
              hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) == hipSuccess;
    b->own_stream = ok;
    auto alloc = [&](void** p, size_t bytes) {
        if (ok && hipMalloc(p, bytes) != hipSuccess) {
            ok = false;
            *p = nullptr;
        }
    };
    alloc((void**)&b->d_sc, n * sizeof(DevScalars));
    alloc((void**)&b->d_runs, n * sizeof(RunDesc));
    if (ok && hipHostMalloc((void**)&b->hsc, n * sizeof(DevScalars), hipHostMallocDefault) != hipSuccess) ok = false;
    std::vector<int2> cmap;
    for (int r = 0; r < n && ok; ++r) {
        RunHost& R = b->runs[r];
        R.cfg = cfgs[r];
        memset(&R.d, 0, sizeof(R.d));
        m2c_fill_grid(&R.d.g, &cfgs[r]);
        const long long N = R.d.g.N;
        R.d.qcap = 3 * N;
        if (R.d.qcap > 65536 && R.d.qcap > N) R.d.qcap = N > 65536 ? N : 65536;
        R.d.nblk_compact = (int)((N + COMPACT_CELLS_PER_BLOCK - 1) / COMPACT_CELLS_PER_BLOCK);
        for (int k = 0; k < 2; ++k) {
            alloc((void**)&R.d.W[k], 6 * N * sizeof(double));
            alloc((void**)&R.d.chi[k], N);
        }
        alloc((void**)&R.d.W1, 6 * N * sizeof(double));
        alloc((void**)&R.d.queue, R.d.qcap * sizeof(int32_t));
        alloc((void**)&R.d.fslot, 3 * N * sizeof(int32_t));
        alloc((void**)&R.d.fluxF, 10 * R.d.qcap * sizeof(double));
        alloc((void**)&R.d.star, 8 * R.d.qcap * sizeof(double));
        alloc((void**)&R.d.flips, N * sizeof(int32_t));
        alloc((void**)&R.d.blockcnt, (size_t)R.d.nblk_compact * sizeof(int32_t));
        R.d.sc = b->d_sc + r;
        for (int k = 0; k < R.d.nblk_compact; ++k) cmap.push_back(make_int2(r, k));
        if (ok && launch_fill_i32(R.d.fslot, 3 * N, -1, b->stream) != hipSuccess) ok = false;
    }
    if (ok) {
        b->ncblocks = (int)cmap.size();
        alloc((void**)&b->d_cmap, cmap.size() * sizeof(int2));
    }
    if (ok && hipMemcpy(b->d_cmap, cmap.data(), cmap.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess)
        ok = false;
    if (ok) {
        memset(b->hsc, 0, n * sizeof(DevScalars));
        for (int r = 0; r < n; ++r) b->hsc[r].err_cell = LLONG_MAX;
        ok = push(b) == M2C_OK && build_items(b) == M2C_OK && hipStreamSynchronize(b->stream) == hipSuccess;
    }
    if (!ok) {
        m2c_batch_destroy(b);
        return M2C_ERR_NOMEM;
    }
    *out = b;
    return M2C_OK;
}

const char* m2c_batch_last_error(const m2c_batch* b) { return b ? b->err : "null batch"; }

int m2c_batch_size(const m2c_batch* b) { return b ? b->n : 0; }

int m2c_batch_set_state(m2c_batch* b, int32_t k, const double* prim6)
{
    if (!b || !prim6 || k < 0 || k >= b->n) return M2C_ERR_ARG;
    BCHK(b, hipSetDevice(b->device));
    RunHost& R = b->runs[k];
    const long long N = R.d.g.N;
    int rc = pull(b);
    if (rc) return rc;
    const int q = b->hsc[k].cur ^ 1;
    b->hsc[k].err = 0;
    b->hsc[k].err_cell = LLONG_MAX;
    rc = push(b);
    if (rc) return rc;
    BCHK(b, hipMemcpyAsync(R.d.W1, prim6, 6 * N * sizeof(double), hipMemcpyHostToDevice, b->stream));
    BCHK(b, launch_prim_to_cons(R.d.g, R.d.W1, R.d.W[q], R.d.chi[q], R.d.sc, b->stream));
    rc = pull(b);
    if (rc) return rc;
    if (b->hsc[k].err != 0) {
        const long long cell = b->hsc[k].err_cell;
        b->hsc[k].err = 0;
        b->hsc[k].err_cell = LLONG_MAX;
        push(b);
        return berr(b, M2C_ERR_NONPHYSICAL, "run %d: inadmissible primitive state at cell %lld", k, cell);
    }
    b->hsc[k].cur = q;
    rc = push(b);
    if (rc) return rc;
    R.has_state = true;
    R.lam_valid = false;
    return M2C_OK;
}

int m2c_batch_get_state(m2c_batch* b, int32_t k, double* prim6, uint8_t* id)
{
    if (!b || !prim6 || k < 0 || k >= b->n) return M2C_ERR_ARG;
    RunHost& R = b->runs[k];
    if (!R.has_state) return berr(b, M2C_ERR_STATE, "run %d has no state", k);
    BCHK(b, hipSetDevice(b->device));
    int rc = pull(b);
    if (rc) return rc;
    const int cur = b->hsc[k].cur;
    const long long N = R.d.g.N;
    BCHK(b, launch_cons_to_prim(R.d.g, R.d.W[cur], R.d.chi[cur], R.d.W1, b->stream));
    BCHK(b, hipMemcpyAsync(prim6, R.d.W1, 6 * N * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    if (id) BCHK(b, hipMemcpyAsync(id, R.d.chi[cur], N, hipMemcpyDeviceToHost, b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));
    return M2C_OK;
}

int m2c_batch_get_conserved(m2c_batch* b, int32_t k, double* w6)
{
    if (!b || !w6 || k < 0 || k >= b->n) return M2C_ERR_ARG;
    RunHost& R = b->runs[k];
    if (!R.has_state) return berr(b, M2C_ERR_STATE, "run %d has no state", k);
    BCHK(b, hipSetDevice(b->device));
    int rc = pull(b);
    if (rc) return rc;
    const int cur = b->hsc[k].cur;
    BCHK(b, hipMemcpyAsync(w6, R.d.W[cur], 6 * R.d.g.N * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));
    return M2C_OK;
}

int m2c_batch_step(m2c_batch* b, int32_t nsteps)
{
    if (!b || nsteps < 0) return M2C_ERR_ARG;
    return run_batch(b, nsteps, nullptr);
}

int m2c_batch_get_stats(m2c_batch* b, int32_t k, m2c_stats* s)
{
    if (!b || !s || k < 0 || k >= b->n) return M2C_ERR_ARG;
    BCHK(b, hipSetDevice(b->device));
    int rc = pull(b);
    if (rc) return rc;
    const DevScalars& d = b->hsc[k];
    memset(s, 0, sizeof(*s));
    s->steps = d.steps_done - b->runs[k].steps_base;
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
    return M2C_OK;
}

int m2c_batch_set_tile(m2c_batch* b, int32_t tx, int32_t ty, int32_t kz)
{
    if (!b || !stage_tile_supported(tx, ty) || kz < 1) return M2C_ERR_ARG;
    BCHK(b, hipSetDevice(b->device));
    b->tx = tx;
    b->ty = ty;
    b->kz = kz;
    return build_items(b);
}

int m2c_batch_get_tile(const m2c_batch* b, int32_t tile[3])
{
    if (!b || !tile) return M2C_ERR_ARG;
    tile[0] = b->tx;
    tile[1] = b->ty;
    tile[2] = b->kz;
    return M2C_OK;
}

int m2c_batch_autotune(m2c_batch* b, int32_t steps, int32_t tile_out[3], float* ms_out)
{
    if (!b || steps < 1) return M2C_ERR_ARG;
    BCHK(b, hipSetDevice(b->device));
    for (int r = 0; r < b->n; ++r)
        if (!b->runs[r].has_state) return berr(b, M2C_ERR_STATE, "run %d has no state", r);
    int rc = pull(b);
    if (rc) return rc;
    // snapshot of every run's current state, ids and device scalars
    std::vector<DevScalars> sc0(b->hsc, b->hsc + b->n);
    std::vector<bool> lam0(b->n);
    size_t bytes = 0;
    for (auto& R : b->runs) bytes += 6 * R.d.g.N * sizeof(double) + R.d.g.N;
    char* snap = nullptr;
    BCHK(b, hipMalloc((void**)&snap, bytes));
    auto copy_states = [&](bool save) -> int {
        size_t off = 0;
        for (int r = 0; r < b->n; ++r) {
            RunHost& R = b->runs[r];
            const int cur = sc0[r].cur;
            const size_t wb = 6 * R.d.g.N * sizeof(double);
            if (save) {
                BCHK(b, hipMemcpyAsync(snap + off, R.d.W[cur], wb, hipMemcpyDeviceToDevice, b->stream));
                BCHK(b, hipMemcpyAsync(snap + off + wb, R.d.chi[cur], R.d.g.N, hipMemcpyDeviceToDevice, b->stream));
            } else {
                BCHK(b, hipMemcpyAsync(R.d.W[cur], snap + off, wb, hipMemcpyDeviceToDevice, b->stream));
                BCHK(b, hipMemcpyAsync(R.d.chi[cur], snap + off + wb, R.d.g.N, hipMemcpyDeviceToDevice, b->stream));
            }
            off += wb + R.d.g.N;
        }
        return M2C_OK;
    };
    for (int r = 0; r < b->n; ++r) lam0[r] = b->runs[r].lam_valid;
    rc = copy_states(true);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = berr(b, M2C_ERR_DEVICE, "event create");
    float best = -1.0f;
    int bt[3] = {b->tx, b->ty, b->kz};
    for (const auto& cand : kTileCandidates) {
        if (rc) break;
        rc = m2c_batch_set_tile(b, cand[0], cand[1], cand[2]);
        if (rc) break;
        // restore, warm up (builds the graph), restore, time
        std::memcpy(b->hsc, sc0.data(), b->n * sizeof(DevScalars));
        if ((rc = push(b)) || (rc = copy_states(false))) break;
        for (int r = 0; r < b->n; ++r) b->runs[r].lam_valid = lam0[r];
        if ((rc = run_batch(b, 1, nullptr))) break;
        std::memcpy(b->hsc, sc0.data(), b->n * sizeof(DevScalars));
        if ((rc = push(b)) || (rc = copy_states(false))) break;
        for (int r = 0; r < b->n; ++r) b->runs[r].lam_valid = lam0[r];
        if (hipEventRecord(e0, b->stream) != hipSuccess) { rc = M2C_ERR_DEVICE; break; }
        if ((rc = run_batch(b, steps, nullptr))) break;
        if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
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
    // leave the batch as it was, with the fastest tile
    int rc2 = m2c_batch_set_tile(b, bt[0], bt[1], bt[2]);
    std::memcpy(b->hsc, sc0.data(), b->n * sizeof(DevScalars));
    if (!rc2) rc2 = push(b);
    if (!rc2) rc2 = copy_states(false);
    if (!rc2 && hipStreamSynchronize(b->stream) != hipSuccess) rc2 = M2C_ERR_DEVICE;
    for (int r = 0; r < b->n; ++r) b->runs[r].lam_valid = lam0[r];
    (void)hipFree(snap);
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

}  // extern "C"
