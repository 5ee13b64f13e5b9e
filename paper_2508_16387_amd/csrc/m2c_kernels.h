// m2c_kernels.h -- launch interfaces of the device kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "m2c_internal.h"

namespace m2c {

// Device buffers of one run of a batch (the kernels pick the state buffers
// from the run's device-side parity sc->cur).
struct RunDesc {
    Grid g;
    double* W[2];
    double* W1;
    uint8_t* chi[2];
    int32_t* queue;
    int32_t* fslot;
    double* fluxF;
    double* star;
    int32_t* flips;
    int32_t* blockcnt;
    DevScalars* sc;
    long long qcap;
    int nblk_compact;
    int tiles_x, tiles_y, tiles_z, kz;
};

// Arguments of one bulk Runge-Kutta stage launch.
struct StageArgs {
    Grid g;
    const double* Win;             // stage input state [6][N]
    const double* W0;              // start-of-step state [6][N] (blended stages)
    double* Wout;                  // stage output [6][N]
    const uint8_t* chi;            // material ids frozen for the step
    uint8_t* chi_next;             // last stage: ids of the new level set
    int32_t* flips;                // last stage: flipped cells (append)
    const int32_t* fslot;          // [3N] face -> queue slot or -1
    const double* fluxF;           // [qcap][10] one-sided interface fluxes
    long long qcap;
    DevScalars* sc;
    int tiles_x, tiles_y, tiles_z, kz;
    double c0, c1;                 // blend of the stage: c0 W0 + c1 (Win + dt R)
};

// Interface work-queue arguments (compaction, FIVER, phase update).
struct IfaceArgs {
    Grid g;
    const double* Win;             // stage input state [6][N]
    const uint8_t* chi;            // ids frozen for the step
    int32_t* queue;
    int32_t* fslot;
    double* fluxF;                 // [qcap][10]
    double* star;                  // [8][qcap]
    int32_t* blockcnt;
    long long qcap;
    int nblk;                      // compaction blocks
    DevScalars* sc;
};

struct PhaseArgs {
    Grid g;
    double* W;                     // new state [6][N] (updated in place at flipped cells)
    const uint8_t* chi_old;        // ids of the step
    const uint8_t* chi_new;        // ids of the new level set
    const int32_t* flips;
    const int32_t* fslot;
    const double* star;
    long long qcap;
    DevScalars* sc;
};

bool stage_tile_supported(int tx, int ty);
// stage: kind 1 (first), 2 (last, blended), 3 (middle of RK3), 4 (forward
// Euler); the batched kernel has kinds 1 and 2 (TVD-RK2)
hipError_t launch_stage(int stage, bool mixed, int tx, int ty, const StageArgs& a, hipStream_t s);
// the same with the configured limiter and flux (any, including MC + HLLC)
hipError_t launch_stage_opts(int stage, bool mixed, int tx, int ty, const StageArgs& a, hipStream_t s);
// general-EOS stage kernels (FP64; tiles 16x15 and 64x2)
bool stage_tile_supported_eos(int tx, int ty);
hipError_t launch_stage_eos(int stage, int tx, int ty, const StageArgs& a, hipStream_t s);
// the default scheme on the 16x15 tile for fs, the set of the two
// materials' families (eos::fam_set): sets with NASG, and the others
hipError_t launch_stage_eos_nasg(int stage, int fs, const StageArgs& a, hipStream_t s);
hipError_t launch_stage_eos_other(int stage, int fs, const StageArgs& a, hipStream_t s);
// items: (run, tile) pairs over all runs of a batch
hipError_t launch_stage_batch(int stage, bool mixed, int tx, int ty, const RunDesc* runs, const int2* items,
                              int nitems, hipStream_t s);

// Interface kernels (k_interface.hip).
constexpr int COMPACT_THREADS = 256;
constexpr int COMPACT_CELLS_PER_THREAD = 16;
constexpr int COMPACT_CELLS_PER_BLOCK = COMPACT_THREADS * COMPACT_CELLS_PER_THREAD;
// count / scan / scatter of the interface queue; the count kernel also runs
// the previous step's phase update (prev_phase, nullable), the scan kernel
// ends the previous step (end_prev) and starts this one (begin: dt, cleared
// accumulators)
hipError_t launch_compact(const IfaceArgs& a, const PhaseArgs* prev_phase, bool end_prev, bool begin,
                          double dt_imposed, hipStream_t s);
hipError_t launch_end_step(DevScalars* sc, int stages, hipStream_t s);
// mlp: the learned guess (null: acoustic).
hipError_t launch_fiver(const IfaceArgs& a, bool record, const MlpDev* mlp, hipStream_t s);
hipError_t launch_phase(const PhaseArgs& a, hipStream_t s);
// Batched forms: cmap maps each compaction block to (run, block of run).
hipError_t launch_compact_batch(const RunDesc* runs, int nruns, const int2* cmap, int ncblocks, hipStream_t s);
hipError_t launch_fiver_batch(const RunDesc* runs, int nruns, int stage, hipStream_t s);
hipError_t launch_phase_batch(const RunDesc* runs, int nruns, hipStream_t s);

// Learned star-pressure guess (k_mlp.hip).
struct MlpDev;
hipError_t launch_mlp_features(long long n, const double* in, const double* eos, const double* ps, float* X,
                               float* tg, hipStream_t s);
hipError_t launch_mlp_forward(long long n, const float* X, const MlpDev& m, float* y, hipStream_t s);
hipError_t launch_mlp_grad(long long i0, long long cnt, long long ntot, float invB, const float* X, const float* T,
                           const MlpDev& m, float* grad, float* sse, hipStream_t s);
hipError_t launch_fill_f32(float* p, long long n, float v, hipStream_t s);
hipError_t launch_adam(const MlpDev& md, float* m, float* v, float* grad, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s);
hipError_t launch_mlp_sync(const MlpDev& m, hipStream_t s);
hipError_t launch_points_guess(long long n, const double* in, const double* eos, const MlpDev& m, double* guess,
                               hipStream_t s);

// Per-step bookkeeping and state conversion (k_misc.hip).
hipError_t launch_begin_batch(const RunDesc* runs, int nruns, double dt_imposed, hipStream_t s);
hipError_t launch_end_batch(const RunDesc* runs, int nruns, int stages, hipStream_t s);
hipError_t launch_lambda(const Grid& g, const double* W, const uint8_t* chi, DevScalars* sc, hipStream_t s);
hipError_t launch_prim_to_cons(const Grid& g, const double* prim6, double* W, uint8_t* chi,
                               DevScalars* sc, hipStream_t s);
hipError_t launch_cons_to_prim(const Grid& g, const double* W, const uint8_t* chi, double* prim6,
                               hipStream_t s);
hipError_t launch_chi_from_phi(const Grid& g, const double* W, uint8_t* chi, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, long long n, int32_t v, hipStream_t s);
hipError_t launch_hllc_points(long long n, const double* qL, const double* qR, double gamma, double pc,
                              bool mixed, double* F, hipStream_t s);
// guess (nullable): candidate initial pressures, judged against the
// acoustic guess; nfb (nullable) counts problems that started from the
// acoustic guess although a candidate was given.
hipError_t launch_riemann_points(long long n, const double* in, const double* eos, const double* guess,
                                 double rtol, int maxit, double* out, int32_t* iters, int32_t* nvac,
                                 unsigned long long* nfb, hipStream_t s);

}  // namespace m2c
