// m2c_internal.h -- structures shared by the host runtime and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "m2c_eos.h"

namespace m2c {

enum { BC_TRANSMISSIVE = 0, BC_WALL = 1, BC_PERIODIC = 2 };
enum { ST_OK = 0, ST_NONPHYSICAL = -2, ST_RIEMANN = -3, ST_OVERFLOW = -7 };
enum { LIM_MC = 0, LIM_VA = 1, LIM_VA_MOD = 2 };       // the values of M2C_LIM_*
enum { FLUX_HLLC = 0, FLUX_LLF = 1 };                  // the values of M2C_FLUX_*

// Device-resident scalars of one simulation.  Everything a step needs from
// the previous step (dt, error state) stays on the device so a whole step
// can be enqueued (or graph-replayed) without host round trips.
struct DevScalars {
    unsigned long long lam_bits;   // max_i lambda_i of the current state (bits of a
                                   // non-negative double: integer max == double max)
    double dt;                     // dt of the step in flight
    double t;                      // simulated time
    int32_t qlen;                  // interface faces in the work queue
    int32_t qlen_prev;             // queue length before the last compaction
    int32_t nflip;                 // flipped cells of the step in flight
    int32_t err;                   // 0 or the first error status
    long long err_cell;            // first failing cell (min over reports)
    long long steps_done;
    long long solves, newton_iters, fallbacks, flips, orphans, mlp_fallbacks;
    double dt_last;
    int32_t qvalid;                // queue and face slots built for the current material ids
    int32_t qreuse;                // this step keeps them (no cell flipped in the last step)
    int32_t cur;                   // batched runs: index (0/1) of the current full state
};

// One simulation grid as the kernels see it.
struct Grid {
    int nx, ny, nz;
    long long N;
    int act[3];                    // axis has more than one cell
    int bc[6];
    double h[3], rh[3], rh6[3];    // width, 1/width, 1/(6 width)
    double gamma[2], pc[2], gpc[2], inv_gm1[2];
    double alpha;
    double cfl, dt_fixed;
    double rtol;
    int maxit;
    int guess;
    int rk_stages;                 // Runge-Kutta stages per step (1, 2 or 3)
    int limiter, limk;             // slope limiter (M2C_LIM_*) and Van Albada exponent
    int flux;                      // numerical flux (M2C_FLUX_*)
    double ls_band;                // > 0: level set advanced only where |phi| < ls_band
    int eosg;                      // materials follow ek[] (general EOS)
    double rds;                    // RK4 step of general-EOS isentropes
    eos::EosK ek[2];               // prepared general EOS of materials 0 and 1
};

// Device buffers of one simulation.
struct Bufs {
    double* W[2];                  // two full states [6][N]: rho, rho u, rho v, rho w, rho E, phi
    double* W1;                    // RK stage state [6][N]
    uint8_t* chi[2];               // material ids of the two states
    int32_t* queue;                // interface face ids, ascending
    int32_t* fslot;                // [3N] face id -> queue index, or -1
    double* fluxF;                 // [qcap][10]: flux for the lower cell (5), upper cell (5)
    double* star;                  // [8][qcap]: p*, u*, rho*_L, rho*_R, vt1_L, vt2_L, vt1_R, vt2_R
    int32_t* flips;                // [N] flipped cells of the step in flight
    int32_t* blockcnt;             // compaction partial counts
    DevScalars* sc;
    long long qcap;
    int nblk_compact;
};

struct MlpDev;                     // learned star-pressure guess (optional)

}  // namespace m2c
