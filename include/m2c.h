/*
 * m2c.h -- C ABI of the MI355X (gfx950) two-material finite-volume library.
 *
 * The library advances the 3D compressible Euler equations for two
 * stiffened-gas materials separated by one level set on a uniform Cartesian
 * grid, following the method of M2C (arXiv 2508.16387):
 *   - cell-centred finite volumes (eq. NS_discretized, inviscid, no source);
 *   - MUSCL reconstruction of the primitive variables with the MC limiter
 *     (appendix "Slope limiters", eqs. theta and AB);
 *   - HLLC fluxes at faces inside one material (appendix "HLLC flux");
 *   - FIVER at faces between materials: the exact two-material Riemann
 *     problem along the face normal (eq. 1DRiemannProblem) gives star
 *     states that feed one one-sided flux per side (section "Spatial
 *     discretization of governing equations");
 *   - level-set advection (eq. levelset) by third-order upwind differences
 *     (section "Level set method");
 *   - TVD Runge-Kutta time integration with a CFL-based time step
 *     (section "Time integration");
 *   - the phase update of the time-step outline (step 6, section "Code
 *     structure") for cells whose level-set sign changed.
 *
 * Conventions shared by every call
 *   - Arrays are structure-of-arrays, x fastest: cell (i,j,k) has index
 *     c = i + nx*(j + ny*k); a field of N = nx*ny*nz cells is N contiguous
 *     values, and "[m][N]" means m such fields back to back.  No ghost cells
 *     cross the ABI.
 *   - Material 1 occupies phi < 0, material 0 phi >= 0.  Material ids are
 *     always derived from phi, never passed in.
 *   - Stiffened gas per material m: p = (gamma_m - 1) rho e - gamma_m pc_m
 *     (eq. NASG_EOS with b = e_c = 0).
 *   - Ownership: the caller owns every pointer it passes; the library copies
 *     what it needs during the call and keeps no caller pointer.  Calls that
 *     take device pointers work on the context's stream (m2c_set_stream) and
 *     the memory must stay valid until that stream has finished the call.
 *   - Errors: every call returns an m2c_status; nothing throws across the
 *     ABI.  m2c_last_error() gives a message for the last failure of a
 *     context.  A context is not thread-safe; distinct contexts are
 *     independent.
 */
#ifndef M2C_H
#define M2C_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum m2c_status {
    M2C_OK = 0,
    M2C_ERR_ARG = -1,           /* invalid argument or configuration           */
    M2C_ERR_NONPHYSICAL = -2,   /* rho <= 0, p + p_c <= 0 or non-finite value  */
    M2C_ERR_RIEMANN = -3,       /* interface Riemann problem with no admissible
                                   star pressure (a vacuum would open)          */
    M2C_ERR_DEVICE = -4,        /* HIP runtime failure                          */
    M2C_ERR_STATE = -5,         /* call out of order (e.g. step before set)     */
    M2C_ERR_UNIMPLEMENTED = -6,
    M2C_ERR_NOMEM = -7
} m2c_status;

enum { M2C_BC_TRANSMISSIVE = 0,  /* zero-gradient copy of the boundary cell    */
       M2C_BC_WALL = 1,          /* mirror image, normal velocity reversed      */
       M2C_BC_PERIODIC = 2 };
enum { M2C_PREC_FP64 = 0,        /* everything in FP64                          */
       M2C_PREC_MIXED = 1 };     /* FP32 reconstruction + HLLC at single-material
                                    faces; FP64 EOS inversion, FIVER, residual
                                    accumulation, level set and time step      */
enum { M2C_GUESS_ACOUSTIC = 0,   /* linearised (acoustic) star-pressure guess   */
       M2C_GUESS_MLP = 1 };      /* learned guess, judged against the acoustic  */
/* Slope limiters, appendix "Slope limiters" (uniform grid, A = B = 1). */
enum { M2C_LIM_MC = 0,           /* monotonized central, parameter limiter_alpha */
       M2C_LIM_VAN_ALBADA = 1,   /* (theta^k + theta) / (theta^k + 1)           */
       M2C_LIM_VAN_ALBADA_MOD = 2 }; /* the same, 0 where negative             */
/* Numerical flux at single-material faces and for the one-sided FIVER
 * fluxes (appendix "Numerical flux functions"). */
enum { M2C_FLUX_HLLC = 0, M2C_FLUX_LLF = 1 };

/* General equations of state p = p(rho, e) (section "Equations of state",
 * eq. eos_all), one per material, for the two-material Riemann problem of
 * eq. 1DRiemannProblem and the time step with eos_general set; the families
 * of that section and its appendix:
 *   M2C_EOS_NASG  Noble-Abel stiffened gas, eq. NASG_EOS:
 *                 p = (gamma - 1) rho (e - e_c) / (1 - rho b) - gamma p_c;
 *                 prm = {gamma > 1, p_c >= 0, b >= 0, e_c}
 *   M2C_EOS_MG    Mie-Grueneisen in the compression / small-tension /
 *                 tensile-cutoff form of the appendix:
 *                 p = p_R(eta) + rho_0 Gamma_0 (e - e_R(eta)), eta = 1 - rho_0/rho;
 *                 prm = {rho_0 > 0, c_0 > 0, Gamma_0 > 0, s >= 0, e_0, eta_min < 0}
 *   M2C_EOS_JWL   Jones-Wilkins-Lee, eq. JWL_EOS (both exponentials decaying):
 *                 p = omega rho e + sum_i A_i (1 - omega rho/(R_i rho_0)) exp(-R_i rho_0/rho);
 *                 prm = {omega > 0, A_1, A_2, R_1 > 0, R_2 > 0, rho_0 > 0}
 * Unused trailing prm entries are ignored.  A state or star pressure must
 * lie above the family's floor by 1e-12 (p_K - floor) + 1e-6 |floor| (floor:
 * -p_c for NASG, p_min = rho_0 c_0^2 eta_min for MG, 0 for JWL); a problem
 * whose sides separate faster than that allows has no star state. */
enum { M2C_EOS_NASG = 0, M2C_EOS_MG = 1, M2C_EOS_JWL = 2 };
#define M2C_EOS_MAX 8                 /* materials per call                   */
typedef struct m2c_eos {
    int32_t family;                   /* M2C_EOS_*                            */
    int32_t reserved;                 /* 0                                    */
    double prm[7];                    /* parameters, in the order above       */
} m2c_eos;

/* Problem and method parameters (the "Mesh", "Equations", "BoundaryCondition",
 * "Space", "Time" and "ExactRiemannSolution" input classes of the paper's
 * input-file table). */
typedef struct m2c_config {
    uint32_t struct_size;       /* = sizeof(m2c_config)                        */
    int32_t nx, ny, nz;         /* cells per axis (>= 1)                       */
    double lo[3], hi[3];        /* domain box                                  */
    double gamma[2], pc[2];     /* stiffened gas of material 0 and 1           */
    int32_t bc[6];              /* -x,+x,-y,+y,-z,+z; periodic must pair up    */
    double limiter_alpha;       /* MC parameter alpha in [0, 2] (paper default
                                   1.2; 0: constant reconstruction)             */
    int32_t rk_order;           /* 1 forward Euler, 2 TVD-RK2 (default), 3
                                   TVD-RK3 (Shu-Osher); batches: 2 only; other
                                   values: M2C_ERR_ARG                           */
    double cfl;                 /* dt = cfl / max_i sum_d (|V_d|+c)/h_d        */
    double dt_fixed;            /* > 0: constant dt instead of the CFL rule    */
    int32_t precision;          /* M2C_PREC_*                                  */
    int32_t guess;              /* M2C_GUESS_ACOUSTIC; a learned guess is
                                   attached with m2c_set_guess (M2C_GUESS_MLP
                                   here: M2C_ERR_ARG)                            */
    double riemann_rtol;        /* Newton stop: |dp| <= rtol (p - p_lo)        */
    int32_t riemann_maxit;      /* Newton steps before the bisection fallback  */
    int32_t tile_x, tile_y, tile_z;  /* stage-kernel tile; 0 = library choice  */
    int32_t limiter;            /* M2C_LIM_* (default MC; batches: MC only)     */
    int32_t limiter_k;          /* Van Albada exponent: even, 2..8 (default 2;
                                   odd k has a pole at theta = -1)              */
    int32_t flux;               /* M2C_FLUX_* (default HLLC; batches: HLLC only) */
    double ls_band;             /* > 0: narrow band -- the level set is advanced
                                   only where the stage-input |phi| < ls_band and
                                   held elsewhere (section "Level set method");
                                   0 (default): whole grid; batches: 0 only     */
    int32_t eos_general;        /* 1: material m follows eos[m] (gamma, pc are
                                   then unused): every conversion, sound speed
                                   and flux takes that EOS, and interface faces
                                   take the general-EOS exact Riemann solve;
                                   FP64 precision and the acoustic guess only,
                                   no batches.  0 (default): stiffened gases   */
    int32_t eos_reserved;       /* 0                                            */
    m2c_eos eos[2];             /* materials 0 and 1 when eos_general           */
    double riemann_ds;          /* RK4 step of general-EOS isentropes (0: 0.01;
                                   else in [1e-3, 0.5])                          */
} m2c_config;

/* Counters and timings since m2c_create (or the last m2c_reset_stats). */
typedef struct m2c_stats {
    int64_t steps;              /* completed steps                              */
    double t;                   /* simulated time                               */
    double dt_last;             /* dt of the last completed step                */
    int64_t iface_faces_last;   /* interface faces (Riemann problems per stage)
                                   of the last step                             */
    int64_t riemann_solves;     /* interface Riemann problems solved            */
    int64_t newton_iters;       /* Newton steps summed over all solves          */
    int64_t bisection_fallbacks;
    int64_t flips;              /* cells whose material changed                 */
    int64_t orphans;            /* flipped cells without a neighbour of their
                                   new material (state kept, re-encoded)        */
    int64_t mlp_fallbacks;      /* with a learned guess: solves that started from
                                   the acoustic guess (judged better, unusable
                                   network output, or near-equilibrium face)    */
    int32_t err_code;           /* m2c_status of the failing step, 0 if none    */
    int32_t pad0;
    int64_t err_cell;           /* first cell (or face/3) found failing, -1     */
    double ms_stage;            /* device time of the bulk stage kernels        */
    double ms_fiver;            /* device time of the interface Riemann kernel  */
    double ms_other;            /* device time of every other kernel of a step  */
    int64_t stage_launches;     /* bulk stage-kernel launches timed             */
    int64_t fiver_launches;
} m2c_stats;

typedef struct m2c_ctx m2c_ctx;

/* Fill a configuration with the defaults: 1 cell, unit box, air/water,
 * transmissive, MC limiter with alpha 1.2 (Van Albada k 2), HLLC, RK2, CFL
 * 0.5, FP64, acoustic guess, rtol 1e-12, maxit 50, library-chosen tiles. */
void m2c_config_default(m2c_config* c);
/* M2C_OK if m2c_create would accept the configuration, else M2C_ERR_ARG
 * (no device work, usable without a GPU). */
int m2c_validate_config(const m2c_config* c);

/* Validate the configuration, select device 'current' and allocate every
 * device buffer of the context: 162 B per cell (two full states, the stage
 * state, two material-id fields, the face -> queue-slot map, the flip list)
 * plus 148 B per interface-queue slot (id, two one-sided fluxes, star
 * record); the queue holds 3N slots for grids up to 65536 cells and N
 * above, about 310 B per cell in all (17.6 GB at 384^3).  A step whose
 * interface faces exceed the queue fails with M2C_ERR_NOMEM.  *out is NULL
 * on failure. */
int m2c_create(const m2c_config* c, m2c_ctx** out);
void m2c_destroy(m2c_ctx* ctx);
const char* m2c_last_error(const m2c_ctx* ctx);
const char* m2c_strerror(int status);

/* Use a caller stream (hipStream_t, e.g. a torch stream) for every later
 * launch of the context; NULL selects the default stream. */
int m2c_set_stream(m2c_ctx* ctx, void* hip_stream);

/* Initial / replacement state from host primitives prim6 = [rho,u,v,w,p,phi][N].
 * Rejects rho <= 0, p + p_c <= 0 and non-finite values (M2C_ERR_NONPHYSICAL,
 * err_cell set) without changing the context's state.  Synchronous. */
int m2c_set_state(m2c_ctx* ctx, const double* prim6);
/* Same from device memory (6N doubles); asynchronous on the context stream
 * except for the validity check, which synchronises. */
int m2c_set_state_device(m2c_ctx* ctx, const double* dprim6);

/* Current state as host primitives [rho,u,v,w,p,phi][N]; id (nullable)
 * receives the N material ids.  Synchronous. */
int m2c_get_state(m2c_ctx* ctx, double* prim6, uint8_t* id);
int m2c_get_state_device(m2c_ctx* ctx, double* dprim6);

/* Conservative state [rho, rho u, rho v, rho w, rho E, phi][N] -- a bit-exact
 * checkpoint (primitive <-> conservative is not a bit-exact round trip). */
int m2c_get_conserved(m2c_ctx* ctx, double* w6);
int m2c_set_conserved(m2c_ctx* ctx, const double* w6);

/* Advance nsteps full time steps (each: CFL dt, RK stages, phase update).
 * Transactional per step: on M2C_ERR_NONPHYSICAL or M2C_ERR_RIEMANN the
 * state is the one after the last completed step and the error is in
 * m2c_get_stats.  *t_out (nullable) receives the simulated time.  Returns
 * after the device has finished. */
int m2c_step(m2c_ctx* ctx, int32_t nsteps, double* t_out);
/* Same, but with dt imposed for every step instead of the CFL rule. */
int m2c_step_dt(m2c_ctx* ctx, int32_t nsteps, double dt, double* t_out);

int m2c_get_stats(m2c_ctx* ctx, m2c_stats* s);
int m2c_reset_stats(m2c_ctx* ctx);
/* every >= 1: time the kernel classes of one step in `every` (the first
 * step after switching on, then every `every`-th step)
 * with HIP events recorded on the context stream around the kernels; the
 * events are read when m2c_step returns and summed into ms_stage, ms_fiver,
 * ms_other and stage_launches of m2c_stats.  Each timed step carries seven
 * event records (a few microseconds).  0: off (default).  Negative:
 * M2C_ERR_ARG. */
int m2c_set_profiling(m2c_ctx* ctx, int every);

/* Interface faces of the current material field: ascending face ids
 * f = 3c + d (face between cell c and its +d neighbour, periodic wrap
 * included), exactly as the Riemann work queue holds them.  Writes at most
 * cap ids to the host array out (nullable) and the total to *count. */
int m2c_interface_faces(m2c_ctx* ctx, int32_t* out, int64_t cap, int64_t* count);

/* Time every supported stage tile (tile_x, tile_y, planes per block) on the
 * context's own grid and state for `steps` steps each and keep the fastest.
 * The state, statistics and simulated time are restored afterwards (the call
 * allocates a temporary copy of the state).  tile_out (nullable) receives
 * the chosen tile, ms_out (nullable) its mean time per step. */
int m2c_autotune(m2c_ctx* ctx, int32_t steps, int32_t tile_out[3], float* ms_out);
int m2c_get_tile(const m2c_ctx* ctx, int32_t tile[3]);

/* ---- batched form: many independent runs advanced together ---------------
 * n runs of uneven grid sizes (one precision and one stage tile for all).
 * One step of all runs is one persistent stage kernel per Runge-Kutta stage
 * (a work list of (run, tile) items over the whole batch) plus the interface
 * kernels, captured once into a hipGraph and replayed per step; every run
 * keeps its own CFL time step, error state and state parity in device
 * memory.  Runs are numbered 0..n-1 in the order of cfgs; the state and
 * statistics calls mean the same as for a single context.  A run that fails
 * a step stops advancing (its last good state is kept) while the others go
 * on; m2c_batch_step then returns the first failing run's status. */
typedef struct m2c_batch m2c_batch;
/* cfgs: n valid configurations with one precision, rk_order 2, the MC
 * limiter and the HLLC flux; otherwise M2C_ERR_ARG. */
int m2c_batch_create(int32_t n, const m2c_config* cfgs, m2c_batch** out);
void m2c_batch_destroy(m2c_batch* b);
const char* m2c_batch_last_error(const m2c_batch* b);
int m2c_batch_size(const m2c_batch* b);
int m2c_batch_set_state(m2c_batch* b, int32_t run, const double* prim6);
int m2c_batch_get_state(m2c_batch* b, int32_t run, double* prim6, uint8_t* id);
int m2c_batch_get_conserved(m2c_batch* b, int32_t run, double* w6);
int m2c_batch_step(m2c_batch* b, int32_t nsteps);
int m2c_batch_get_stats(m2c_batch* b, int32_t run, m2c_stats* s);
int m2c_batch_set_tile(m2c_batch* b, int32_t tile_x, int32_t tile_y, int32_t planes);
int m2c_batch_get_tile(const m2c_batch* b, int32_t tile[3]);
/* Autotuner of the batch: as m2c_autotune, over all runs at once. */
int m2c_batch_autotune(m2c_batch* b, int32_t steps, int32_t tile_out[3], float* ms_out);

/* ---- kernel-level entry points (device pointers, given stream) ---------- */

/* HLLC flux at n faces in the face frame: qL, qR = [rho,u_n,v_t1,v_t2,p][n]
 * (SoA), one stiffened gas (gamma, pc); F = [5][n].  prec selects the FP64
 * or the FP32 flux of the mixed form (inputs and outputs stay FP64). */
int m2c_eval_hllc(int64_t n, const double* qL, const double* qR, double gamma, double pc,
                  int32_t prec, double* F, void* hip_stream);

/* Exact two-material Riemann problems: in = [rho_L,u_L,p_L,rho_R,u_R,p_R][n],
 * eos = [gamma_L,pc_L,gamma_R,pc_R][n], out = [p*,u*,rho*_L,rho*_R][n],
 * iters (nullable) = Newton steps per problem (negative: bisection fallback;
 * 0: no admissible star pressure, out = NaN).  Always-FP64 safeguarded Newton
 * from the acoustic guess; guess must be M2C_GUESS_ACOUSTIC (other values:
 * M2C_ERR_UNIMPLEMENTED; the learned guess: m2c_riemann_solve_learned).
 * Returns M2C_ERR_RIEMANN if any problem had no admissible star pressure. */
int m2c_riemann_solve(int64_t n, const double* in, const double* eos, int32_t guess,
                      double rtol, int32_t maxit, double* out, int32_t* iters,
                      void* hip_stream);

/* ---- learned star-pressure guess --------------------------------------------
 * The paper accelerates its exact two-material Riemann solver without new
 * approximations (section "Spatial discretization of governing equations").
 * Here the acceleration is a learned initial guess for the star-pressure
 * Newton iteration: a network 8 -> 64 -> 64 -> 1 (tanh hidden layers; BF16
 * weights on the matrix cores, FP32 accumulation) maps eight dimensionless
 * features of a problem to y = ln((p* - p_lo)/P), p_lo = -min(pc_L, pc_R),
 * P = sqrt((p_L - p_lo)(p_R - p_lo)).  The solver starts Newton from the
 * learned guess p_lo + P exp(y) only when it is finite, admissible and its
 * |g| is no larger than the value the tangent of g there predicts at the
 * acoustic guess; otherwise from the acoustic guess ("fallback and judge").
 * It then iterates to the same tolerance, so the star state does not depend
 * on the network.
 * Parameters: 4801 FP32 values, W1 (64x8 row-major), b1 (64), W2 (64x64
 * row-major), b2 (64), w3 (64), b3 (1).  Device pointers below are in the
 * given stream's device memory; n-long arrays are SoA. */
typedef struct m2c_mlp m2c_mlp;
typedef struct m2c_train_opts {
    uint32_t struct_size;       /* = sizeof(m2c_train_opts)                      */
    int32_t epochs;             /* passes over the data set                      */
    int32_t batch;              /* minibatch size (>= 16)                        */
    float lr, lr_final;         /* Adam step size, decayed geometrically to lr_final */
    float beta1, beta2, eps;    /* Adam moments                                  */
} m2c_train_opts;
void m2c_train_opts_default(m2c_train_opts* o);
/* params: host array of 4801 values, or NULL for seeded Glorot-uniform weights. */
int m2c_mlp_create(const float* params, uint64_t seed, m2c_mlp** out);
void m2c_mlp_destroy(m2c_mlp* m);
int m2c_mlp_get_params(const m2c_mlp* m, float* params);
/* Features X8 [8][n] (and targets [n] when pstar is given) of n problems
 * in [6][n] = (rho_L,u_L,p_L,rho_R,u_R,p_R), eos [4][n] = (gamma_L,pc_L,
 * gamma_R,pc_R); device pointers. */
int m2c_mlp_features(int64_t n, const double* in, const double* eos, const double* pstar, float* X8,
                     float* target, void* hip_stream);
/* Network outputs y [n] for features X8 [8][n] (device pointers). */
int m2c_mlp_forward(const m2c_mlp* m, int64_t n, const float* X8, float* y, void* hip_stream);
/* Gradient of the mean squared error over the n samples into the host
 * array grad[4801]; *loss (nullable) = the mean squared error. */
int m2c_mlp_grad(const m2c_mlp* m, int64_t n, const float* X8, const float* t, float* grad, float* loss,
                 void* hip_stream);
/* Minibatch Adam on the GPU over the data set (device X8 [8][n], t [n]);
 * loss_per_epoch (host, nullable) receives the epoch-mean squared error. */
int m2c_mlp_train(m2c_mlp* m, int64_t n, const float* X8, const float* t, const m2c_train_opts* opts,
                  float* loss_per_epoch, void* hip_stream);
/* As m2c_riemann_solve with the learned guess (m NULL: acoustic guess);
 * *n_fallback (nullable) counts problems that started from the acoustic
 * guess: it was better, the network output was unusable, or the two states
 * differ by less than 1e-3 in pressure (relative to the smaller p + p_c) and
 * in velocity (relative to the smaller sound speed), where the acoustic
 * guess is taken without consulting the network. */
int m2c_riemann_solve_learned(const m2c_mlp* m, int64_t n, const double* in, const double* eos, double rtol,
                              int32_t maxit, double* out, int32_t* iters, int64_t* n_fallback, void* hip_stream);
/* The same solves as m2c_riemann_solve_learned (m = NULL: the acoustic
 * guess), for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.  It
 * allocates nothing and does not synchronise: the learned guesses go to a
 * library-owned device buffer of M2C_NOALLOC_MAX_PROBLEMS doubles per GPU
 * (8 MiB, held until the process ends), and the call only enqueues the
 * kernels on hip_stream.  Layouts, out and iters are those of
 * m2c_riemann_solve_learned (iters[i] = 0 and NaN out: no admissible star
 * pressure); the vacuum and acoustic-start counts are not reported.  Every
 * call on a GPU shares that GPU's buffer, so calls that overlap on one GPU
 * (other streams or threads) race.  M2C_ERR_ARG for n > M2C_NOALLOC_MAX_PROBLEMS
 * or invalid arguments, M2C_ERR_DEVICE if a launch fails. */
#define M2C_NOALLOC_MAX_PROBLEMS (1 << 20)
int m2c_riemann_solve_learned_noalloc(const m2c_mlp* m, int64_t n, const double* in, const double* eos,
                                      double rtol, int32_t maxit, double* out, int32_t* iters,
                                      void* hip_stream);
/* Use a copy of the network for every interface Riemann problem of later
 * steps (NULL: back to the acoustic guess).  With eos_general, m is a
 * network of the general-EOS features (m2c_mlp_features_eos), consulted
 * when the two materials' families take the learned start (a JWL side and
 * no Mie-Grueneisen side, as for m2c_riemann_solve_eos_learned); other
 * pairs keep the acoustic start. */
int m2c_set_guess(m2c_ctx* ctx, const m2c_mlp* m);

/* ---- level-set reinitialization (section "Level set method", eq. reinit) --
 * iters forward-Euler pseudo-time steps (dtau = 0.5 of the smallest cell
 * width over the axes with more than one cell) of
 *   d phi/d tau + S(phi_0)(|grad phi| - 1) = 0,  S = phi_0/sqrt(phi_0^2 + eps^2),
 * eps = the smallest cell width, |grad phi| by the Godunov upwind form of
 * one-sided differences.  Cells with a face neighbour on the other side of
 * the zero level set (phi >= 0 counting as the non-negative side) keep their
 * value (fixed first layer), so the interface and the material ids stay
 * where they are; band > 0 restricts the update to |phi_0| < band (narrow
 * band), band = 0 updates the whole grid.  Boundary images as in the step:
 * periodic axes wrap, transmissive and wall sides repeat the boundary cell.
 * FP64, deterministic (Jacobi iterates). */
/* On the context's current level set, between steps (stream-ordered on the
 * context's stream, which it synchronises once; uses the context's stage
 * buffer as workspace).
 * M2C_ERR_STATE before a state is set; M2C_ERR_ARG for iters < 0 or
 * band < 0. */
int m2c_reinit(m2c_ctx* ctx, int32_t iters, double band);
/* Workspace bytes m2c_reinit_field needs for an nx x ny x nz grid:
 * 16 N + 4 (1 + ceil(nx/64) ceil(ny/4) nz). */
int m2c_reinit_workspace(int32_t nx, int32_t ny, int32_t nz, int64_t* bytes);
/* On a level set phi [N] (device, x fastest, updated in place) with cell
 * widths h[3] and boundary codes bc[6] (host), work = device workspace of
 * m2c_reinit_workspace bytes; asynchronous on hip_stream.  M2C_ERR_ARG for
 * invalid sizes, widths, boundary codes (periodic must pair up), iters < 0,
 * band < 0, or null pointers when iters > 0.  Synchronises hip_stream once
 * (after the setup kernel, to size the step launches). */
int m2c_reinit_field(int32_t nx, int32_t ny, int32_t nz, const double h[3], const int32_t bc[6], double* phi,
                     void* work, int32_t iters, double band, void* hip_stream);

/* ---- general-EOS exact Riemann problems (device pointers, given stream) --
 * (materials: m2c_eos above) */

/* n problems: in = [rho_L,u_L,p_L,rho_R,u_R,p_R][n] (SoA), mat = [2][n]
 * material indices (left row, then right row) into the host table eos[nmat]
 * (1 <= nmat <= M2C_EOS_MAX); out = [p*,u*,rho*_L,rho*_R][n], iters
 * (nullable) = star-pressure Newton steps per problem (negative: bisection
 * fallback; 0: no star state or an inadmissible input, out = NaN).
 * Shocks: Hugoniot energy relation solved for the specific volume.
 * Rarefactions: the isentrope in closed form for NASG, JWL (its Riemann
 * invariant by Gauss-Legendre quadrature) and the Mie-Grueneisen tension and
 * cutoff branches; on the Mie-Grueneisen compression branch integrated with
 * classical RK4 over y = ln(p - floor) at steps of at most ds (0: 0.01; else
 * in [1e-3, 0.5]); the error of the RK4 part
 * falls as ds^4 (at most about 2e-10 of the sound speed in u* at 0.01 on the
 * materials of the tests).
 * FP64 throughout.  rtol: Newton stop |dp| <= rtol (p - floor) on the closer
 * side.  The problems are grouped by material pair on the device (a
 * workspace of about 4n bytes that the call allocates and frees); a problem
 * whose right side has the lower EOS family is solved in its mirror image,
 * so a problem and its reflection (sides swapped, velocities negated) give
 * the same p* bit for bit.  The call synchronises hip_stream before it
 * returns.  Returns M2C_ERR_RIEMANN if any problem had no star state,
 * M2C_ERR_ARG for invalid arguments or EOS parameters, M2C_ERR_NOMEM if the
 * workspace cannot be allocated. */
int m2c_riemann_solve_eos(int64_t n, const double* in, const int32_t* mat, int32_t nmat, const m2c_eos* eos,
                          double rtol, int32_t maxit, double ds, double* out, int32_t* iters, void* hip_stream);
/* Learned start for the general-EOS solve (the acceleration of the exact
 * Riemann solves that section "Spatial discretization of governing
 * equations" calls for; it matters most here, where each outer Newton step
 * integrates wave curves).  The network of m2c_mlp (8 -> 64 -> 64 -> 1)
 * with these features of a problem, taken in the orientation it is solved
 * in (lower family on the left):
 *   x0 = ln(rho_L/rho_R)/2, x1 = (u_R - u_L)/U, x2 = ln(a_L/a_R)/2,
 *   x3 = ln(rho_L c_L^2/a_L), x4 = ln(rho_R c_R^2/a_R),
 *   x5 = ln((p_ac - p_lo)/P) with p_ac the acoustic start,
 *   x6, x7 = family - 1 (M2C_EOS_*) of the left and right side,
 * p_lo the higher of the two pressure floors, a_K = p_K - p_lo,
 * P = sqrt(a_L a_R), U = sqrt(P / sqrt(rho_L rho_R)); the target is
 * y = ln((p* - p_lo)/P).  X8 [8][n], target [n] (nullable; NaN where p* is
 * not above p_lo or the problem is inadmissible, with zero features);
 * pstar [n] (nullable): the star pressures the targets come from.  Device
 * pointers; asynchronous on hip_stream. */
int m2c_mlp_features_eos(int64_t n, const double* in, const int32_t* mat, int32_t nmat, const m2c_eos* eos,
                         const double* pstar, float* X8, float* target, void* hip_stream);
/* As m2c_riemann_solve_eos with the learned start of network m (NULL: the
 * acoustic start, the same solves as m2c_riemann_solve_eos).  The network
 * is consulted for problems with a JWL side and no Mie-Grueneisen side
 * (where an outer step saved pays for it; with NASG on both sides a step
 * is cheaper than the network, and with a Mie-Grueneisen side the cost is
 * the length of the isentrope walks, not the number of outer steps), and
 * not at all in a set that also holds Mie-Grueneisen problems; problems
 * whose pressures and velocities agree to 1e-3 (relative to the smaller
 * p_K - p_lo and sound speed) start from the acoustic guess as well.  A learned start is evaluated (F and F' of the outer iteration,
 * which serve as its first Newton step when it is kept) and kept unless the
 * tangent there predicts a smaller |F| at the acoustic start; the iteration
 * then runs to the same tolerance, so the star state does not depend on the
 * network beyond rtol.  *n_fallback (nullable): problems with a star state
 * that started from the acoustic guess.  Return codes as for
 * m2c_riemann_solve_eos. */
int m2c_riemann_solve_eos_learned(const m2c_mlp* m, int64_t n, const double* in, const int32_t* mat, int32_t nmat,
                                  const m2c_eos* eos, double rtol, int32_t maxit, double ds, double* out,
                                  int32_t* iters, int64_t* n_fallback, void* hip_stream);
/* Pressure and sound speed of n states (rho, e) of materials mat[n] of the
 * table eos[nmat] (device arrays; p, c = NaN where c^2 <= 0 or the index is
 * out of range). */
int m2c_eos_eval(int64_t n, const double* rho, const double* e, const int32_t* mat, int32_t nmat,
                 const m2c_eos* eos, double* p, double* c, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* M2C_H */
