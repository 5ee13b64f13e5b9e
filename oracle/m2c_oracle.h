/*
 * m2c_oracle.h -- plain FP64 CPU oracle of the two-material finite-volume
 * time step (TEST INFRASTRUCTURE ONLY).
 *
 * This is the slow, obviously-correct reference that the GPU library is
 * checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the product path never does.  It shares no
 * code, header, table or constant with the GPU library.
 *
 * What it computes (one time step, paper sections "Spatial discretization of
 * governing equations", "Time integration", "Level set method" and the step
 * outline in "Code structure"):
 *   cell-centred finite volumes on a uniform Cartesian grid (eq.
 *   NS_discretized, inviscid, no source); primitive-variable MUSCL with the MC
 *   limiter (appendix "Slope limiters", eqs. theta/AB); HLLC at faces inside
 *   one material (appendix "HLLC flux"); FIVER at faces whose two cells hold
 *   different materials: an exact two-material Riemann problem (eq.
 *   1DRiemannProblem) whose star states feed one one-sided HLLC flux per side;
 *   level-set advection (eq. levelset) with third-order upwind differences;
 *   TVD Runge-Kutta in time with a CFL-based dt; and the phase update for
 *   cells whose level-set sign flipped.  Stiffened gas per material:
 *   p = (gamma-1) rho e - gamma p_c (eq. NASG_EOS with b = e_c = 0), or a
 *   general EOS per material (NASG, Mie-Grueneisen, JWL) whose interface
 *   Riemann problems are solved by a caller-given function.
 *
 * Arrays are structure-of-arrays, x fastest: cell (i,j,k) is at
 * i + nx*(j + ny*k).  Material 1 occupies phi < 0.
 */
#ifndef M2C_ORACLE_H
#define M2C_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_OK = 0, ORA_ERR_ARG = -1, ORA_ERR_NONPHYSICAL = -2, ORA_ERR_RIEMANN = -3,
       ORA_ERR_NOMEM = -7 };
enum { ORA_BC_TRANSMISSIVE = 0, ORA_BC_WALL = 1, ORA_BC_PERIODIC = 2 };

/* General EOS of one material: family and parameters in the order
 *   NASG (gamma, p_c, b, e_c), eq. NASG_EOS;
 *   MG   (rho_0, c_0, Gamma_0, s, e_0, eta_min), appendix on equations of state;
 *   JWL  (omega, A_1, A_2, R_1, R_2, rho_0), eq. JWL_EOS. */
enum { ORA_EOS_NASG = 0, ORA_EOS_MG = 1, ORA_EOS_JWL = 2 };
typedef struct {
    int32_t family;
    int32_t reserved;
    double prm[7];
} ora_eos;
/* Star state (p*, u*, rho*_L, rho*_R) of the two-material Riemann problem
 * in = (rho_L, u_L, p_L, rho_R, u_R, p_R) between materials ml and mr. */
typedef int32_t (*ora_riemann_fn)(int32_t ml, int32_t mr, const double* in, double* out);

typedef struct {
    int32_t nx, ny, nz;
    double lo[3], hi[3];
    double gamma[2], pc[2];   /* material 0 (phi >= 0), material 1 (phi < 0) */
    int32_t bc[6];            /* -x,+x,-y,+y,-z,+z */
    double alpha;             /* MC limiter parameter (paper default 1.2)       */
    int32_t rk_order;         /* 1 forward Euler, 2 TVD-RK2, 3 TVD-RK3            */
    double cfl, dt_fixed;     /* dt_fixed > 0 overrides the CFL rule             */
    double rtol;              /* Newton stopping tolerance on p*                 */
    int32_t maxit;            /* Newton iterations before bisection              */
    int32_t limiter;          /* ORA_LIM_MC, ORA_LIM_VA, ORA_LIM_VA_MOD            */
    int32_t limiter_k;        /* Van Albada exponent k                           */
    int32_t flux;             /* ORA_FLUX_HLLC, ORA_FLUX_LLF                     */
    double ls_band;           /* > 0: level set advanced only where |phi| < band */
    /* General equations of state (section "Equations of state"): with
     * eos_general set, material m follows eos[m] instead of the stiffened
     * gas (gamma[m], pc[m]), and interface faces take their star states from
     * riemann (which returns ORA_OK, or an error code when the problem has
     * no star state). */
    int32_t eos_general;
    ora_eos eos[2];
    ora_riemann_fn riemann;
} ora_cfg;

enum { ORA_LIM_MC = 0, ORA_LIM_VA = 1, ORA_LIM_VA_MOD = 2 };
enum { ORA_FLUX_HLLC = 0, ORA_FLUX_LLF = 1 };

typedef struct {
    int64_t steps;
    double t, dt_last;
    int64_t iface_faces_last;   /* interface faces in the last step            */
    int64_t newton_iters;       /* summed over all solves                      */
    int64_t riemann_solves;
    int64_t bisection_fallbacks;
    int64_t flips, orphans;     /* phase update counters (all steps)           */
    int64_t err_cell;           /* first failing cell (or -1)                  */
} ora_stats;

typedef struct ora_sim ora_sim;

ora_sim* ora_create(const ora_cfg* cfg);
void     ora_destroy(ora_sim* s);
/* prim6 = [rho,u,v,w,p,phi][N]; material ids follow from phi. */
int      ora_set_prim(ora_sim* s, const double* prim6);
int      ora_get_prim(const ora_sim* s, double* prim6, uint8_t* chi /* nullable */);
/* w6 = [rho, rho u, rho v, rho w, rho E, phi][N] (exact checkpoint). */
int      ora_set_cons(ora_sim* s, const double* w6);
int      ora_get_cons(const ora_sim* s, double* w6);
int      ora_step(ora_sim* s, int32_t nsteps);
/* Same as ora_step but with dt imposed for every step (for sampled checks). */
int      ora_step_dt(ora_sim* s, int32_t nsteps, double dt);
double   ora_dt(const ora_sim* s);
void     ora_get_stats(const ora_sim* s, ora_stats* st);
/* Interface faces of the current material field, ascending face ids
 * f = 3*c + d (face between cell c and its +d neighbour).  Returns count;
 * writes at most cap ids. */
int64_t  ora_interface_faces(const ora_sim* s, int32_t* out, int64_t cap);
/* Threads the loops use: omp_get_max_threads() in the OpenMP build, else 1. */
int32_t  ora_num_threads(void);

/* ---- point functions ---------------------------------------------------- */
/* Stiffened-gas primitive -> conservative and back (one cell). */
void ora_prim_to_cons(const double* q5, double gamma, double pc, double* w5);
void ora_cons_to_prim(const double* w5, double gamma, double pc, double* q5);
/* Speed of sound of a stiffened-gas state. */
double ora_sound_speed(double rho, double p, double gamma, double pc);
/* MC-limited slope from the backward and forward differences. */
double ora_mc_slope(double dminus, double dplus, double alpha);
/* Van Albada slope (modified: clamped at 0) with exponent k. */
double ora_va_slope(double dminus, double dplus, int32_t k, int32_t modified);
/* HLLC flux along +x in the face frame: q = (rho, u_n, v_t1, v_t2, p). */
void ora_hllc(const double* qL, const double* qR, double gamma, double pc, double* F5);
/* General EOS point functions: p(rho, e), e(rho, p), c^2(rho, p) and the
 * lowest admissible pressure of one material. */
double ora_eos_p(const ora_eos* m, double rho, double e);
double ora_eos_e(const ora_eos* m, double rho, double p);
double ora_eos_c2(const ora_eos* m, double rho, double p);
double ora_eos_floor(const ora_eos* m);
/* Local Lax-Friedrichs flux, same conventions. */
void ora_llf(const double* qL, const double* qR, double gamma, double pc, double* F5);
/* Exact two-material stiffened-gas Riemann problem.
 * in = (rho_L, u_L, p_L, rho_R, u_R, p_R), eos = (gamma_L, pc_L, gamma_R, pc_R)
 * out = (p*, u*, rho*_L, rho*_R); returns ORA_OK or ORA_ERR_RIEMANN (vacuum). */
int  ora_riemann(const double* in, const double* eos, double rtol, int32_t maxit,
                 double* out, int32_t* iters);
/* ora_riemann over n problems stored row by row; returns the number of
 * problems without an admissible star pressure (their out = NaN). */
int64_t ora_riemann_many(int64_t n, const double* in, const double* eos, double rtol, int32_t maxit,
                         double* out, int32_t* iters);
/* Third-order upwind-biased derivative of phi at the centre of a 5-point
 * stencil f[0..4] = phi_{i-2..i+2} for advection speed v. */
double ora_ls_derivative(const double* f, double v, double h);

#ifdef __cplusplus
}
#endif
#endif
