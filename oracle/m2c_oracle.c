/*
 * m2c_oracle.c -- plain FP64 CPU oracle of the two-material finite-volume time
 * step.  TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and
 * the benchmark's CPU-baseline leg; never by the product path.
 *
 * Written for clarity, not speed: whole-field loops, padded ghost arrays,
 * one face at a time.  Every function names the passage of the paper it
 * follows.  Where the paper is silent the reading is stated in a comment.
 *
 * Parity pins: every part of this file is pinned by tests that do not retype
 * its formulas (closed forms, conservation, invariants, exact Riemann
 * solutions from an independent bisection solver, a 30-digit hand-written
 * forward-Euler step and single-face fluxes).  The zero-slope rule next to an
 * interface and the phase-update rule are readings of under-specified steps:
 * the code is pinned to the readings as stated, the readings themselves are
 * choices the paper does not fix.
 *
 * Threads: built with -fopenmp (the all-core CPU baseline), the cell and
 * line loops run in parallel.  Every cell's arithmetic and its order are the
 * same as in the serial build (sums over a cell's faces stay in axis order,
 * the time step is a maximum, error cells are the first in loop order), so
 * both builds give bit-identical results; only the storage order of the
 * interface star records differs, and they are read through the face map.
 */
#include "m2c_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the oracle's loops use (1 in the serial build). */
int32_t ora_num_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Stiffened-gas EOS: eq. NASG_EOS with b = 0 and e_c = 0 (section
 * "Thermodynamic equation of state"), p = (gamma-1) rho e - gamma p_c, and
 * the total energy E = e + |V|^2/2 of section "Input and output".          */

void ora_prim_to_cons(const double* q, double gamma, double pc, double* w)
{
    double rho = q[0], u = q[1], v = q[2], ww = q[3], p = q[4];
    double e = (p + gamma * pc) / ((gamma - 1.0) * rho);
    w[0] = rho;
    w[1] = rho * u;
    w[2] = rho * v;
    w[3] = rho * ww;
    w[4] = rho * (e + 0.5 * (u * u + v * v + ww * ww));
}

void ora_cons_to_prim(const double* w, double gamma, double pc, double* q)
{
    double rho = w[0];
    double u = w[1] / rho, v = w[2] / rho, ww = w[3] / rho;
    double e = w[4] / rho - 0.5 * (u * u + v * v + ww * ww);
    q[0] = rho;
    q[1] = u;
    q[2] = v;
    q[3] = ww;
    q[4] = (gamma - 1.0) * rho * e - gamma * pc;
}

/* Speed of sound c^2 = p_rho + Gamma p / rho (appendix "Flux Jacobians"),
 * which for the stiffened gas is gamma (p + p_c) / rho. */
static double sound_speed(double rho, double p, double gamma, double pc)
{
    return sqrt(gamma * (p + pc) / rho);
}

double ora_sound_speed(double rho, double p, double gamma, double pc)
{
    return sound_speed(rho, p, gamma, pc);
}

/* ------------------------------------------------------------------------ */
/* General equations of state (section "Equations of state", eq. eos_all):
 * p = p(rho, e) per family, e(rho, p) its inverse in e (each family is
 * affine in e), and c^2 = dp/drho|_e + p dp/de|_rho / rho^2.
 *   NASG (eq. NASG_EOS): p = (gamma - 1) rho (e - e_c) / (1 - b rho) - gamma p_c;
 *   Mie-Grueneisen (appendix on equations of state): p = p_R(eta) +
 *     rho_0 Gamma_0 (e - e_R(eta)), eta = 1 - rho_0/rho, with the reference
 *     curves of compression (eta >= 0, where e_R takes the Hugoniot pressure
 *     of the reference state to be p_R), small tension (eta_min <= eta < 0)
 *     and the tensile cutoff below eta_min;
 *   JWL (eq. JWL_EOS, both exponentials decaying):
 *     p = omega rho e + sum_i A_i (1 - omega rho / (R_i rho_0)) exp(-R_i rho_0 / rho).
 * Lowest admissible pressure: -p_c (NASG), rho_0 c_0^2 eta_min (MG), 0 (JWL). */

/* MG reference curves p_R, e_R and their eta-derivatives. */
static void mg_reference(const double* a, double eta, double* pR, double* eR, double* dpR, double* deR)
{
    double r0 = a[0], K0 = a[0] * a[1] * a[1], s = a[3], e0 = a[4], em = a[5];
    if (eta >= 0.0) {
        double d = 1.0 - s * eta;
        *pR = K0 * eta / (d * d);
        *dpR = K0 * (1.0 + s * eta) / (d * d * d);
        *eR = *pR * eta / (2.0 * r0) + e0;
        *deR = (*dpR * eta + *pR) / (2.0 * r0);
    } else if (eta >= em) {
        *pR = K0 * eta;
        *dpR = K0;
        *eR = K0 * eta * eta / (2.0 * r0) + e0;
        *deR = K0 * eta / r0;
    } else {
        double pmin = K0 * em;
        *pR = pmin;
        *dpR = 0.0;
        *eR = K0 * em * em / (2.0 * r0) + e0 + pmin / r0 * (eta - em);
        *deR = pmin / r0;
    }
}

/* JWL: T(rho) = sum_i A_i (1 - omega rho/(R_i rho_0)) exp(-R_i rho_0/rho) and dT/drho. */
static void jwl_exp_terms(const double* a, double rho, double* T, double* dT)
{
    double w = a[0], r0 = a[5];
    *T = 0.0;
    *dT = 0.0;
    for (int i = 0; i < 2; ++i) {
        double A = a[1 + i], R = a[3 + i];
        double x = exp(-R * r0 / rho);
        double f = 1.0 - w * rho / (R * r0);
        *T += A * f * x;
        *dT += A * (-w / (R * r0) * x + f * x * R * r0 / (rho * rho));
    }
}

double ora_eos_p(const ora_eos* m, double rho, double e)
{
    const double* a = m->prm;
    if (m->family == ORA_EOS_NASG)
        return (a[0] - 1.0) * rho * (e - a[3]) / (1.0 - a[2] * rho) - a[0] * a[1];
    if (m->family == ORA_EOS_MG) {
        double pR, eR, dpR, deR;
        mg_reference(a, 1.0 - a[0] / rho, &pR, &eR, &dpR, &deR);
        return pR + a[0] * a[2] * (e - eR);
    }
    double T, dT;
    jwl_exp_terms(a, rho, &T, &dT);
    return a[0] * rho * e + T;
}

double ora_eos_e(const ora_eos* m, double rho, double p)
{
    const double* a = m->prm;
    if (m->family == ORA_EOS_NASG)
        return (p + a[0] * a[1]) * (1.0 - a[2] * rho) / ((a[0] - 1.0) * rho) + a[3];
    if (m->family == ORA_EOS_MG) {
        double pR, eR, dpR, deR;
        mg_reference(a, 1.0 - a[0] / rho, &pR, &eR, &dpR, &deR);
        return eR + (p - pR) / (a[0] * a[2]);
    }
    double T, dT;
    jwl_exp_terms(a, rho, &T, &dT);
    return (p - T) / (a[0] * rho);
}

double ora_eos_c2(const ora_eos* m, double rho, double p)
{
    const double* a = m->prm;
    double e = ora_eos_e(m, rho, p), p_rho, p_e;
    if (m->family == ORA_EOS_NASG) {
        double d = 1.0 - a[2] * rho;
        p_rho = (a[0] - 1.0) * (e - a[3]) / (d * d);
        p_e = (a[0] - 1.0) * rho / d;
    } else if (m->family == ORA_EOS_MG) {
        double pR, eR, dpR, deR;
        mg_reference(a, 1.0 - a[0] / rho, &pR, &eR, &dpR, &deR);
        p_rho = (dpR - a[0] * a[2] * deR) * a[0] / (rho * rho);
        p_e = a[0] * a[2];
    } else {
        double T, dT;
        jwl_exp_terms(a, rho, &T, &dT);
        p_rho = a[0] * e + dT;
        p_e = a[0] * rho;
    }
    return p_rho + p * p_e / (rho * rho);
}

double ora_eos_floor(const ora_eos* m)
{
    const double* a = m->prm;
    if (m->family == ORA_EOS_NASG) return -a[1];
    if (m->family == ORA_EOS_MG) return a[0] * a[1] * a[1] * a[5];
    return 0.0;
}

/* ------------------------------------------------------------------------ */
/* MC limiter, appendix "Slope limiters", eqs. theta and AB on a uniform
 * grid: theta = (w_i - w_{i-1}) / (w_{i+1} - w_i), A = B = 1,
 * phi = max(0, min(alpha theta, B (theta + 1)/(A + 1), alpha)), and the
 * limited slope is phi(theta) (w_{i+1} - w_i).  When w_{i+1} = w_i the
 * slope is 0 (phi is bounded by alpha).                                    */
double ora_mc_slope(double dminus, double dplus, double alpha)
{
    if (dplus == 0.0) return 0.0;
    const double h = 1.0;                       /* uniform widths             */
    const double A = (h + h) / (h + h);
    const double B = 2.0 * h / (h + h);
    double theta = dminus / dplus;
    double lim = fmin(alpha * theta, B / (A + 1.0) * (theta + 1.0));
    lim = fmin(lim, alpha);
    lim = fmax(0.0, lim);
    return lim * dplus;
}

/* Van Albada limiter, appendix "Slope limiters", eq. vanalbada on a uniform
 * grid (A = B = 1): phi(theta) = B (theta^k + theta) / (theta^k + A); the
 * modified limiter (eq. vanalbada_mod) sets phi = 0 where it is negative.
 * The limited slope is phi(theta) (w_{i+1} - w_i), 0 when w_{i+1} = w_i;
 * where theta^k overflows, phi takes its limit B.                         */
double ora_va_slope(double dminus, double dplus, int32_t k, int32_t modified)
{
    if (dplus == 0.0) return 0.0;
    const double h = 1.0;
    const double A = (h + h) / (h + h);
    const double B = 2.0 * h / (h + h);
    double theta = dminus / dplus;
    double tk = 1.0;
    for (int32_t e = 0; e < k; ++e) tk *= theta;
    double lim = isfinite(tk) ? B * (tk + theta) / (tk + A) : B;
    if (modified && lim < 0.0) lim = 0.0;
    return lim * dplus;
}

static double limited_slope(const ora_cfg* c, double dminus, double dplus)
{
    if (c->limiter == ORA_LIM_MC) return ora_mc_slope(dminus, dplus, c->alpha);
    return ora_va_slope(dminus, dplus, c->limiter_k, c->limiter == ORA_LIM_VA_MOD);
}

/* ------------------------------------------------------------------------ */
/* HLLC, appendix "HLLC flux".  States in the face frame: q = (rho, u, v, w, p)
 * with u the component along n_ij.  Davis wave-speed estimates S_ij, S_ji
 * and the contact speed S_* as printed.  The star energy is not written in
 * the paper; it is the one of its cited source (Toro):
 * E*_K = E_K + (S_* - u_K)(S_* + p_K / (rho_K (S_K - u_K))).               */
static void euler_flux(const double* q, double E, double* F)
{
    double rho = q[0], u = q[1], p = q[4];
    F[0] = rho * u;
    F[1] = rho * u * u + p;
    F[2] = rho * u * q[2];
    F[3] = rho * u * q[3];
    F[4] = (rho * E + p) * u;
}

static double specific_total_energy(const double* q, double gamma, double pc)
{
    double e = (q[4] + gamma * pc) / ((gamma - 1.0) * q[0]);
    return e + 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
}

/* HLLC with the sound speeds and specific total energies of the two
 * states given (they are all the flux needs of the EOS). */
static void hllc_ce(const double* qL, const double* qR, double cL, double cR, double EL, double ER, double* F)
{
    double rL = qL[0], uL = qL[1], pL = qL[4];
    double rR = qR[0], uR = qR[1], pR = qR[4];

    double SL = fmin(uL - cL, uR - cR);
    double SR = fmax(uL + cL, uR + cR);
    double Ss = (pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR)) /
                (rL * (SL - uL) - rR * (SR - uR));

    if (0.0 <= SL) {
        euler_flux(qL, EL, F);
    } else if (0.0 <= Ss) {
        double FL[5], UL[5], Us[5];
        euler_flux(qL, EL, FL);
        UL[0] = rL; UL[1] = rL * uL; UL[2] = rL * qL[2]; UL[3] = rL * qL[3]; UL[4] = rL * EL;
        double fac = rL * (SL - uL) / (SL - Ss);
        Us[0] = fac;
        Us[1] = fac * Ss;
        Us[2] = fac * qL[2];
        Us[3] = fac * qL[3];
        Us[4] = fac * (EL + (Ss - uL) * (Ss + pL / (rL * (SL - uL))));
        for (int v = 0; v < 5; ++v) F[v] = FL[v] + SL * (Us[v] - UL[v]);
    } else if (0.0 <= SR) {
        double FR[5], UR[5], Us[5];
        euler_flux(qR, ER, FR);
        UR[0] = rR; UR[1] = rR * uR; UR[2] = rR * qR[2]; UR[3] = rR * qR[3]; UR[4] = rR * ER;
        double fac = rR * (SR - uR) / (SR - Ss);
        Us[0] = fac;
        Us[1] = fac * Ss;
        Us[2] = fac * qR[2];
        Us[3] = fac * qR[3];
        Us[4] = fac * (ER + (Ss - uR) * (Ss + pR / (rR * (SR - uR))));
        for (int v = 0; v < 5; ++v) F[v] = FR[v] + SR * (Us[v] - UR[v]);
    } else {
        euler_flux(qR, ER, F);
    }
}

void ora_hllc(const double* qL, const double* qR, double gamma, double pc, double* F)
{
    double cL = sound_speed(qL[0], qL[4], gamma, pc);
    double cR = sound_speed(qR[0], qR[4], gamma, pc);
    double EL = specific_total_energy(qL, gamma, pc);
    double ER = specific_total_energy(qR, gamma, pc);
    hllc_ce(qL, qR, cL, cR, EL, ER, F);
}

/* ------------------------------------------------------------------------ */
/* Local Lax-Friedrichs, appendix "Local Lax-Friedrichs flux" (eq.
 * Lax-Friedrichs): the mean of the two physical fluxes minus half the
 * fastest wave speed max(|u_L| + c_L, |u_R| + c_R) times the jump of the
 * conservative state.                                                     */
static void llf_ce(const double* qL, const double* qR, double cL, double cR, double EL, double ER, double* F)
{
    double FL[5], FR[5], UL[5], UR[5];
    euler_flux(qL, EL, FL);
    euler_flux(qR, ER, FR);
    UL[0] = qL[0]; UL[1] = qL[0] * qL[1]; UL[2] = qL[0] * qL[2]; UL[3] = qL[0] * qL[3]; UL[4] = qL[0] * EL;
    UR[0] = qR[0]; UR[1] = qR[0] * qR[1]; UR[2] = qR[0] * qR[2]; UR[3] = qR[0] * qR[3]; UR[4] = qR[0] * ER;
    double lmax = fmax(fabs(qL[1]) + cL, fabs(qR[1]) + cR);
    for (int v = 0; v < 5; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * lmax * (UR[v] - UL[v]);
}

void ora_llf(const double* qL, const double* qR, double gamma, double pc, double* F)
{
    llf_ce(qL, qR, sound_speed(qL[0], qL[4], gamma, pc), sound_speed(qR[0], qR[4], gamma, pc),
           specific_total_energy(qL, gamma, pc), specific_total_energy(qR, gamma, pc), F);
}

/* The numerical flux of the configuration (section "Spatial discretization
 * of governing equations": one flux function Phi for every face, the
 * one-sided FIVER fluxes included).                                       */
static void num_flux(const ora_cfg* c, const double* qL, const double* qR, int m, double* F)
{
    if (!c->eos_general) {
        if (c->flux == ORA_FLUX_LLF) ora_llf(qL, qR, c->gamma[m], c->pc[m], F);
        else ora_hllc(qL, qR, c->gamma[m], c->pc[m], F);
        return;
    }
    const ora_eos* e = &c->eos[m];
    double cL = sqrt(ora_eos_c2(e, qL[0], qL[4])), cR = sqrt(ora_eos_c2(e, qR[0], qR[4]));
    double EL = ora_eos_e(e, qL[0], qL[4]) + 0.5 * (qL[1] * qL[1] + qL[2] * qL[2] + qL[3] * qL[3]);
    double ER = ora_eos_e(e, qR[0], qR[4]) + 0.5 * (qR[1] * qR[1] + qR[2] * qR[2] + qR[3] * qR[3]);
    if (c->flux == ORA_FLUX_LLF) llf_ce(qL, qR, cL, cR, EL, ER, F);
    else hllc_ce(qL, qR, cL, cR, EL, ER, F);
}

/* Conservative <-> primitive and sound speed of material m of the
 * configuration (stiffened gas or general EOS). */
static void mat_cons_to_prim(const ora_cfg* c, int m, const double* w, double* q)
{
    if (!c->eos_general) { ora_cons_to_prim(w, c->gamma[m], c->pc[m], q); return; }
    double rho = w[0];
    double u = w[1] / rho, v = w[2] / rho, ww = w[3] / rho;
    double e = w[4] / rho - 0.5 * (u * u + v * v + ww * ww);
    q[0] = rho; q[1] = u; q[2] = v; q[3] = ww;
    q[4] = ora_eos_p(&c->eos[m], rho, e);
}

static void mat_prim_to_cons(const ora_cfg* c, int m, const double* q, double* w)
{
    if (!c->eos_general) { ora_prim_to_cons(q, c->gamma[m], c->pc[m], w); return; }
    double rho = q[0], u = q[1], v = q[2], ww = q[3];
    double e = ora_eos_e(&c->eos[m], rho, q[4]);
    w[0] = rho; w[1] = rho * u; w[2] = rho * v; w[3] = rho * ww;
    w[4] = rho * (e + 0.5 * (u * u + v * v + ww * ww));
}

static double mat_sound_speed(const ora_cfg* c, int m, double rho, double p)
{
    if (!c->eos_general) return sound_speed(rho, p, c->gamma[m], c->pc[m]);
    return sqrt(ora_eos_c2(&c->eos[m], rho, p));
}

/* ------------------------------------------------------------------------ */
/* Exact two-material Riemann problem (eq. 1DRiemannProblem) for stiffened
 * gases.  The paper cites its solver without stating it; for a stiffened gas
 * the shifted pressure pbar = p + p_c obeys the ideal-gas shock and
 * rarefaction relations, so each side K contributes the classical wave
 * function f_K(p) and the star pressure is the root of
 * g(p) = f_L(p) + f_R(p) + u_R - u_L on p > p_lo = -min(pc_L, pc_R).
 * Newton from the acoustic (linearised) guess, with a step that would leave
 * the admissible range replaced by halving the distance to p_lo; bisection
 * if Newton has not met the tolerance after maxit steps.                   */
typedef struct {
    double rho, u, p, gamma, pc;
    double pbar, c, A, B, mu;
} ora_side;

static void side_init(ora_side* s, double rho, double u, double p, double gamma, double pc)
{
    s->rho = rho; s->u = u; s->p = p; s->gamma = gamma; s->pc = pc;
    s->pbar = p + pc;
    s->c = sqrt(gamma * s->pbar / rho);
    s->mu = (gamma - 1.0) / (gamma + 1.0);
    s->A = 2.0 / ((gamma + 1.0) * rho);
    s->B = s->mu * s->pbar;
}

/* Wave function of side K at trial pressure p, and its derivative. */
static double wave_f(const ora_side* s, double p, double* dfdp)
{
    double pb = p + s->pc;
    if (p > s->p) {                                    /* shock            */
        double q = sqrt(s->A / (pb + s->B));
        if (dfdp) *dfdp = q * (1.0 - (p - s->p) / (2.0 * (pb + s->B)));
        return (p - s->p) * q;
    } else {                                           /* rarefaction      */
        double g = s->gamma;
        double r = pb / s->pbar;
        if (dfdp) *dfdp = pow(r, -(g + 1.0) / (2.0 * g)) / (s->rho * s->c);
        return 2.0 * s->c / (g - 1.0) * (pow(r, (g - 1.0) / (2.0 * g)) - 1.0);
    }
}

static double star_density(const ora_side* s, double pstar)
{
    double ratio = (pstar + s->pc) / s->pbar;
    if (pstar > s->p)                                  /* shock Hugoniot   */
        return s->rho * (ratio + s->mu) / (s->mu * ratio + 1.0);
    return s->rho * pow(ratio, 1.0 / s->gamma);        /* isentrope        */
}

int ora_riemann(const double* in, const double* eos, double rtol, int32_t maxit,
                double* out, int32_t* iters)
{
    ora_side L, R;
    side_init(&L, in[0], in[1], in[2], eos[0], eos[1]);
    side_init(&R, in[3], in[4], in[5], eos[2], eos[3]);
    double du = R.u - L.u;
    double plo = -fmin(L.pc, R.pc);
    if (iters) *iters = 0;

    /* No admissible root (a vacuum would open) when g(p_lo) >= 0. */
    double glo = wave_f(&L, plo, NULL) + wave_f(&R, plo, NULL) + du;
    if (!(glo < 0.0)) return ORA_ERR_RIEMANN;

    double ZL = L.rho * L.c, ZR = R.rho * R.c;
    double pac = (ZR * L.p + ZL * R.p + ZL * ZR * (L.u - R.u)) / (ZL + ZR);
    double p = fmax(pac, plo + 1e-6 * fmin(L.p - plo, R.p - plo));

    int converged = 0, it = 0;
    while (it < maxit) {
        double dL, dR;
        double g = wave_f(&L, p, &dL) + wave_f(&R, p, &dR) + du;
        double pn = p - g / (dL + dR);
        if (pn <= plo) pn = plo + 0.5 * (p - plo);
        ++it;
        converged = fabs(pn - p) <= rtol * (pn - plo);
        p = pn;
        if (converged) break;
    }
    if (!converged) {
        double a = plo, b = fmax(L.p, R.p);
        while (wave_f(&L, b, NULL) + wave_f(&R, b, NULL) + du < 0.0) b = plo + 2.0 * (b - plo);
        for (int k = 0; k < 400 && (b - a) > rtol * (b - plo); ++k) {
            double m = 0.5 * (a + b);
            if (wave_f(&L, m, NULL) + wave_f(&R, m, NULL) + du < 0.0) a = m; else b = m;
        }
        p = 0.5 * (a + b);
        it = -it;                   /* negative count flags the fallback */
    }
    if (iters) *iters = it;
    out[0] = p;
    out[1] = 0.5 * (L.u + R.u) + 0.5 * (wave_f(&R, p, NULL) - wave_f(&L, p, NULL));
    out[2] = star_density(&L, p);
    out[3] = star_density(&R, p);
    return ORA_OK;
}

/* The same for n problems stored row by row (in[n][6], eos[n][4],
 * out[n][4], iters[n]); returns the number without an admissible root. */
int64_t ora_riemann_many(int64_t n, const double* in, const double* eos, double rtol, int32_t maxit,
                         double* out, int32_t* iters)
{
    int64_t bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t it = 0;
        if (ora_riemann(in + 6 * i, eos + 4 * i, rtol, maxit, out + 4 * i, &it) != ORA_OK) {
            ++bad;
            for (int v = 0; v < 4; ++v) out[4 * i + v] = NAN;
            it = 0;
        }
        if (iters) iters[i] = it;
    }
    return bad;
}

/* ------------------------------------------------------------------------ */
/* Level-set derivative, section "Level set method": finite differences with
 * a third-order upwind scheme.  Reading: the one-sided four-point stencils
 * biased to the upwind side, exact for cubics:
 *   v > 0: (2 f_{i+1} + 3 f_i - 6 f_{i-1} + f_{i-2}) / (6 h)
 *   v < 0: (-f_{i+2} + 6 f_{i+1} - 3 f_i - 2 f_{i-1}) / (6 h)             */
double ora_ls_derivative(const double* f, double v, double h)
{
    if (v > 0.0) return (2.0 * f[3] + 3.0 * f[2] - 6.0 * f[1] + f[0]) / (6.0 * h);
    if (v < 0.0) return (-f[4] + 6.0 * f[3] - 3.0 * f[2] - 2.0 * f[1]) / (6.0 * h);
    return 0.0;
}

/* ------------------------------------------------------------------------ */
/* Grid state.                                                              */
typedef struct {
    double pstar, ustar, rhoL, rhoR;
    double VL[3], VR[3];          /* cell velocities of the lower/upper side */
} ora_star;

struct ora_sim {
    ora_cfg c;
    int64_t N;
    double h[3];
    int act[3];                   /* axis has more than one cell            */
    int g[3], o[3];               /* padded extents and ghost offsets       */
    int64_t PN;
    double* W[5];
    double* phi;
    uint8_t* chi;
    /* work arrays */
    double* P[6];                 /* padded primitives + phi                */
    uint8_t* X;                   /* padded material ids                    */
    int32_t* slot;                /* 3N face -> star record (or -1)         */
    ora_star* rec;
    int64_t nrec, caprec;
    ora_stats st;
};

static int64_t pidx(const ora_sim* s, int i, int j, int k)
{
    return (int64_t)(i + s->o[0]) + (int64_t)s->g[0] * ((j + s->o[1]) + (int64_t)s->g[1] * (k + s->o[2]));
}

ora_sim* ora_create(const ora_cfg* cfg)
{
    if (!cfg || cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1) return NULL;
    if (cfg->eos_general) {
        if (!cfg->riemann) return NULL;
        for (int m = 0; m < 2; ++m)
            if (cfg->eos[m].family < ORA_EOS_NASG || cfg->eos[m].family > ORA_EOS_JWL) return NULL;
    }
    ora_sim* s = (ora_sim*)calloc(1, sizeof(ora_sim));
    if (!s) return NULL;
    s->c = *cfg;
    int n[3] = {cfg->nx, cfg->ny, cfg->nz};
    s->N = (int64_t)n[0] * n[1] * n[2];
    s->PN = 1;
    for (int d = 0; d < 3; ++d) {
        s->h[d] = (cfg->hi[d] - cfg->lo[d]) / n[d];
        s->act[d] = n[d] > 1;
        s->g[d] = s->act[d] ? n[d] + 4 : 1;
        s->o[d] = s->act[d] ? 2 : 0;
        s->PN *= s->g[d];
    }
    int ok = 1;
    for (int v = 0; v < 5; ++v) ok &= (s->W[v] = (double*)calloc(s->N, sizeof(double))) != NULL;
    ok &= (s->phi = (double*)calloc(s->N, sizeof(double))) != NULL;
    ok &= (s->chi = (uint8_t*)calloc(s->N, 1)) != NULL;
    for (int v = 0; v < 6; ++v) ok &= (s->P[v] = (double*)calloc(s->PN, sizeof(double))) != NULL;
    ok &= (s->X = (uint8_t*)calloc(s->PN, 1)) != NULL;
    ok &= (s->slot = (int32_t*)malloc(3 * s->N * sizeof(int32_t))) != NULL;
    if (!ok) { ora_destroy(s); return NULL; }
    for (int64_t f = 0; f < 3 * s->N; ++f) s->slot[f] = -1;
    s->st.err_cell = -1;
    return s;
}

void ora_destroy(ora_sim* s)
{
    if (!s) return;
    for (int v = 0; v < 5; ++v) free(s->W[v]);
    free(s->phi); free(s->chi);
    for (int v = 0; v < 6; ++v) free(s->P[v]);
    free(s->X); free(s->slot); free(s->rec);
    free(s);
}

/* Material 1 occupies phi < 0 (reading of the signed-distance convention). */
static uint8_t material_of(double phi) { return phi < 0.0 ? 1 : 0; }

/* Admissible primitive state of material m: finite, rho > 0 and p above
 * the material's floor (p + p_c > 0 for the stiffened gas); with a general
 * EOS also c^2 > 0 (the EOS is used only where it is convex). */
static int physical(const ora_cfg* c, int m, const double* q)
{
    for (int v = 0; v < 5; ++v) if (!isfinite(q[v])) return 0;
    if (!c->eos_general) return q[0] > 0.0 && q[4] + c->pc[m] > 0.0;
    return q[0] > 0.0 && q[4] > ora_eos_floor(&c->eos[m]) && ora_eos_c2(&c->eos[m], q[0], q[4]) > 0.0;
}

int ora_set_prim(ora_sim* s, const double* prim6)
{
    for (int64_t c = 0; c < s->N; ++c) {
        double q[5], w[5];
        for (int v = 0; v < 5; ++v) q[v] = prim6[v * s->N + c];
        double phi = prim6[5 * s->N + c];
        uint8_t m = material_of(phi);
        if (!physical(&s->c, m, q) || !isfinite(phi)) { s->st.err_cell = c; return ORA_ERR_NONPHYSICAL; }
        mat_prim_to_cons(&s->c, m, q, w);
        for (int v = 0; v < 5; ++v) s->W[v][c] = w[v];
        s->phi[c] = phi;
        s->chi[c] = m;
    }
    return ORA_OK;
}

int ora_set_cons(ora_sim* s, const double* w6)
{
    for (int64_t c = 0; c < s->N; ++c) {
        for (int v = 0; v < 5; ++v) s->W[v][c] = w6[v * s->N + c];
        s->phi[c] = w6[5 * s->N + c];
        s->chi[c] = material_of(s->phi[c]);
    }
    return ORA_OK;
}

int ora_get_cons(const ora_sim* s, double* w6)
{
    for (int64_t c = 0; c < s->N; ++c) {
        for (int v = 0; v < 5; ++v) w6[v * s->N + c] = s->W[v][c];
        w6[5 * s->N + c] = s->phi[c];
    }
    return ORA_OK;
}

int ora_get_prim(const ora_sim* s, double* prim6, uint8_t* chi)
{
    for (int64_t c = 0; c < s->N; ++c) {
        double w[5], q[5];
        for (int v = 0; v < 5; ++v) w[v] = s->W[v][c];
        uint8_t m = s->chi[c];
        mat_cons_to_prim(&s->c, m, w, q);
        for (int v = 0; v < 5; ++v) prim6[v * s->N + c] = q[v];
        prim6[5 * s->N + c] = s->phi[c];
        if (chi) chi[c] = m;
    }
    return ORA_OK;
}

void ora_get_stats(const ora_sim* s, ora_stats* st) { *st = s->st; }

/* ------------------------------------------------------------------------ */
/* dt from a CFL number (section "Time integration").  The rule is not given;
 * reading: dt = CFL / max_i sum_{d: n_d > 1} (|V_d| + c) / h_d.            */
static double dt_of(const ora_sim* s, double* const W[5], const uint8_t* chi)
{
    double lmax = 0.0;
#pragma omp parallel for schedule(static) reduction(max : lmax)
    for (int64_t c = 0; c < s->N; ++c) {
        double w[5], q[5];
        for (int v = 0; v < 5; ++v) w[v] = W[v][c];
        uint8_t m = chi[c];
        mat_cons_to_prim(&s->c, m, w, q);
        double cs = mat_sound_speed(&s->c, m, q[0], q[4]);
        double lam = 0.0;
        for (int d = 0; d < 3; ++d)
            if (s->act[d]) lam += (fabs(q[1 + d]) + cs) / s->h[d];
        if (lam > lmax) lmax = lam;
    }
    return s->c.cfl / lmax;
}

double ora_dt(const ora_sim* s)
{
    if (s->c.dt_fixed > 0.0) return s->c.dt_fixed;
    return dt_of(s, s->W, s->chi);
}

/* ------------------------------------------------------------------------ */
/* Ghost layers (two per side).  Transmissive: copy of the nearest interior
 * cell; wall: mirror image with the normal velocity negated; periodic: wrap.
 * Material ids and phi are carried along, so no material interface is ever
 * seen at a transmissive or wall boundary.                                 */
static void fill_ghosts(ora_sim* s)
{
    int n[3] = {s->c.nx, s->c.ny, s->c.nz};
    for (int d = 0; d < 3; ++d) {
        if (!s->act[d]) continue;
        int a1 = (d + 1) % 3, a2 = (d + 2) % 3;
        for (int t2 = 0; t2 < n[a2]; ++t2)
            for (int t1 = 0; t1 < n[a1]; ++t1)
                for (int side = 0; side < 2; ++side)
                    for (int gl = 1; gl <= 2; ++gl) {
                        int bc = s->c.bc[2 * d + side];
                        int dst = side == 0 ? -gl : n[d] - 1 + gl;
                        int src;
                        if (bc == ORA_BC_PERIODIC) src = side == 0 ? n[d] - gl : gl - 1;
                        else if (bc == ORA_BC_WALL) src = side == 0 ? gl - 1 : n[d] - gl;
                        else src = side == 0 ? 0 : n[d] - 1;
                        int is[3], id[3];
                        is[d] = src; id[d] = dst;
                        is[a1] = id[a1] = t1;
                        is[a2] = id[a2] = t2;
                        int64_t ps = pidx(s, is[0], is[1], is[2]);
                        int64_t pd = pidx(s, id[0], id[1], id[2]);
                        for (int v = 0; v < 6; ++v) s->P[v][pd] = s->P[v][ps];
                        s->X[pd] = s->X[ps];
                        if (bc == ORA_BC_WALL) s->P[1 + d][pd] = -s->P[1 + d][ps];
                    }
    }
}

static void add_record(ora_sim* s, int64_t face, const ora_star* r)
{
    if (s->nrec == s->caprec) {
        s->caprec = s->caprec ? 2 * s->caprec : 1024;
        s->rec = (ora_star*)realloc(s->rec, s->caprec * sizeof(ora_star));
    }
    s->slot[face] = (int32_t)s->nrec;
    s->rec[s->nrec++] = *r;
}

static void clear_records(ora_sim* s)
{
    for (int64_t f = 0; f < 3 * s->N; ++f) s->slot[f] = -1;
    s->nrec = 0;
}

/* Residual of eq. NS_discretized (inviscid, no source) and of the level-set
 * equation (eq. levelset) for the state (W, phi) with frozen material ids:
 *   R_i = -sum_d (F_{i,d+} - F_{i,d-}) / h_d,    L_i = -sum_d V_{d,i} D_d phi_i.
 * F_{i,d+-} is the flux through the face that cell i sees: the MUSCL-HLLC
 * flux when both cells hold the same material, otherwise the FIVER flux of
 * cell i's own side.                                                       */
static int residual(ora_sim* s, double* const W[5], const double* phi, const uint8_t* chi,
                    double* R[5], double* L, int record)
{
    int n[3] = {s->c.nx, s->c.ny, s->c.nz};
    int rc = ORA_OK;

    /* primitives of every interior cell, then ghosts */
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                int64_t c = i + (int64_t)n[0] * (j + (int64_t)n[1] * k);
                double w[5], q[5];
                for (int v = 0; v < 5; ++v) w[v] = W[v][c];
                uint8_t m = chi[c];
                mat_cons_to_prim(&s->c, m, w, q);
                int64_t pc = pidx(s, i, j, k);
                for (int v = 0; v < 5; ++v) s->P[v][pc] = q[v];
                s->P[5][pc] = phi[c];
                s->X[pc] = m;
            }
    fill_ghosts(s);

#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < s->N; ++c) {
        for (int v = 0; v < 5; ++v) R[v][c] = 0.0;
        L[c] = 0.0;
    }
    if (record) clear_records(s);

    for (int d = 0; d < 3; ++d) {
        if (!s->act[d]) continue;
        int a1 = (d + 1) % 3, a2 = (d + 2) % 3;
        int64_t stride = (d == 0) ? 1 : (d == 1) ? s->g[0] : (int64_t)s->g[0] * s->g[1];
        int64_t cstride = (d == 0) ? 1 : (d == 1) ? n[0] : (int64_t)n[0] * n[1];
        /* lines along d, in the serial order (t2 outer, t1 inner); each line
         * writes only its own cells.  A general EOS calls back into the
         * caller's solver, which is not asked to be thread-safe. */
        const int64_t nlines = (int64_t)n[a1] * n[a2];
        int64_t solves = 0, iters = 0, fallbacks = 0;
        int64_t bad_line = nlines, bad_cell = -1;
#pragma omp parallel for schedule(static) reduction(+ : solves, iters, fallbacks) if (!s->c.eos_general)
        for (int64_t line = 0; line < nlines; ++line) {
                const int t1 = (int)(line % n[a1]), t2 = (int)(line / n[a1]);
                double FL[n[d] + 1][5], FU[n[d] + 1][5];
                int ib[3];
                ib[d] = 0; ib[a1] = t1; ib[a2] = t2;
                int64_t p0 = pidx(s, ib[0], ib[1], ib[2]);      /* line start  */
                int64_t c0 = ib[0] + (int64_t)n[0] * (ib[1] + (int64_t)n[1] * ib[2]);

                /* faces m = 0..n_d, face m between line cells m-1 and m */
                for (int m = 0; m <= n[d]; ++m) {
                    int64_t pa = p0 + (int64_t)(m - 1) * stride;
                    int64_t pb = p0 + (int64_t)m * stride;
                    uint8_t xa = s->X[pa], xb = s->X[pb];
                    double qa[5], qb[5];      /* face frame: (rho, u_n, v_t1, v_t2, p) */
                    int comp[5] = {0, 1 + d, 1 + a1, 1 + a2, 4};
                    for (int v = 0; v < 5; ++v) {
                        int V = comp[v];
                        qa[v] = s->P[V][pa];
                        qb[v] = s->P[V][pb];
                    }
                    double Fr_l[5], Fr_u[5];
                    if (xa == xb) {
                        /* MUSCL on primitive variables; the slope of a cell
                         * vanishes along d when a d-neighbour holds the other
                         * material (reading: no stencil crosses an interface). */
                        int flat_a = s->X[pa - stride] != xa || s->X[pa + stride] != xa;
                        int flat_b = s->X[pb - stride] != xb || s->X[pb + stride] != xb;
                        double la[5], rb[5];
                        for (int v = 0; v < 5; ++v) {
                            int V = comp[v];
                            double sa = flat_a ? 0.0 :
                                limited_slope(&s->c, s->P[V][pa] - s->P[V][pa - stride],
                                              s->P[V][pa + stride] - s->P[V][pa]);
                            double sb = flat_b ? 0.0 :
                                limited_slope(&s->c, s->P[V][pb] - s->P[V][pb - stride],
                                              s->P[V][pb + stride] - s->P[V][pb]);
                            la[v] = qa[v] + 0.5 * sa;
                            rb[v] = qb[v] - 0.5 * sb;
                        }
                        num_flux(&s->c, la, rb, xa, Fr_l);
                        for (int v = 0; v < 5; ++v) Fr_u[v] = Fr_l[v];
                    } else {
                        /* FIVER: exact two-material Riemann problem along the
                         * face normal, then one one-sided flux per side,
                         * each with its own EOS.  The paper's second formula
                         * lists the j-side state first; the arguments are
                         * taken here in their order along n_ij (star state on
                         * the left of cell j's state), which is the reading
                         * that makes the flux consistent.                   */
                        double in[6] = {qa[0], qa[1], qa[4], qb[0], qb[1], qb[4]};
                        double eos[4] = {s->c.gamma[xa], s->c.pc[xa], s->c.gamma[xb], s->c.pc[xb]};
                        double out[4];
                        int32_t it = 0;
                        int e = s->c.eos_general ? s->c.riemann(xa, xb, in, out)
                                                 : ora_riemann(in, eos, s->c.rtol, s->c.maxit, out, &it);
                        solves++;
                        iters += it < 0 ? -it : it;
                        if (it < 0) fallbacks++;
                        if (e != ORA_OK) {
                            /* the first failing face in loop order names the cell */
#pragma omp critical(ora_residual_error)
                            {
                                rc = e;
                                if (line < bad_line) {
                                    int ic[3]; ic[d] = m < n[d] ? m : n[d] - 1; ic[a1] = t1; ic[a2] = t2;
                                    bad_line = line;
                                    bad_cell = ic[0] + (int64_t)n[0] * (ic[1] + (int64_t)n[1] * ic[2]);
                                }
                            }
                            for (int v = 0; v < 5; ++v) Fr_l[v] = Fr_u[v] = 0.0;
                        } else {
                            double sa[5] = {out[2], out[1], qa[2], qa[3], out[0]};
                            double sb[5] = {out[3], out[1], qb[2], qb[3], out[0]};
                            num_flux(&s->c, qa, sa, xa, Fr_l);
                            num_flux(&s->c, sb, qb, xb, Fr_u);
                            if (record && m >= 1) {
                                ora_star r;
                                r.pstar = out[0]; r.ustar = out[1]; r.rhoL = out[2]; r.rhoR = out[3];
                                for (int a = 0; a < 3; ++a) {
                                    r.VL[a] = s->P[1 + a][pa];
                                    r.VR[a] = s->P[1 + a][pb];
                                }
                                int64_t ca = c0 + (int64_t)(m - 1) * cstride;
#pragma omp critical(ora_records)
                                add_record(s, 3 * ca + d, &r);
                            }
                        }
                    }
                    /* back to x, y, z momentum components */
                    for (int v = 0; v < 5; ++v) {
                        FL[m][comp[v]] = Fr_l[v];
                        FU[m][comp[v]] = Fr_u[v];
                    }
                }
                /* accumulate (F_{i,d+} - F_{i,d-}) / h_d and the level-set term */
                for (int i = 0; i < n[d]; ++i) {
                    int64_t c = c0 + (int64_t)i * cstride;
                    int64_t pcl = p0 + (int64_t)i * stride;
                    for (int v = 0; v < 5; ++v) R[v][c] += (FL[i + 1][v] - FU[i][v]) / s->h[d];
                    double f[5];
                    for (int q = 0; q < 5; ++q) f[q] = s->P[5][pcl + (int64_t)(q - 2) * stride];
                    double Vd = s->P[1 + d][pcl];
                    L[c] += Vd * ora_ls_derivative(f, Vd, s->h[d]);
                }
            }
        s->st.riemann_solves += solves;
        s->st.newton_iters += iters;
        s->st.bisection_fallbacks += fallbacks;
        if (bad_cell >= 0 && s->st.err_cell < 0) s->st.err_cell = bad_cell;
    }
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < s->N; ++c) {
        for (int v = 0; v < 5; ++v) R[v][c] = -R[v][c];
        L[c] = -L[c];
        /* narrow band (section "Level set method" of the numerical methods):
         * the level-set equation is solved only where the stage-input |phi|
         * is below the bandwidth; elsewhere phi is held */
        if (s->c.ls_band > 0.0 && fabs(phi[c]) >= s->c.ls_band) L[c] = 0.0;
    }
    return rc;
}

/* A stage result is admissible when rho > 0, p + p_c > 0 (with the frozen
 * material ids) and all values are finite. */
static int check_state(ora_sim* s, double* const W[5], const double* phi, const uint8_t* chi)
{
    int64_t bad = s->N;                 /* first failing cell */
#pragma omp parallel for schedule(static) reduction(min : bad)
    for (int64_t c = 0; c < s->N; ++c) {
        double w[5], q[5];
        for (int v = 0; v < 5; ++v) w[v] = W[v][c];
        uint8_t m = chi[c];
        mat_cons_to_prim(&s->c, m, w, q);
        if (!physical(&s->c, m, q) || !isfinite(phi[c])) {
            if (c < bad) bad = c;
        }
    }
    if (bad < s->N) {
        if (s->st.err_cell < 0) s->st.err_cell = bad;
        return ORA_ERR_NONPHYSICAL;
    }
    return ORA_OK;
}

/* Phase update, step (6) of the time-step outline in section "Code
 * structure": material ids follow the sign of the new level set, and cells
 * whose id changed get a state of their new material.  The paper does not
 * state the rule; reading: a cell that flipped from material A to B takes
 * the mean, over its faces (order -x,+x,-y,+y,-z,+z) whose neighbour held B
 * during the step, of the B-side star state of the last stage's Riemann
 * problem at that face (density rho*_B, the B cell's velocity with the
 * normal component replaced by u*, pressure p*), re-encoded with B's EOS.
 * Without such a face the cell keeps its primitive state ("orphan").  */
static int phase_update(ora_sim* s)
{
    int n[3] = {s->c.nx, s->c.ny, s->c.nz};
    int64_t cstr[3] = {1, n[0], (int64_t)n[0] * n[1]};
    uint8_t* newchi = (uint8_t*)malloc(s->N);
    int rc = ORA_OK;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < s->N; ++c) newchi[c] = material_of(s->phi[c]);

    int64_t flips = 0, orphans = 0, bad = s->N;    /* bad: first non-physical cell */
#pragma omp parallel for schedule(static) reduction(+ : flips, orphans) reduction(min : bad)
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                int64_t c = i + (int64_t)n[0] * (j + (int64_t)n[1] * k);
                uint8_t A = s->chi[c], B = newchi[c];
                if (A == B) continue;
                flips++;
                int ijk[3] = {i, j, k};
                double sum[5] = {0, 0, 0, 0, 0};
                int cnt = 0;
                for (int d = 0; d < 3; ++d) {
                    if (!s->act[d]) continue;
                    for (int side = 0; side < 2; ++side) {        /* - then + */
                        int nb = ijk[d] + (side ? 1 : -1);
                        if (nb < 0 || nb >= n[d]) {
                            if (s->c.bc[2 * d + side] != ORA_BC_PERIODIC) continue;
                            nb = (nb + n[d]) % n[d];
                        }
                        int64_t ck = c + (int64_t)(nb - ijk[d]) * cstr[d];
                        if (s->chi[ck] != B) continue;
                        int64_t lower = side ? c : ck;
                        int32_t sl = s->slot[3 * lower + d];
                        if (sl < 0) continue;
                        const ora_star* r = &s->rec[sl];
                        double q[5];
                        q[0] = side ? r->rhoR : r->rhoL;
                        for (int a = 0; a < 3; ++a) q[1 + a] = side ? r->VR[a] : r->VL[a];
                        q[1 + d] = r->ustar;
                        q[4] = r->pstar;
                        for (int v = 0; v < 5; ++v) sum[v] += q[v];
                        ++cnt;
                    }
                }
                double q[5], w[5];
                if (cnt) {
                    for (int v = 0; v < 5; ++v) q[v] = sum[v] / cnt;
                } else {
                    for (int v = 0; v < 5; ++v) w[v] = s->W[v][c];
                    mat_cons_to_prim(&s->c, A, w, q);
                    orphans++;
                }
                if (!physical(&s->c, B, q) && c < bad) bad = c;
                mat_prim_to_cons(&s->c, B, q, w);
                for (int v = 0; v < 5; ++v) s->W[v][c] = w[v];
            }
    s->st.flips += flips;
    s->st.orphans += orphans;
    if (bad < s->N) {
        if (s->st.err_cell < 0) s->st.err_cell = bad;
        rc = ORA_ERR_NONPHYSICAL;
    }
    memcpy(s->chi, newchi, s->N);
    free(newchi);
    return rc;
}

/* One time step: TVD Runge-Kutta of the chosen order (section "Time
 * integration") applied to the coupled fluid + level-set system, with the
 * material ids frozen at their start-of-step values for every stage; then
 * the phase update.  On failure the start-of-step state is restored.     */
static int one_step(ora_sim* s, double dt_imposed)
{
    const int64_t N = s->N;
    double *W0[5], *W1[5], *W2[5], *R[5];
    double *phi0, *phi1, *phi2, *L;
    for (int v = 0; v < 5; ++v) {
        W0[v] = (double*)malloc(N * sizeof(double));
        W1[v] = (double*)malloc(N * sizeof(double));
        W2[v] = (double*)malloc(N * sizeof(double));
        R[v] = (double*)malloc(N * sizeof(double));
        memcpy(W0[v], s->W[v], N * sizeof(double));
    }
    phi0 = (double*)malloc(N * sizeof(double));
    phi1 = (double*)malloc(N * sizeof(double));
    phi2 = (double*)malloc(N * sizeof(double));
    L = (double*)malloc(N * sizeof(double));
    memcpy(phi0, s->phi, N * sizeof(double));

    double dt = dt_imposed > 0.0 ? dt_imposed
              : (s->c.dt_fixed > 0.0 ? s->c.dt_fixed : dt_of(s, s->W, s->chi));
    int rc = ORA_OK;
    const int order = s->c.rk_order;
    int64_t solves0 = s->st.riemann_solves;

    /* stage 1: W(1) = W^n + dt R(W^n) */
    rc = residual(s, W0, phi0, s->chi, R, L, order == 1);
    s->st.iface_faces_last = s->st.riemann_solves - solves0;
    if (rc == ORA_OK) {
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < N; ++c) {
            for (int v = 0; v < 5; ++v) W1[v][c] = W0[v][c] + dt * R[v][c];
            phi1[c] = phi0[c] + dt * L[c];
        }
        rc = check_state(s, W1, phi1, s->chi);
    }
    if (rc == ORA_OK && order == 2) {
        /* W^{n+1} = 1/2 W^n + 1/2 (W(1) + dt R(W(1))) */
        rc = residual(s, W1, phi1, s->chi, R, L, 1);
        if (rc == ORA_OK) {
    #pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < N; ++c) {
                for (int v = 0; v < 5; ++v) W2[v][c] = 0.5 * W0[v][c] + 0.5 * (W1[v][c] + dt * R[v][c]);
                phi2[c] = 0.5 * phi0[c] + 0.5 * (phi1[c] + dt * L[c]);
            }
            rc = check_state(s, W2, phi2, s->chi);
        }
    } else if (rc == ORA_OK && order == 3) {
        /* W(2) = 3/4 W^n + 1/4 W(1) + 1/4 dt R(W(1));
         * W^{n+1} = 1/3 W^n + 2/3 W(2) + 2/3 dt R(W(2)) */
        rc = residual(s, W1, phi1, s->chi, R, L, 0);
        if (rc == ORA_OK) {
    #pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < N; ++c) {
                for (int v = 0; v < 5; ++v) W2[v][c] = 0.75 * W0[v][c] + 0.25 * W1[v][c] + 0.25 * dt * R[v][c];
                phi2[c] = 0.75 * phi0[c] + 0.25 * phi1[c] + 0.25 * dt * L[c];
            }
            rc = check_state(s, W2, phi2, s->chi);
        }
        if (rc == ORA_OK) rc = residual(s, W2, phi2, s->chi, R, L, 1);
        if (rc == ORA_OK) {
    #pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < N; ++c) {
                for (int v = 0; v < 5; ++v)
                    W2[v][c] = W0[v][c] / 3.0 + 2.0 / 3.0 * W2[v][c] + 2.0 / 3.0 * dt * R[v][c];
                phi2[c] = phi0[c] / 3.0 + 2.0 / 3.0 * phi2[c] + 2.0 / 3.0 * dt * L[c];
            }
            rc = check_state(s, W2, phi2, s->chi);
        }
    }
    if (rc == ORA_OK) {
        double** Wn = order == 1 ? W1 : W2;
        double* phin = order == 1 ? phi1 : phi2;
        for (int v = 0; v < 5; ++v) memcpy(s->W[v], Wn[v], N * sizeof(double));
        memcpy(s->phi, phin, N * sizeof(double));
        rc = phase_update(s);
        if (rc != ORA_OK) {
            for (int v = 0; v < 5; ++v) memcpy(s->W[v], W0[v], N * sizeof(double));
            memcpy(s->phi, phi0, N * sizeof(double));
            for (int64_t c = 0; c < N; ++c) s->chi[c] = material_of(phi0[c]);
        } else {
            s->st.steps++;
            s->st.t += dt;
            s->st.dt_last = dt;
        }
    }
    for (int v = 0; v < 5; ++v) { free(W0[v]); free(W1[v]); free(W2[v]); free(R[v]); }
    free(phi0); free(phi1); free(phi2); free(L);
    return rc;
}

int ora_step(ora_sim* s, int32_t nsteps)
{
    for (int32_t k = 0; k < nsteps; ++k) {
        int rc = one_step(s, 0.0);
        if (rc != ORA_OK) return rc;
    }
    return ORA_OK;
}

int ora_step_dt(ora_sim* s, int32_t nsteps, double dt)
{
    if (!(dt > 0.0)) return ORA_ERR_ARG;
    for (int32_t k = 0; k < nsteps; ++k) {
        int rc = one_step(s, dt);
        if (rc != ORA_OK) return rc;
    }
    return ORA_OK;
}

int64_t ora_interface_faces(const ora_sim* s, int32_t* out, int64_t cap)
{
    int n[3] = {s->c.nx, s->c.ny, s->c.nz};
    int64_t cstr[3] = {1, n[0], (int64_t)n[0] * n[1]};
    int64_t cnt = 0;
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                int64_t c = i + (int64_t)n[0] * (j + (int64_t)n[1] * k);
                int ijk[3] = {i, j, k};
                for (int d = 0; d < 3; ++d) {
                    if (!s->act[d]) continue;
                    int nb = ijk[d] + 1;
                    if (nb >= n[d]) {
                        if (s->c.bc[2 * d + 1] != ORA_BC_PERIODIC) continue;
                        nb = 0;
                    }
                    int64_t ck = c + (int64_t)(nb - ijk[d]) * cstr[d];
                    if (s->chi[c] != s->chi[ck]) {
                        if (cnt < cap) out[cnt] = (int32_t)(3 * c + d);
                        ++cnt;
                    }
                }
            }
    return cnt;
}
