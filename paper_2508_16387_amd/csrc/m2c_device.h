// m2c_device.h -- per-face and per-cell device arithmetic of the method.
//
// Stiffened gas (eq. NASG_EOS with b = e_c = 0): p = (gamma-1) rho e - gamma p_c,
// c^2 = gamma (p + p_c)/rho.  Flux and limiter follow the appendices "HLLC
// flux" and "Slope limiters"; the interface Riemann problem is eq.
// 1DRiemannProblem for two stiffened gases.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "m2c_internal.h"

namespace m2c {

// Material parameter of material x (0 or 1) as a select rather than an
// indexed load, so that per-lane material ids never force the parameter
// arrays into private memory.
__device__ __forceinline__ double pick(const double (&a)[2], int x) { return x ? a[1] : a[0]; }

// Field access through a 32-bit byte offset from a wave-uniform base (grids
// are limited to 2^29 cells), so the address lives in one VGPR instead of a
// 64-bit pair per field and access.
__device__ __forceinline__ double ldf(const double* base, uint32_t c)
{
    return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + (c << 3));
}
__device__ __forceinline__ void stf(double* base, uint32_t c, double v)
{
    *reinterpret_cast<double*>(reinterpret_cast<char*>(base) + (c << 3)) = v;
}

// ------------------------------------------------------- fast rcp / sqrt --
// Reciprocal and square root from the hardware estimates refined by
// Newton-Raphson (reciprocal) and Goldschmidt (square root) iterations,
// accurate to about one ulp for the positive normal arguments of the flux
// and EOS formulas; far shorter dependency chains than the correctly
// rounded library sequences.
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float rcp_nr(float x)
{
    float r = __builtin_amdgcn_rcpf(x);
    const float e = fmaf(-x, r, 1.0f);
    return fmaf(r, e, r);
}
__device__ __forceinline__ double sqrt_nr(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, x);
    return fma(d, h, g);
}
__device__ __forceinline__ float sqrt_nr(float x)
{
    const float y = __builtin_amdgcn_rsqf(x);
    float g = x * y;
    const float h = 0.5f * y;
    const float d = fmaf(-g, g, x);
    return fmaf(d, h, g);
}

// ---------------------------------------------------------------- EOS ------
// Conservative -> primitive for one cell; returns the pressure.
__device__ __forceinline__ double eos_prim(double r, double mx, double my, double mz, double E,
                                           double gm1, double gpc,
                                           double& u, double& v, double& w)
{
    const double ri = rcp_nr(r);
    u = mx * ri;
    v = my * ri;
    w = mz * ri;
    const double ke = 0.5 * (mx * u + my * v + mz * w);
    return gm1 * (E - ke) - gpc;
}

// Total energy per unit volume of a primitive state.
template <typename T>
__device__ __forceinline__ T eos_energy(T r, T u, T v, T w, T p, T gpc, T inv_gm1)
{
    return (p + gpc) * inv_gm1 + T(0.5) * r * (u * u + v * v + w * w);
}

// ------------------------------------------------------------ limiter ------
// MC-limited slope: with theta = dm/dp the paper's phi(theta) dp on a uniform
// grid equals minmod(alpha dm, (dm + dp)/2, alpha dp); this is the
// division-free form of the same function.
// (alpha min(|dm|, |dp|) equals min(alpha |dm|, alpha |dp|) exactly, since
// rounding is monotone.)
template <typename T>
__device__ __forceinline__ T mc_slope(T dm, T dp, T alpha)
{
    const T a = fmin(alpha * fmin(fabs(dm), fabs(dp)), T(0.5) * fabs(dm + dp));
    return (dm * dp > T(0)) ? copysign(a, dp) : T(0);
}

// Van Albada slope (appendix "Slope limiters", eq. vanalbada with A = B = 1
// on a uniform grid): phi(theta) = (theta^k + theta) / (theta^k + 1) with
// theta = dm / dp, times dp; the modified limiter (eq. vanalbada_mod) takes
// phi = 0 where it is negative; where theta^k overflows, phi takes its
// limit 1; dp = 0 gives 0.
template <typename T>
__device__ __forceinline__ T va_slope(T dm, T dp, int k, bool modified)
{
    if (dp == T(0)) return T(0);
    const T theta = dm / dp;
    T tk = T(1);
    for (int e = 0; e < k; ++e) tk *= theta;
    T lim = isfinite(tk) ? (tk + theta) / (tk + T(1)) : T(1);
    if (modified && lim < T(0)) lim = T(0);
    return lim * dp;
}

// Limited slope of the configured limiter (limiter uniform over a launch).
template <typename T>
__device__ __forceinline__ T lim_slope(int limiter, int k, T dm, T dp, T alpha)
{
    if (limiter == LIM_MC) return mc_slope<T>(dm, dp, alpha);
    return va_slope<T>(dm, dp, k, limiter == LIM_VA_MOD);
}

// Half the limited slope (the offset of a face value from the cell value
// in the linear reconstruction), or 0 where the cell's stencil along the
// axis reaches the other material (flat).  halpha = alpha / 2.  For the MC
// limiter the halving is folded into the limiter's constants, which gives
// the same value as halving the slope (scaling by a power of two commutes
// with rounding), and the flag joins the limiter's own sign test, so the
// slope stays one select and never becomes a divergent branch per variable.
template <typename T>
__device__ __forceinline__ T lim_half_slope_flat(int limiter, int k, T dm, T dp, T halpha, bool flat)
{
    if (limiter == LIM_MC) {
        const T a = fmin(halpha * fmin(fabs(dm), fabs(dp)), T(0.25) * fabs(dm + dp));
        return ((!flat) & (dm * dp > T(0))) ? copysign(a, dp) : T(0);
    }
    return flat ? T(0) : T(0.5) * va_slope<T>(dm, dp, k, limiter == LIM_VA_MOD);
}

// --------------------------------------------------------------- HLLC ------
// Flux through a face with normal +n in the face frame: state = (rho, u_n,
// v_t1, v_t2, p).  Davis wave speeds, contact speed S_*, and the star state
// rho_K (S_K - u_K)/(S_K - S_*) [1, S_*, v_t1, v_t2, E*_K] with Toro's E*.
// The case selection reproduces the four cases of the appendix in the
// same order, without divergent branches.
// hllc_ce takes each state's 1/rho, sound speed and total energy per unit
// volume (all the flux needs of the EOS); hllc computes them for a
// stiffened gas.
template <typename T>
__device__ __forceinline__ void hllc_ce(T rL, T uL, T aL, T bL, T pL, T riL, T cL, T EL,
                                        T rR, T uR, T aR, T bR, T pR, T riR, T cR, T ER, T F[5])
{
    const T SL = fmin(uL - cL, uR - cR);
    const T SR = fmax(uL + cL, uR + cR);
    const T dL = rL * (SL - uL), dR = rR * (SR - uR);
    const T Ss = (pR - pL + uL * dL - uR * dR) * rcp_nr(dL - dR);

    const bool left_sup = T(0) <= SL;
    const bool useL = left_sup || (T(0) <= Ss);
    const bool star = useL ? !left_sup : (T(0) <= SR);

    const T r = useL ? rL : rR, u = useL ? uL : uR, a = useL ? aL : aR, b = useL ? bL : bR;
    const T p = useL ? pL : pR, E = useL ? EL : ER, S = useL ? SL : SR;
    const T ri = useL ? riL : riR;
    const T mu = r * u;
    T Fk[5];
    Fk[0] = mu;
    Fk[1] = mu * u + p;
    Fk[2] = mu * a;
    Fk[3] = mu * b;
    Fk[4] = (E + p) * u;
    if (star) {
        const T inv = rcp_nr(S - Ss);
        const T fac = r * (S - u) * inv;
        const T Us0 = fac;
        const T Us1 = fac * Ss;
        const T Us2 = fac * a;
        const T Us3 = fac * b;
        const T Us4 = fac * E * ri + (Ss - u) * (fac * Ss + p * inv);
        F[0] = Fk[0] + S * (Us0 - r);
        F[1] = Fk[1] + S * (Us1 - mu);
        F[2] = Fk[2] + S * (Us2 - r * a);
        F[3] = Fk[3] + S * (Us3 - r * b);
        F[4] = Fk[4] + S * (Us4 - E);
    } else {
        for (int v = 0; v < 5; ++v) F[v] = Fk[v];
    }
}

template <typename T>
__device__ __forceinline__ void hllc(T rL, T uL, T aL, T bL, T pL,
                                     T rR, T uR, T aR, T bR, T pR,
                                     T g, T pc, T gpc, T inv_gm1, T F[5])
{
    const T riL = rcp_nr(rL), riR = rcp_nr(rR);
    const T cL = sqrt_nr(g * (pL + pc) * riL);
    const T cR = sqrt_nr(g * (pR + pc) * riR);
    const T EL = eos_energy<T>(rL, uL, aL, bL, pL, gpc, inv_gm1);
    const T ER = eos_energy<T>(rR, uR, aR, bR, pR, gpc, inv_gm1);
    hllc_ce<T>(rL, uL, aL, bL, pL, riL, cL, EL, rR, uR, aR, bR, pR, riR, cR, ER, F);
}

// ------------------------------------------------ local Lax-Friedrichs ----
// Appendix "Local Lax-Friedrichs flux" (eq. Lax-Friedrichs), face frame as
// for hllc: the mean of the physical fluxes minus half the fastest wave
// speed max(|u_L| + c_L, |u_R| + c_R) times the jump of the conservative
// state.
template <typename T>
__device__ __forceinline__ void llf_ce(T rL, T uL, T aL, T bL, T pL, T cL, T EL, T rR, T uR, T aR, T bR, T pR,
                                       T cR, T ER, T F[5])
{
    const T lm = fmax(fabs(uL) + cL, fabs(uR) + cR);
    const T mL = rL * uL, mR = rR * uR;
    F[0] = T(0.5) * (mL + mR) - T(0.5) * lm * (rR - rL);
    F[1] = T(0.5) * (mL * uL + pL + (mR * uR + pR)) - T(0.5) * lm * (mR - mL);
    F[2] = T(0.5) * (mL * aL + mR * aR) - T(0.5) * lm * (rR * aR - rL * aL);
    F[3] = T(0.5) * (mL * bL + mR * bR) - T(0.5) * lm * (rR * bR - rL * bL);
    F[4] = T(0.5) * ((EL + pL) * uL + (ER + pR) * uR) - T(0.5) * lm * (ER - EL);
}

template <typename T>
__device__ __forceinline__ void llf(T rL, T uL, T aL, T bL, T pL, T rR, T uR, T aR, T bR, T pR, T g, T pc,
                                    T gpc, T inv_gm1, T F[5])
{
    const T EL = eos_energy<T>(rL, uL, aL, bL, pL, gpc, inv_gm1);
    const T ER = eos_energy<T>(rR, uR, aR, bR, pR, gpc, inv_gm1);
    const T cL = sqrt_nr(g * (pL + pc) * rcp_nr(rL));
    const T cR = sqrt_nr(g * (pR + pc) * rcp_nr(rR));
    llf_ce<T>(rL, uL, aL, bL, pL, cL, EL, rR, uR, aR, bR, pR, cR, ER, F);
}

// ------------------------------------------------------- general EOS -----
// A material with a general EOS (section "Equations of state": NASG,
// Mie-Grueneisen, JWL; FP64 only).  Conservative -> primitive: returns p.
// The NASG and JWL forms are written out here with the refined reciprocal
// and the density the caller already has (r = 1/vi), so that neither takes
// an IEEE division (the liquids, gases and detonation products of the
// common cases); Mie-Grueneisen takes the general functions.
// S: the set of families the material may have (bit mask, eos::fam_set);
// a kernel compiled for the families of its two materials carries only
// their code, eos::FAM_ALL dispatches on the tag at run time.
template <int S = eos::FAM_ALL>
__device__ __forceinline__ double geos_p(const eos::EosK& m, double r, double vi, double e)
{
    if (eos::fam_of<S>(m) == M2C_EOS_NASG) return (e - m.k[3]) * rcp_nr((vi - m.k[2]) * m.k[4]) - m.k[5];
    if (eos::fam_of<S>(m) == M2C_EOS_JWL) {
        double T, dT;
        eos::jwl_terms_rho(m, vi, r, T, dT);
        return m.k[0] * e * r + T;
    }
    return eos::eos_p<S>(m, vi, e);
}
template <int S = eos::FAM_ALL>
__device__ __forceinline__ double geos_e(const eos::EosK& m, double r, double vi, double p)
{
    if (eos::fam_of<S>(m) == M2C_EOS_NASG) return (p + m.k[5]) * (vi - m.k[2]) * m.k[4] + m.k[3];
    if (eos::fam_of<S>(m) == M2C_EOS_JWL) {
        double T, dT;
        eos::jwl_terms_rho(m, vi, r, T, dT);
        return (p - T) * vi * m.k[7];
    }
    return eos::eos_e<S>(m, vi, p);
}
template <int S = eos::FAM_ALL>
__device__ __forceinline__ double geos_c2v(const eos::EosK& m, double r, double vi, double p)
{
    if (eos::fam_of<S>(m) == M2C_EOS_NASG) return m.k[0] * (p + m.k[1]) * vi * vi * rcp_nr(vi - m.k[2]);
    if (eos::fam_of<S>(m) == M2C_EOS_JWL) {
        double T, dT;
        eos::jwl_terms_rho(m, vi, r, T, dT);
        return ((1.0 + m.k[0]) * p - T) * vi + dT;
    }
    return eos::eos_c2<S>(m, vi, p);
}

template <int S = eos::FAM_ALL>
__device__ __forceinline__ double geos_prim(const eos::EosK& m, double r, double mx, double my, double mz,
                                            double E, double& u, double& v, double& w)
{
    const double ri = rcp_nr(r);
    u = mx * ri;
    v = my * ri;
    w = mz * ri;
    const double ke = 0.5 * (mx * u + my * v + mz * w);
    return geos_p<S>(m, r, ri, (E - ke) * ri);
}

// Total energy per unit volume of a primitive state.
__device__ __forceinline__ double geos_energy(const eos::EosK& m, double r, double u, double v, double w, double p)
{
    return r * geos_e(m, r, rcp_nr(r), p) + 0.5 * r * (u * u + v * v + w * w);
}

// c^2 of a state (<= 0 or NaN where the EOS is not hyperbolic).
template <int S = eos::FAM_ALL>
__device__ __forceinline__ double geos_c2(const eos::EosK& m, double r, double p)
{
    return geos_c2v<S>(m, r, rcp_nr(r), p);
}

// Admissible primitive state: finite, rho > 0, p above the floor, c^2 > 0.
__device__ __forceinline__ bool geos_ok(const eos::EosK& m, double r, double p)
{
    return r > 0.0 && p > m.k[eos::KFLOOR] && geos_c2(m, r, p) > 0.0;
}

// Numerical flux between two states of one general-EOS material.
template <int S = eos::FAM_ALL>
__device__ __forceinline__ void geos_flux(const eos::EosK& m, int flux, double rL, double uL, double aL, double bL,
                                          double pL, double rR, double uR, double aR, double bR, double pR,
                                          double F[5])
{
    const double riL = rcp_nr(rL), riR = rcp_nr(rR);
    const double cL = sqrt_nr(geos_c2v<S>(m, rL, riL, pL)), cR = sqrt_nr(geos_c2v<S>(m, rR, riR, pR));
    const double EL = rL * geos_e<S>(m, rL, riL, pL) + 0.5 * rL * (uL * uL + aL * aL + bL * bL);
    const double ER = rR * geos_e<S>(m, rR, riR, pR) + 0.5 * rR * (uR * uR + aR * aR + bR * bR);
    if (flux == FLUX_LLF) llf_ce<double>(rL, uL, aL, bL, pL, cL, EL, rR, uR, aR, bR, pR, cR, ER, F);
    else hllc_ce<double>(rL, uL, aL, bL, pL, riL, cL, EL, rR, uR, aR, bR, pR, riR, cR, ER, F);
}

// Copy of the two materials' general EOS into LDS (per-lane material ids
// then index LDS); every thread of the block calls it before any exit, and
// it ends with a barrier.
__device__ __forceinline__ void geos_stage(const Grid& G, eos::EosK* s)
{
    constexpr int W = (int)(sizeof(eos::EosK) / sizeof(double));
    static_assert(sizeof(eos::EosK) % sizeof(double) == 0, "EosK layout");
    const double* src = reinterpret_cast<const double*>(G.ek);
    double* dst = reinterpret_cast<double*>(s);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int t = 0; t < 2 * W; ++t) dst[t] = src[t];
    }
    __syncthreads();
}

// Numerical flux of the configuration (flux uniform over a launch).
template <typename T>
__device__ __forceinline__ void num_flux(int flux, T rL, T uL, T aL, T bL, T pL, T rR, T uR, T aR, T bR, T pR,
                                         T g, T pc, T gpc, T inv_gm1, T F[5])
{
    if (flux == FLUX_LLF) llf<T>(rL, uL, aL, bL, pL, rR, uR, aR, bR, pR, g, pc, gpc, inv_gm1, F);
    else hllc<T>(rL, uL, aL, bL, pL, rR, uR, aR, bR, pR, g, pc, gpc, inv_gm1, F);
}

// ----------------------------------------------- two-material Riemann ------
// For a stiffened gas the shifted pressure pbar = p + p_c follows the
// ideal-gas shock and rarefaction relations, so side K contributes the
// classical wave function f_K(p); the star pressure is the root of
// g(p) = f_L + f_R + u_R - u_L on p > p_lo = -min(pc_L, pc_R).
struct RSide {
    double r, u, p, pc, pbar, c, A, B, mu, z, k2c, rc;
    double ipbar, irc, sqA;       // 1/pbar, 1/(rho c), sqrt(A)
};

__device__ __forceinline__ void rside_init(RSide& s, double r, double u, double p, double g, double pc)
{
    s.r = r; s.u = u; s.p = p; s.pc = pc;
    s.pbar = p + pc;
    s.c = sqrt(g * s.pbar / r);
    s.mu = (g - 1.0) / (g + 1.0);
    s.A = 2.0 / ((g + 1.0) * r);
    s.B = s.mu * s.pbar;
    s.z = (g - 1.0) / (2.0 * g);
    s.k2c = 2.0 * s.c / (g - 1.0);
    s.rc = r * s.c;
    s.ipbar = 1.0 / s.pbar;
    s.irc = 1.0 / s.rc;
    s.sqA = sqrt(s.A);
}

// Reciprocal square root from the hardware estimate refined by two
// Newton-Raphson steps (about one ulp for positive normal arguments).
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    return y * fma(-h * y, y, 1.5);
}

// f_K(p) and f_K'(p).  Shock: (p - p_K) sqrt(A/(pbar + B)); rarefaction:
// 2c/(gamma-1) ((pbar/pbar_K)^z - 1) with z = (gamma-1)/(2 gamma); the
// derivative of the latter is (pbar/pbar_K)^(z-1) / (rho c).  Written with
// the side's reciprocals, the refined reciprocal and reciprocal square root,
// and the power as exp2(z log2 x): no IEEE division in the iteration.
__device__ __forceinline__ double rside_f(const RSide& s, double p, double& df)
{
    const double pb = p + s.pc;
    if (p > s.p) {
        const double den = pb + s.B;
        const double rs = rsqrt_nr(den);
        const double q = s.sqA * rs;
        df = q * (1.0 - (p - s.p) * 0.5 * rs * rs);
        return (p - s.p) * q;
    }
    const double x = pb * s.ipbar;
    const double t = exp2(s.z * log2(x));
    df = t * rcp_nr(x) * s.irc;
    return s.k2c * (t - 1.0);
}

__device__ __forceinline__ double rside_f(const RSide& s, double p)
{
    double d;
    return rside_f(s, p, d);
}

__device__ __forceinline__ double rside_star_rho(const RSide& s, double g, double ps)
{
    const double x = (ps + s.pc) / s.pbar;
    if (ps > s.p) return s.r * (x + s.mu) / (s.mu * x + 1.0);
    return s.r * pow(x, 1.0 / g);
}

// Safeguarded Newton from the acoustic guess, or from a candidate guess
// when one is given and its |g| is no larger than the tangent at it predicts
// for the acoustic guess (the candidate must be finite and above p_lo); then
// bisection if maxit steps did not meet
// |dp| <= rtol (p - p_lo).  Returns the Newton step count (negative:
// bisection fallback, 0: no admissible root).  out = (p*, u*, rho*_L,
// rho*_R); *used (nullable) tells whether the candidate was the start.
__device__ __forceinline__ int riemann_solve(double rL, double uL, double pL, double gL, double pcL,
                                             double rR, double uR, double pR, double gR, double pcR,
                                             double rtol, int maxit, bool have_guess, double guess,
                                             double out[4], bool* used = nullptr)
{
    RSide L, R;
    rside_init(L, rL, uL, pL, gL, pcL);
    rside_init(R, rR, uR, pR, gR, pcR);
    const double du = uR - uL;
    const double plo = -fmin(pcL, pcR);
    const double glo = rside_f(L, plo) + rside_f(R, plo) + du;
    if (used) *used = false;
    if (!(glo < 0.0)) {
        out[0] = out[1] = out[2] = out[3] = __builtin_nan("");
        return 0;
    }
    const double ZL = L.rc, ZR = R.rc;
    const double pac = (ZR * pL + ZL * pR + ZL * ZR * (uL - uR)) / (ZL + ZR);
    double p = fmax(pac, plo + 1e-6 * fmin(pL - plo, pR - plo));
    // judged start: g and g' at the candidate (they are the first Newton
    // step's when it is kept); the acoustic start's |g| is predicted from the
    // tangent there, and the candidate is kept unless the acoustic start is
    // predicted closer to the root.  (g is increasing and concave, so the
    // tangent bounds g from above and Newton converges from either start.)
    bool first = false;
    double g0 = 0.0, d0 = 1.0;
    if (have_guess && isfinite(guess) && guess > plo) {
        double dgL, dgR;
        const double gg = rside_f(L, guess, dgL) + rside_f(R, guess, dgR) + du;
        const double dg = dgL + dgR;
        if (fabs(gg) <= fabs(gg + dg * (p - guess))) {
            first = true;
            p = guess;
            g0 = gg;
            d0 = dg;
            if (used) *used = true;
        }
    }
    int it = 0;
    bool conv = false;
    while (it < maxit) {
        double gv, dv;
        if (first && it == 0) {
            gv = g0;
            dv = d0;
        } else {
            double dLf, dRf;
            gv = rside_f(L, p, dLf) + rside_f(R, p, dRf) + du;
            dv = dLf + dRf;
        }
        double pn = p - gv * rcp_nr(dv);
        if (pn <= plo) pn = plo + 0.5 * (p - plo);
        ++it;
        conv = fabs(pn - p) <= rtol * (pn - plo);
        p = pn;
        if (conv) break;
    }
    if (!conv) {
        double a = plo, b = fmax(pL, pR);
        for (int k = 0; k < 2000 && rside_f(L, b) + rside_f(R, b) + du < 0.0; ++k) b = plo + 2.0 * (b - plo);
        for (int k = 0; k < 400 && (b - a) > rtol * (b - plo); ++k) {
            const double m = 0.5 * (a + b);
            if (rside_f(L, m) + rside_f(R, m) + du < 0.0) a = m; else b = m;
        }
        p = 0.5 * (a + b);
        it = -it;
    }
    out[0] = p;
    out[1] = 0.5 * (uL + uR) + 0.5 * (rside_f(R, p) - rside_f(L, p));
    out[2] = rside_star_rho(L, gL, p);
    out[3] = rside_star_rho(R, gR, p);
    return it;
}

// Acoustic (linearised) guess and the admissible floor, for judging a
// learned guess.
__device__ __forceinline__ double riemann_g(double rL, double uL, double pL, double gL, double pcL,
                                           double rR, double uR, double pR, double gR, double pcR,
                                           double p)
{
    RSide L, R;
    rside_init(L, rL, uL, pL, gL, pcL);
    rside_init(R, rR, uR, pR, gR, pcR);
    return rside_f(L, p) + rside_f(R, p) + uR - uL;
}

// --------------------------------------------------------- atomics --------
__device__ __forceinline__ void atomic_max_nonneg(unsigned long long* addr, double v)
{
    atomicMax(addr, (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ void report_error(int* err, long long* err_cell, int code, long long cell)
{
    atomicCAS(err, 0, code);
    atomicMin(err_cell, cell);
}

// Lower cell c, upper cell cn and axis d of an interface face f = 3c + d
// (32-bit index arithmetic: grids hold at most 2^29 cells).  The face is an
// interface face, so a face on the upper domain boundary is periodic.
__device__ __forceinline__ void face_cells(int gnx, int gny, int gnz, uint32_t f, uint32_t& c, uint32_t& cn, int& d)
{
    const uint32_t nx = gnx, ny = gny, nz = gnz, sxy = nx * ny;
    c = f / 3u;
    d = (int)(f - 3u * c);
    const uint32_t k = c / sxy, r = c - k * sxy, j = r / nx, i = r - j * nx;
    if (d == 0) cn = i + 1 < nx ? c + 1 : c - (nx - 1);
    else if (d == 1) cn = j + 1 < ny ? c + nx : c - (ny - 1) * nx;
    else cn = k + 1 < nz ? c + sxy : c - (nz - 1) * sxy;
}

// Source index along one axis for a (possibly ghost) index i in [-2, n+1]
// under the boundary types of the two ends; 'mirror' is set when the ghost
// is a wall image (its normal velocity must be reversed).
__device__ __forceinline__ int bc_index(int i, int n, int blo, int bhi, bool& mirror)
{
    mirror = false;
    if (i < 0) {
        if (blo == 2) i += n;
        else if (blo == 1) { i = -1 - i; mirror = true; }
        else i = 0;
    } else if (i >= n) {
        if (bhi == 2) i -= n;
        else if (bhi == 1) { i = 2 * n - 1 - i; mirror = true; }
        else i = n - 1;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

}  // namespace m2c
