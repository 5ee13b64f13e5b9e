// m2c_eos.h -- general equations of state and the exact two-material
// Riemann solve for one problem (internal; device code, and plain C++ when
// M2C_HD is defined empty before inclusion).
//
// The interface fluxes of FIVER come from the exact solution of the 1D
// bimaterial Riemann problem (eq. 1DRiemannProblem); with EOS other than the
// stiffened gas the wave curves have no closed form, and the solve is the
// nested iteration the paper points to as the expensive part ("Spatial
// discretization", FIVER): an outer Newton iteration on the star pressure
// p*, and for each side and each trial pressure either a Hugoniot solve
// (shock) or an integration along the isentrope (rarefaction).
//
// Families (section "Equations of state" and its appendix): Noble-Abel
// stiffened gas (eq. NASG_EOS), Mie-Grueneisen with its compression, small
// tension and tensile-cutoff reference curves, JWL (eq. JWL_EOS, both
// exponentials decaying in the specific volume).
//
// For each side K and trial pressure p, the velocity change f_K(p)
// (u*_L = u_L - f_L, u*_R = u_R + f_R, F(p) = f_L + f_R + u_R - u_L = 0):
//   shock (p > p_K): the Hugoniot energy relation
//     H(v) = e(v, p) - e_K - (p + p_K)(v_K - v)/2 = 0
//   solved by safeguarded Newton in the specific volume v (linear in v for
//   NASG, so one step there), f = sqrt((p - p_K)(v_K - v));
//   rarefaction (p <= p_K): the isentrope with y = ln(p - floor) as the
//   independent variable, carrying s = ln(rho/rho_K) and f:
//   ds/dy = (p - floor)/(rho c^2), df/dy = c ds/dy, by classical RK4 at
//   steps of at most ds in y, straight to the trial pressure (no inner
//   iteration).  Along y the stiffened-gas isentrope is exactly linear
//   (ds/dy = 1/gamma), and the curves stay smooth where p approaches the
//   floor at a finite density (JWL states below the reference isentrope),
//   where a march in s would meet a logarithmic singularity.  The
//   Mie-Grueneisen branch points (eta = 0, eta_min) are stepped onto
//   exactly and each RK4 step stays on one branch.  The walk along each
//   isentrope is kept between outer iterations and continued from where it
//   stopped, so a solve integrates each rarefaction path about once.
// Sound speeds and the derivatives the Newton steps need are written per
// family in closed form of (rho, p): c^2 = dp/drho|_e + p dp/de|_rho / rho^2
// reduces to gamma (p + p_c) v^2 / (v - b) (NASG), rho_0 v^2 (p_R' -
// rho_0 Gamma_0 e_R' + Gamma_0 p) (MG) and ((1 + omega) p - T) v + T'
// (JWL, T the exponential terms), with no subtraction of large energies.
#pragma once
#include <math.h>
#include <stdint.h>

#include "m2c.h"

#ifndef M2C_HD
#define M2C_HD __device__
#endif
// the wave-curve code is inlined into every kernel that uses it: kernels
// that share one family's functions would otherwise call them, and a call
// keeps the solver's state on the stack
#define M2C_HDI M2C_HD __attribute__((always_inline)) inline

namespace m2c {
namespace eos {

// Prepared constants of one material (host-computed from m2c_eos).
//   NASG: k0 gamma, k1 p_c, k2 b, k3 e_c, k4 1/(gamma - 1), k5 gamma p_c
//   MG:   k0 rho_0, k1 Gamma_0, k2 s, k3 e_0, k4 eta_min, k5 K_0 = rho_0 c_0^2,
//         k6 rho_0 Gamma_0, k7 e_R(eta_min), k8 1/(rho_0 Gamma_0), k9 1/rho_0
//   JWL:  k0 omega, k1 A_1, k2 A_2, k3 R_1 rho_0, k4 R_2 rho_0,
//         k5 omega/(R_1 rho_0), k6 omega/(R_2 rho_0), k7 1/omega
//   all:  k10 smallest specific volume (b, (1 - 1/s)/rho_0 or 0), k11 floor
struct EosK {
    int fam;
    int pad;
    double k[12];
};
struct EosTable {
    int n;
    int pad;
    EosK m[M2C_EOS_MAX];
};
constexpr int KVMIN = 10, KFLOOR = 11;

// Sets of families as bit masks (bit f for family f = M2C_EOS_NASG, _MG,
// _JWL): the code below is compiled for a set S of families that the
// material may have.  A kernel that knows its materials' families keeps only
// their code; ALL dispatches on the material's tag at run time.
constexpr int FAM_ALL = 7;
constexpr int fam_set(int f) { return f < 0 ? FAM_ALL : 1 << f; }

// Family of material m as the code dispatches on it: a constant for a
// one-family set, a choice between the two families of a two-family set
// (so the compiler drops the third family's branch), the tag otherwise.
template <int S>
M2C_HD inline int fam_of(const EosK& m)
{
    static_assert(S >= 1 && S <= FAM_ALL, "family set");
    if constexpr (S == 1 || S == 2 || S == 4) return S == 1 ? 0 : (S == 2 ? 1 : 2);
    else if constexpr (S == 3) return m.fam == 1 ? 1 : 0;
    else if constexpr (S == 5) return m.fam == 2 ? 2 : 0;
    else if constexpr (S == 6) return m.fam == 2 ? 2 : 1;
    else return m.fam;
}

// Reciprocal from the hardware estimate refined by two Newton-Raphson
// steps: about one ulp for the positive normal arguments of the formulas
// below, at a fraction of the IEEE division sequence (the iterations of the
// solver evaluate the EOS many times per problem).  A host compilation of
// this header (CPU checks of the numerics) divides.
M2C_HD inline double rcp(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
#else
    return 1.0 / x;
#endif
}

// Mie-Grueneisen reference curves and their eta-derivatives.
struct Ref {
    double pR, eR, dpR, deR;
};
// Branch of the reference curves at eta: 0 compression, 1 small tension,
// 2 tensile cutoff.
M2C_HD inline int mg_branch(const EosK& m, double eta)
{
    return eta >= 0.0 ? 0 : (eta >= m.k[4] ? 1 : 2);
}

// Reference curves on a given branch (extended smoothly past its ends).
M2C_HD inline Ref mg_ref_on(const EosK& m, double eta, int br)
{
    const double ir0 = m.k[9], s = m.k[2], e0 = m.k[3], em = m.k[4], K0 = m.k[5];
    Ref r;
    if (br == 0) {
        const double a = rcp(1.0 - s * eta);
        r.pR = K0 * eta * a * a;
        r.dpR = K0 * (1.0 + s * eta) * a * a * a;
        r.eR = 0.5 * r.pR * eta * ir0 + e0;
        r.deR = 0.5 * (r.dpR * eta + r.pR) * ir0;
    } else if (br == 1) {
        r.pR = K0 * eta;
        r.dpR = K0;
        r.eR = 0.5 * K0 * eta * eta * ir0 + e0;
        r.deR = K0 * eta * ir0;
    } else {
        const double pmin = m.k[KFLOOR];
        r.pR = pmin;
        r.dpR = 0.0;
        r.eR = m.k[7] + pmin * ir0 * (eta - em);
        r.deR = pmin * ir0;
    }
    return r;
}

M2C_HD inline Ref mg_ref(const EosK& m, double eta)
{
    return mg_ref_on(m, eta, mg_branch(m, eta));
}

// JWL exponential terms T(rho) = sum_i A_i (1 - omega rho/(R_i rho_0))
// exp(-R_i rho_0 v) and dT/drho, with rho = 1/v given.
M2C_HD inline void jwl_terms_rho(const EosK& m, double v, double rho, double& T, double& dT)
{
    const double x1 = exp(-m.k[3] * v), x2 = exp(-m.k[4] * v);
    const double a1 = 1.0 - m.k[5] * rho, a2 = 1.0 - m.k[6] * rho;
    const double v2 = v * v;
    T = m.k[1] * a1 * x1 + m.k[2] * a2 * x2;
    dT = m.k[1] * x1 * (a1 * m.k[3] * v2 - m.k[5]) + m.k[2] * x2 * (a2 * m.k[4] * v2 - m.k[6]);
}

M2C_HD inline void jwl_terms(const EosK& m, double v, double& T, double& dT)
{
    jwl_terms_rho(m, v, rcp(v), T, dT);
}

// e(v, p)
template <int S = FAM_ALL>
M2C_HDI double eos_e(const EosK& m, double v, double p)
{
    if (fam_of<S>(m) == M2C_EOS_NASG) return (p + m.k[5]) * (v - m.k[2]) * m.k[4] + m.k[3];
    if (fam_of<S>(m) == M2C_EOS_MG) {
        const Ref r = mg_ref(m, 1.0 - m.k[0] * v);
        return r.eR + (p - r.pR) * m.k[8];
    }
    double T, dT;
    jwl_terms(m, v, T, dT);
    return (p - T) * v * m.k[7];
}

// p(v, e)
template <int S = FAM_ALL>
M2C_HDI double eos_p(const EosK& m, double v, double e)
{
    if (fam_of<S>(m) == M2C_EOS_NASG) return (e - m.k[3]) * rcp((v - m.k[2]) * m.k[4]) - m.k[5];
    if (fam_of<S>(m) == M2C_EOS_MG) {
        const Ref r = mg_ref(m, 1.0 - m.k[0] * v);
        return r.pR + m.k[6] * (e - r.eR);
    }
    double T, dT;
    jwl_terms(m, v, T, dT);
    return m.k[0] * e * rcp(v) + T;
}

// c^2(v, p)
template <int S = FAM_ALL>
M2C_HDI double eos_c2(const EosK& m, double v, double p)
{
    if (fam_of<S>(m) == M2C_EOS_NASG) return m.k[0] * (p + m.k[1]) * v * v * rcp(v - m.k[2]);
    if (fam_of<S>(m) == M2C_EOS_MG) {
        const Ref r = mg_ref(m, 1.0 - m.k[0] * v);
        return m.k[0] * v * v * (r.dpR - m.k[6] * r.deR + m.k[1] * p);
    }
    double T, dT;
    jwl_terms(m, v, T, dT);
    return ((1.0 + m.k[0]) * p - T) * v + dT;
}

// c^2(v, p) with the Mie-Grueneisen branch given (other families: eos_c2).
template <int S = FAM_ALL>
M2C_HDI double eos_c2_on(const EosK& m, double v, double p, int br)
{
    if (fam_of<S>(m) == M2C_EOS_MG) {
        const Ref r = mg_ref_on(m, 1.0 - m.k[0] * v, br);
        return m.k[0] * v * v * (r.dpR - m.k[6] * r.deR + m.k[1] * p);
    }
    return eos_c2<S>(m, v, p);
}

// de/dv at constant p, and de/dp at constant v.
template <int S = FAM_ALL>
M2C_HDI void eos_ederiv(const EosK& m, double v, double p, double& ev, double& ep)
{
    if (fam_of<S>(m) == M2C_EOS_NASG) {
        ev = (p + m.k[5]) * m.k[4];
        ep = (v - m.k[2]) * m.k[4];
    } else if (fam_of<S>(m) == M2C_EOS_MG) {
        const Ref r = mg_ref(m, 1.0 - m.k[0] * v);
        ev = r.dpR * (m.k[0] * m.k[8]) - m.k[0] * r.deR;
        ep = m.k[8];
    } else {
        double T, dT;
        jwl_terms(m, v, T, dT);
        ev = (p - T + dT * rcp(v)) * m.k[7];
        ep = v * m.k[7];
    }
}

// One side of the problem and its wave-curve state between outer iterations.
struct Side {
    double rho, v, p, e, c;        // state K
    double fl;                     // pressure floor of the material
    double s, y, f;                // current point of the isentrope walk
    double vh;                     // last Hugoniot volume (0: none yet)
    double jC;                     // JWL: constant of the isentrope through K
};

struct Wave {
    double f, df, rho;
};

// One classical RK4 step of the isentrope over y = ln(p - floor), from
// (y, s, f) to y + h: ds/dy = (p - floor)/(rho c^2), df/dy = c ds/dy.
// False where c^2 <= 0 (outside the convex part of the EOS).
template <int S = FAM_ALL>
M2C_HDI bool rk4_y(const EosK& m, const Side& K, double y, double h, double& s, double& f)
{
    double ks[4], kf[4];
    // every stage on one Mie-Grueneisen branch: a step never spans a branch
    // point (the walk ends steps on them), but a stage predictor near one may
    // overshoot it, and a step may start on one.  The branch is the one a
    // quarter step ahead (s moves with y, ds/dy > 0).
    int br = 0;
    if (fam_of<S>(m) == M2C_EOS_MG) {
        const double rho0 = K.rho * exp(s), q0 = exp(y);
        const double c20 = eos_c2<S>(m, rcp(rho0), K.fl + q0);
        if (!(c20 > 0.0)) return false;
        const double probe = s + 0.25 * h * q0 * rcp(rho0 * c20);
        br = mg_branch(m, 1.0 - m.k[0] * rcp(K.rho * exp(probe)));
    }
    for (int j = 0; j < 4; ++j) {
        const double a = j == 0 ? 0.0 : (j == 3 ? h : 0.5 * h);
        const double ss = j == 0 ? s : s + a * ks[j - 1];
        const double q = exp(y + a), rho = K.rho * exp(ss);
        const double c2 = eos_c2_on<S>(m, rcp(rho), K.fl + q, br);
        if (!(c2 > 0.0) || !isfinite(c2)) return false;
        ks[j] = q * rcp(rho * c2);
        kf[j] = ks[j] * sqrt(c2);
    }
    s += h * (ks[0] + 2.0 * ks[1] + 2.0 * ks[2] + ks[3]) * (1.0 / 6.0);
    f += h * (kf[0] + 2.0 * kf[1] + 2.0 * kf[2] + kf[3]) * (1.0 / 6.0);
    return isfinite(s) && isfinite(f);
}

// Walk the side's isentrope from its current point to y = Y in steps of at
// most hmax.  For Mie-Grueneisen the branch points of the reference curves
// (eta = 0 and eta = eta_min, where the slope of c^2 jumps) are stepped onto
// exactly -- a Newton iteration on the length of the step that ends there --
// so that no RK4 step spans one and each keeps its order.
template <int S = FAM_ALL>
M2C_HDI bool walk(const EosK& m, Side& K, double Y, double hmax)
{
    double kink[2] = {INFINITY, INFINITY};
    if (fam_of<S>(m) == M2C_EOS_MG) {
        kink[0] = log(m.k[0] / K.rho);
        kink[1] = log(m.k[0] / ((1.0 - m.k[4]) * K.rho));
    }
    for (int guard = 0; guard < 100000; ++guard) {
        const double rem = Y - K.y;
        if (rem == 0.0) return true;
        if (fam_of<S>(m) == M2C_EOS_MG) {
            // below eta_min the isentrope is known in closed form: there
            // c^2 = rho_0 Gamma_0 (p - p_min) v^2, so ds/dy = rho/(rho_0
            // Gamma_0), i.e. exp(-s) falls linearly in y, and df/dy =
            // sqrt((p - p_min)/(rho_0 Gamma_0))
            const double dir = rem > 0.0 ? 1.0 : -1.0;
            if (mg_branch(m, 1.0 - m.k[0] / (K.rho * exp(K.s + dir * 1e-10))) == 2) {
                const double a = K.rho * m.k[8];
                double yend = Y;
                bool to_kink = false;
                if (dir > 0.0 && isfinite(kink[1])) {
                    const double yk = K.y + (exp(-K.s) - exp(-kink[1])) / a;
                    if (yk < Y) {
                        yend = yk;
                        to_kink = true;
                    }
                }
                const double em = exp(-K.s) - a * (yend - K.y);
                if (!(em > 0.0)) return false;
                K.f += 2.0 * sqrt(m.k[8]) * (exp(0.5 * yend) - exp(0.5 * K.y));
                K.s = to_kink ? kink[1] + 1e-12 * (1.0 + fabs(kink[1])) : -log(em);
                K.y = yend;
                if (to_kink) kink[1] = INFINITY;
                continue;
            }
            if (mg_branch(m, 1.0 - m.k[0] / (K.rho * exp(K.s + dir * 1e-10))) == 1) {
                // small tension: along the isentrope e - e_R(eta) decays as
                // exp(-rho_0 Gamma_0 v) (de = -p dv with p_R = K_0 eta, e_R
                // quadratic), so p(v) = K_0 (1 - rho_0 v) + (p_a - K_0 eta_a)
                // exp(-rho_0 Gamma_0 (v - v_a)); v at the target pressure by
                // Newton, f by Gauss-Legendre; the branch ends (eta_min when
                // p falls, eta = 0 when it rises) are stepped onto exactly
                const double r0 = m.k[0], G = m.k[6], K0 = m.k[5];
                const double va = K.v * exp(-K.s);
                const double ga = (K.fl + exp(K.y)) - K0 * (1.0 - r0 * va);     // rho_0 Gamma_0 (e - e_R)
                auto P = [&](double v) { return K0 * (1.0 - r0 * v) + ga * exp(-G * (v - va)); };
                auto mdP = [&](double v) { return K0 * r0 + G * ga * exp(-G * (v - va)); };   // -dp/dv
                const int j = dir < 0.0 ? 1 : 0;
                const double vk = dir < 0.0 ? (1.0 - m.k[4]) / r0 : 1.0 / r0;
                const double pt = K.fl + exp(Y), pk = P(vk);
                const bool to_kink = dir < 0.0 ? pt <= pk : pt >= pk;
                double v = vk;
                if (!to_kink) {
                    double lo = fmin(va, vk), hi = fmax(va, vk);      // P(lo) > pt > P(hi)
                    v = va;
                    bool conv = false;
                    for (int it = 0; it < 100; ++it) {
                        const double d = mdP(v);
                        if (!(d > 0.0)) return false;
                        const double r = P(v) - pt;
                        if (r > 0.0) lo = v; else hi = v;
                        // converged (before the bracket test): a step of a few
                        // ulp, or a bracket closed to that width
                        if (fabs(r / d) <= 1e-15 * v || hi - lo <= 4e-16 * v) {
                            v += r / d;
                            v = fmin(fmax(v, lo), hi);
                            conv = true;
                            break;
                        }
                        double vn = v + r / d;
                        if (!(vn > lo && vn < hi)) vn = 0.5 * (lo + hi);
                        v = vn;
                    }
                    if (!conv) return false;
                }
                // f -= int_{va}^{v} sqrt(-dp/dv) dv
                {
                    const double gx[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267,
                                          0.9602898564975363};
                    const double gw[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745,
                                          0.1012285362903763};
                    const int np = 1 + (int)(G * fabs(v - va) / 0.5);
                    const double hv = (v - va) / np;
                    double I = 0.0;
                    for (int i = 0; i < np; ++i) {
                        const double vm = va + (i + 0.5) * hv;
                        for (int q = 0; q < 8; ++q) {
                            const double d = mdP(vm + 0.5 * hv * (q < 4 ? -gx[q] : gx[q - 4]));
                            if (!(d > 0.0)) return false;
                            I += 0.5 * hv * gw[q & 3] * sqrt(d);
                        }
                    }
                    K.f -= I;
                }
                if (to_kink) {
                    K.s = kink[j] + (dir < 0.0 ? -1e-12 : 1e-12) * (1.0 + fabs(kink[j]));
                    if (!isfinite(kink[j])) K.s = log(K.v / vk);
                    K.y = log(pk - K.fl);
                    kink[j] = INFINITY;
                } else {
                    K.s = log(K.v / v);
                    K.y = Y;
                }
                continue;
            }
        }
        const int n = (int)ceil(fabs(rem) / hmax);
        const double h = rem / (double)n;
        double s = K.s, f = K.f;
        if (!rk4_y<S>(m, K, K.y, h, s, f)) return false;
        int crossed = -1;
        for (int j = 0; j < 2; ++j)
            if ((K.s - kink[j]) * (s - kink[j]) < 0.0) crossed = j;
        if (crossed < 0) {
            K.y = n == 1 ? Y : K.y + h;
            K.s = s;
            K.f = f;
            continue;
        }
        // shorten the step so that it ends on the branch point: root of
        // g(hk) = s(hk) - s_kink on [0, h] by the Illinois variant of
        // regula falsi (c^2, and with it the slope of g, may jump there)
        const double sk = kink[crossed];
        double a = 0.0, ga = K.s - sk, b = h, gb = s - sk;
        double hk = b, sk_got = s, fk_got = f;
        int side = 0;
        for (int it = 0; it < 80; ++it) {
            hk = (a * gb - b * ga) / (gb - ga);
            sk_got = K.s;
            fk_got = K.f;
            if (!rk4_y<S>(m, K, K.y, hk, sk_got, fk_got)) return false;
            const double g = sk_got - sk;
            if (fabs(g) <= 1e-14 * (1.0 + fabs(sk)) || fabs(b - a) <= 1e-15 * fabs(h)) break;
            if ((g < 0.0) == (gb < 0.0)) {
                b = hk;
                gb = g;
                if (side == -1) ga *= 0.5;
                side = -1;
            } else {
                a = hk;
                ga = g;
                if (side == 1) gb *= 0.5;
                side = 1;
            }
        }
        // land just beyond the branch point, so that the first stage of the
        // next step sees the branch the walk is entering (c^2 itself jumps
        // at eta_min); the offset is far below the step error
        const double dir = s > K.s ? 1.0 : -1.0;
        K.y += hk;
        K.s = sk_got + dir * 1e-12 * (1.0 + fabs(sk));
        K.f = fk_got;
        kink[crossed] = INFINITY;            // passed
    }
    return false;
}

// JWL isentropes in closed form: along the isentrope through K
//   p_s(v) = A_1 exp(-a_1 v) + A_2 exp(-a_2 v) + C v^-(1 + omega),  a_i = R_i rho_0,
// with C fixed by p_s(v_K) = p_K (the homogeneous part of de = -p dv for
// eq. JWL_EOS), so rho^2 c^2 = -dp_s/dv and f = -int_{v_K}^{v} sqrt(-p_s') dv.
M2C_HD inline void jwl_ps(const EosK& m, double C, double v, double& ps, double& dps)
{
    const double x1 = exp(-m.k[3] * v), x2 = exp(-m.k[4] * v);
    const double vp = exp(-(1.0 + m.k[0]) * log(v));
    ps = m.k[1] * x1 + m.k[2] * x2 + C * vp;
    dps = -m.k[1] * m.k[3] * x1 - m.k[2] * m.k[4] * x2 - (1.0 + m.k[0]) * C * vp / v;
}

// int_{v0}^{v1} sqrt(-p_s'(v)) dv: 8-point Gauss-Legendre on panels of at
// most 0.1 in ln v; where both exponentials are below e^-40 of their
// amplitude the integrand is the power law sqrt((1 + omega) C) v^-(1 + omega/2)
// and the rest is integrated in closed form.  False where -p_s' <= 0.
M2C_HDI bool jwl_quad(const EosK& m, double C, double v0, double v1, double& I)
{
    const double gx[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267, 0.9602898564975363};
    const double gw[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763};
    const double w = m.k[0];
    const double ve = 40.0 / fmin(m.k[3], m.k[4]);        // beyond: exponentials negligible
    const double lo = fmin(v0, v1), hi = fmax(v0, v1);
    double acc = 0.0;                                   // integral over [lo, hi]
    if (hi > ve) {                                      // tail [max(lo, ve), hi] in closed form
        if (!(C > 0.0)) return false;
        const double t0 = fmax(lo, ve);
        // int v^-(1 + w/2) dv = -(2/w) v^(-w/2)
        acc += sqrt((1.0 + w) * C) * (2.0 / w) * (exp(-0.5 * w * log(t0)) - exp(-0.5 * w * log(hi)));
    }
    if (lo < ve) {                                      // body [lo, min(hi, ve)] by quadrature
        const double u0 = log(lo), u1 = log(fmin(hi, ve));
        const int n = (int)ceil((u1 - u0) / 0.1);
        const double hu = n > 0 ? (u1 - u0) / n : 0.0;
        for (int i = 0; i < n; ++i) {
            const double um = u0 + (i + 0.5) * hu;
            double sum = 0.0;
            for (int j = 0; j < 8; ++j) {
                const double u = um + 0.5 * hu * (j < 4 ? -gx[j] : gx[j - 4]);
                const double v = exp(u);
                double ps, dps;
                jwl_ps(m, C, v, ps, dps);
                if (!(dps < 0.0)) return false;
                sum += gw[j & 3] * sqrt(-dps) * v;
            }
            acc += 0.5 * hu * sum;
        }
    }
    I = v1 >= v0 ? acc : -acc;
    return isfinite(I);
}

// f_K(p) for p <= p_K on a JWL side: v* from p_s(v*) = p by safeguarded
// Newton in ln v, f continued from the last point of this isentrope.
M2C_HDI bool jwl_rarefaction(const EosK& m, Side& K, double p, Wave& w)
{
    const double C = K.jC;
    double lo = K.v, hi = INFINITY;                     // p_s(lo) >= p > p_s(hi)
    double v = K.v * exp(-K.s);                         // start from the last point
    if (!(v > lo)) v = K.v * exp(log(K.p / p) / (1.0 + m.k[0]));
    bool ok = false;
    double ps = 0.0, dps = 0.0;
    for (int it = 0; it < 200; ++it) {
        jwl_ps(m, C, v, ps, dps);
        if (!(dps < 0.0) || !isfinite(ps)) {            // past the convex part
            hi = v;
            v = isinf(hi) ? 0.5 * (lo + v) : sqrt(lo * hi);
            continue;
        }
        if (ps > p) lo = v; else hi = v;
        const double du = (p - ps) / (dps * v);
        // converged (before the bracket test): ln v to 1e-14 (the power
        // term is evaluated as exp(-(1 + omega) ln v), whose rounding grows
        // with ln v), or a bracket closed to a few ulp
        if (fabs(du) <= 1e-14 || (isfinite(hi) && hi - lo <= 4e-16 * hi)) {
            v *= exp(du);
            v = fmin(fmax(v, lo), hi);
            ok = true;
            break;
        }
        double vn = v * exp(du);
        if (!(vn > lo && vn < hi)) vn = isinf(hi) ? 2.0 * v : sqrt(lo * hi);
        v = vn;
    }
    if (!ok) return false;
    jwl_ps(m, C, v, ps, dps);
    if (!(dps < 0.0)) return false;
    double I;
    const double vlast = K.v * exp(-K.s);
    if (!jwl_quad(m, C, vlast, v, I)) return false;
    K.f -= I;
    K.s = log(K.v / v);
    w.f = K.f;
    w.rho = 1.0 / v;
    w.df = 1.0 / sqrt(-dps);                            // 1/(rho c)
    return true;
}

// f_K(p) for p <= p_K: the isentrope walked to y = ln(p - floor).
template <int S = FAM_ALL>
M2C_HDI bool rarefaction(const EosK& m, Side& K, double p, double hmax, Wave& w)
{
    if (fam_of<S>(m) == M2C_EOS_JWL) {
        if (p == K.p) {
            w.f = 0.0;
            w.rho = K.rho;
            w.df = 1.0 / (K.rho * K.c);
            return true;
        }
        return jwl_rarefaction(m, K, p, w);
    }
    if (fam_of<S>(m) == M2C_EOS_NASG) {
        // closed form: along the isentrope (p + p_c)(v - b)^gamma is
        // constant, and integrating dp/(rho c) with c^2 = gamma (p + p_c)
        // v^2/(v - b) gives f = 2 c_K (1 - b rho_K)/(gamma - 1)
        // ((p + p_c)/(p_K + p_c))^((gamma - 1)/(2 gamma)) - 1)
        const double g = m.k[0], pc = m.k[1], b = m.k[2];
        const double qb = p + pc, qK = K.p + pc;
        if (!(qb > 0.0)) return false;
        // ln((p + p_c)/(p_K + p_c)), accurate near 0 and near cavitation
        const double lr = fabs(p - K.p) < 0.5 * qK ? log1p((p - K.p) / qK) : log(qb / qK);
        const double VK = K.v - b, V = VK * exp(-lr / g);
        w.f = 2.0 * K.c * (VK / K.v) / (g - 1.0) * expm1(0.5 * (g - 1.0) / g * lr);
        w.rho = 1.0 / (V + b);
        w.df = sqrt(V / (g * qb));                        // 1/(rho c)
        return true;
    }
    const Side good = K;
    if (!walk<S>(m, K, log(p - K.fl), hmax)) {
        K = good;
        return false;
    }
    const double r = K.rho * exp(K.s);
    const double c2 = eos_c2<S>(m, 1.0 / r, p);
    if (!(c2 > 0.0)) {
        K = good;
        return false;
    }
    w.f = K.f;
    w.rho = r;
    w.df = 1.0 / (r * sqrt(c2));
    return true;
}

// f_K(p) for p > p_K: Hugoniot volume by Newton in v, bracketed by
// (v_min, v_K].
template <int S = FAM_ALL>
M2C_HDI bool shock(const EosK& m, Side& K, double p, Wave& w)
{
    const double vK = K.v, half = 0.5 * (p + K.p);
    double lo = m.k[KVMIN], hi = vK;
    double v = K.vh;
    if (!(v > lo && v < hi)) {
        v = vK - (p - K.p) * vK * vK / (K.c * K.c);       // acoustic estimate
        if (!(v > lo)) v = lo + 0.5 * (hi - lo);
    }
    bool ok = false;
    for (int it = 0; it < 100; ++it) {
        const double H = eos_e<S>(m, v, p) - K.e - half * (vK - v);
        double ev, ep;
        eos_ederiv<S>(m, v, p, ev, ep);
        if (!(ev + half > 0.0)) {
            // H does not increase here: a stretch below the branch the
            // shock takes (JWL has a second, unphysical root at strong
            // compression, which an acoustic start far above p_K can pass);
            // the physical root is the largest one, above v
            lo = v;
            v = 0.5 * (lo + hi);
            continue;
        }
        if (H > 0.0) hi = v; else lo = v;
        const double step = H * rcp(ev + half);
        // a converged Newton step is taken before the bracket is consulted
        // (a step below rounding would otherwise fail the bracket test and
        // restart a bisection)
        if (fabs(step) <= 1e-15 * v || hi - lo <= 4e-16 * hi) {
            v -= step;
            v = fmin(fmax(v, lo), hi);
            ok = true;
            break;
        }
        double vn = v - step;
        if (!(vn > lo && vn < hi)) vn = 0.5 * (lo + hi);
        v = vn;
    }
    // (v = v_K: a shock too weak for the volume to change in FP64)
    if (!ok || !(v > m.k[KVMIN]) || !(v <= vK)) return false;
    K.vh = v;
    const double dp = p - K.p, dvol = vK - v;
    w.f = sqrt(dp * dvol);
    w.rho = 1.0 / v;
    // slope of f along the Hugoniot: v'(p) = -H_p / H_v
    double ev, ep;
    eos_ederiv<S>(m, v, p, ev, ep);
    const double vp = -(ep - 0.5 * dvol) / (ev + half);
    // (the acoustic slope where the shock is too weak for the quotient)
    w.df = dp > 1e-10 * (K.p - K.fl) ? (dvol - dp * vp) / (2.0 * w.f) : 1.0 / (K.rho * K.c);
    return true;
}

template <int S = FAM_ALL>
M2C_HDI bool wave(const EosK& m, Side& K, double p, double hmax, Wave& w)
{
    return p > K.p ? shock<S>(m, K, p, w) : rarefaction<S>(m, K, p, hmax, w);
}

M2C_HD inline double floor_margin(const Side& K)
{
    return 1e-12 * (K.p - K.fl) + 1e-6 * fabs(K.fl);
}

template <int S = FAM_ALL>
M2C_HDI bool side_init(const EosK& m, double rho, double p, Side& K)
{
    K.fl = m.k[KFLOOR];
    if (!(rho > 0.0) || !isfinite(rho) || !isfinite(p)) return false;
    K.rho = rho;
    K.v = 1.0 / rho;
    K.p = p;
    if (!(K.v > m.k[KVMIN])) return false;
    if (!(p - K.fl > floor_margin(K))) return false;
    const double c2 = eos_c2<S>(m, K.v, p);
    if (!(c2 > 0.0) || !isfinite(c2)) return false;
    K.c = sqrt(c2);
    K.e = eos_e<S>(m, K.v, p);
    K.s = 0.0;
    K.y = log(p - K.fl);
    K.f = 0.0;
    K.vh = 0.0;
    K.jC = 0.0;
    if (fam_of<S>(m) == M2C_EOS_JWL) {
        const double vK = K.v;
        K.jC = (p - m.k[1] * exp(-m.k[3] * vK) - m.k[2] * exp(-m.k[4] * vK)) * exp((1.0 + m.k[0]) * log(vK));
    }
    return true;
}

// Bisection point of the star-pressure bracket (lo, hi): geometric in the
// distance from the higher floor when the bracket spans decades (near
// cavitation the root sits many decades below the initial pressures),
// arithmetic otherwise.
M2C_HD inline double bisect(double lo, double hi, double base)
{
    const double a = lo - base, b = hi - base;
    return b > 1e3 * a ? base + sqrt(a * b) : 0.5 * (lo + hi);
}

// One problem set up for the outer iteration: both sides' states and the
// acoustic start.
struct Pair {
    Side L, R;
    double uL, uR, du;
    double pfl;                    // lowest admissible trial pressure
    double base;                   // the higher floor (reference of the geometric bisection)
    double pac;                    // acoustic start, kept above pfl
};

// Set-up of q = (rho_L, u_L, p_L, rho_R, u_R, p_R) of materials mL, mR;
// false for an inadmissible input.
template <int SL = FAM_ALL, int SR = FAM_ALL>
M2C_HDI bool pair_init(const EosK& mL, const EosK& mR, const double* q, Pair& P)
{
    if (!side_init<SL>(mL, q[0], q[2], P.L) || !side_init<SR>(mR, q[3], q[5], P.R)) return false;
    P.uL = q[1];
    P.uR = q[4];
    P.du = P.uR - P.uL;
    P.pfl = fmax(P.L.fl + floor_margin(P.L), P.R.fl + floor_margin(P.R));
    P.base = fmax(P.L.fl, P.R.fl);
    const double zL = P.L.rho * P.L.c, zR = P.R.rho * P.R.c;
    double p = (zR * P.L.p + zL * P.R.p - zL * zR * P.du) / (zL + zR);
    if (!(p > P.pfl)) p = P.pfl + 0.5 * (fmin(P.L.p, P.R.p) - P.pfl);
    P.pac = p;
    return true;
}

// Outer iteration of a set-up problem: res = (p*, u*, rho*_L, rho*_R) or
// NaN; returns the Newton steps (negative after a bisection step; 0: no
// star state).  guess: a candidate start (NaN: none).  F and F' are
// evaluated there (they become the first Newton step when it is kept, and
// F's sign narrows the bracket either way); the candidate is kept unless
// the tangent there predicts a smaller |F| at the acoustic start.  F is
// increasing in p, so Newton converges from either start, and the answer
// does not depend on the candidate beyond the stopping tolerance.  *used
// (nullable): the candidate was the start.
template <int SL = FAM_ALL, int SR = FAM_ALL>
M2C_HDI int pair_solve(const EosK& mL, const EosK& mR, Pair& P, double rtol, int maxit, double hmax,
                             double guess, double* res, bool* used = nullptr)
{
    for (int k = 0; k < 4; ++k) res[k] = __builtin_nan("");
    if (used) *used = false;
    Side& L = P.L;
    Side& R = P.R;
    const double uL = P.uL, uR = P.uR, du = P.du, pfl = P.pfl, base = P.base;
    double p = P.pac;
    double lo = pfl, hi = INFINITY;
    bool bis = false, floor_checked = false, conv = false, first = false;
    Wave wl, wr;
    if (guess > pfl && isfinite(guess)) {
        Wave a, b;
        if (wave<SL>(mL, L, guess, hmax, a) && wave<SR>(mR, R, guess, hmax, b)) {
            const double F = a.f + b.f + du, dF = a.df + b.df;
            if (F < 0.0) lo = guess; else hi = guess;
            if (fabs(F) <= fabs(F + dF * (p - guess))) {
                p = guess;
                wl = a;
                wr = b;
                first = true;
                if (used) *used = true;
            }
        }
        // (a candidate where a wave curve cannot be evaluated is dropped)
    }
    int its;
    for (its = 1; its <= maxit; ++its) {
        if (!(first && its == 1) && (!wave<SL>(mL, L, p, hmax, wl) || !wave<SR>(mR, R, p, hmax, wr))) {
            // p lies below where an isentrope ends (c^2 reaches zero
            // before the floor): it bounds the bracket from below
            lo = fmax(lo, p);
            p = isinf(hi) ? 0.5 * (p + fmax(L.p, R.p)) : bisect(lo, hi, base);
            bis = true;
            continue;
        }
        const double F = wl.f + wr.f + du;
        if (F < 0.0) lo = fmax(lo, p); else hi = fmin(hi, p);
        double pn = p - F * rcp(wl.df + wr.df);
        const double tol = rtol * fmin(p - L.fl, p - R.fl);
        if (fabs(pn - p) <= tol && pn > pfl) {
            p = pn;
            conv = true;
            break;
        }
        // F at the rounding level of its terms, or a bracket closed to a
        // few ulps: p is as good as FP64 resolves it (near cavitation
        // the stopping rule above asks for more)
        if (fabs(F) <= 8e-16 * (fabs(wl.f) + fabs(wr.f) + fabs(uL) + fabs(uR)) ||
            (isfinite(hi) && hi - lo <= 4e-16 * fabs(hi))) {
            conv = true;
            break;
        }
        if (!(pn > lo && pn < hi)) {
            if (!(pn > lo) && lo == pfl && !floor_checked) {
                // the Newton step leaves the admissible range: is
                // there a star state above the floor at all?
                floor_checked = true;
                Wave a, b;
                if (!wave<SL>(mL, L, pfl, hmax, a) || !wave<SR>(mR, R, pfl, hmax, b)) break;
                if (a.f + b.f + du > 0.0) break;          // cavitation
            }
            pn = isinf(hi) ? p + fmax(p - pfl, fabs(p) + 1.0) : bisect(lo, hi, base);
            bis = true;
        }
        p = pn;
    }
    if (conv && wave<SL>(mL, L, p, hmax, wl) && wave<SR>(mR, R, p, hmax, wr)) {
        res[0] = p;
        res[1] = 0.5 * (uL - wl.f + uR + wr.f);
        res[2] = wl.rho;
        res[3] = wr.rho;
        return bis ? -its : its;
    }
    return 0;
}

// One problem: q = (rho_L, u_L, p_L, rho_R, u_R, p_R) of materials mL, mR
// from the acoustic start; res and the return value as for pair_solve (0
// also for an inadmissible input).
template <int SL = FAM_ALL, int SR = FAM_ALL>
M2C_HDI int solve_pair(const EosK& mL, const EosK& mR, const double* q, double rtol, int maxit, double hmax,
                             double* res)
{
    Pair P;
    if (!pair_init<SL, SR>(mL, mR, q, P)) {
        for (int k = 0; k < 4; ++k) res[k] = __builtin_nan("");
        return 0;
    }
    return pair_solve<SL, SR>(mL, mR, P, rtol, maxit, hmax, __builtin_nan(""), res);
}

// The same for materials ml, mr of a table (0 for an index out of range).
M2C_HD inline int solve_one(const EosTable& tab, int ml, int mr, const double* q, double rtol, int maxit,
                            double hmax, double* res)
{
    if (ml < 0 || ml >= tab.n || mr < 0 || mr >= tab.n) {
        for (int k = 0; k < 4; ++k) res[k] = __builtin_nan("");
        return 0;
    }
    return solve_pair(tab.m[ml], tab.m[mr], q, rtol, maxit, hmax, res);
}

// Table of prepared constants; false for invalid parameters.
inline bool prepare(int32_t nmat, const m2c_eos* eos, EosTable& t)
{
    if (nmat < 1 || nmat > M2C_EOS_MAX || !eos) return false;
    t = EosTable{};
    t.n = nmat;
    for (int i = 0; i < nmat; ++i) {
        const double* a = eos[i].prm;
        for (int j = 0; j < 7; ++j)
            if (!isfinite(a[j])) return false;
        EosK& m = t.m[i];
        m.fam = eos[i].family;
        double* k = m.k;
        switch (m.fam) {
            case M2C_EOS_NASG:
                if (!(a[0] > 1.0) || !(a[1] >= 0.0) || !(a[2] >= 0.0)) return false;
                k[0] = a[0];
                k[1] = a[1];
                k[2] = a[2];
                k[3] = a[3];
                k[4] = 1.0 / (a[0] - 1.0);
                k[5] = a[0] * a[1];
                k[KVMIN] = a[2];
                k[KFLOOR] = -a[1];
                break;
            case M2C_EOS_MG: {
                if (!(a[0] > 0.0) || !(a[1] > 0.0) || !(a[2] > 0.0) || !(a[3] >= 0.0) || !(a[5] < 0.0))
                    return false;
                const double K0 = a[0] * a[1] * a[1];
                k[0] = a[0];
                k[1] = a[2];
                k[2] = a[3];
                k[3] = a[4];
                k[4] = a[5];
                k[5] = K0;
                k[6] = a[0] * a[2];
                k[7] = 0.5 * K0 * a[5] * a[5] / a[0] + a[4];
                k[8] = 1.0 / (a[0] * a[2]);
                k[9] = 1.0 / a[0];
                k[KVMIN] = a[3] > 1.0 ? (1.0 - 1.0 / a[3]) / a[0] : 0.0;
                k[KFLOOR] = K0 * a[5];
                break;
            }
            case M2C_EOS_JWL:
                if (!(a[0] > 0.0) || !(a[3] > 0.0) || !(a[4] > 0.0) || !(a[5] > 0.0)) return false;
                k[0] = a[0];
                k[1] = a[1];
                k[2] = a[2];
                k[3] = a[3] * a[5];
                k[4] = a[4] * a[5];
                k[5] = a[0] / (a[3] * a[5]);
                k[6] = a[0] / (a[4] * a[5]);
                k[7] = 1.0 / a[0];
                k[KVMIN] = 0.0;
                k[KFLOOR] = 0.0;
                break;
            default:
                return false;
        }
    }
    return true;
}

}  // namespace eos
}  // namespace m2c
