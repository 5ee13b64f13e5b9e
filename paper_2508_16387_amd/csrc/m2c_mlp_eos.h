// m2c_mlp_eos.h -- the learned start of the general-EOS outer iteration
// (internal; device code): its features, the near-equilibrium test and the
// family pairs that take it.  Used by the point solver (k_riemann_eos.hip)
// and by the general-EOS FIVER kernel of the grid step (k_interface.hip).
#pragma once
#include <math.h>

#include "m2c.h"
#include "m2c_eos.h"

namespace m2c {

// Learned start of the general-EOS outer iteration: the network of the
// stiffened-gas guess (8 -> 64 -> 64 -> 1) with features of a set-up
// problem in the orientation it is solved in (lower family on the left):
//   x0 = ln(rho_L/rho_R)/2, x1 = (u_R - u_L)/U, x2 = ln(a_L/a_R)/2,
//   x3 = ln(rho_L c_L^2/a_L), x4 = ln(rho_R c_R^2/a_R) (the sides'
//   effective isentropic exponents), x5 = ln((p_ac - p_lo)/P) (the acoustic
//   start), x6, x7 = family - 1 of each side,
// with p_lo the higher floor, a_K = p_K - p_lo, P = sqrt(a_L a_R) and
// U = sqrt(P / sqrt(rho_L rho_R)); the target is y = ln((p* - p_lo)/P), so
// the guess p_lo + P exp(y) lies above both floors for any y.  False where
// a side's pressure does not exceed the other side's floor.
__device__ __forceinline__ bool eos_features(const eos::Pair& P, int famL, int famR, float x[8], double& plo,
                                             double& Pn)
{
    plo = P.base;
    const double aL = P.L.p - plo, aR = P.R.p - plo;
    if (!(aL > 0.0) || !(aR > 0.0)) return false;
    Pn = sqrt(aL * aR);
    const double U = sqrt(Pn / sqrt(P.L.rho * P.R.rho));
    x[0] = (float)(0.5 * log(P.L.rho / P.R.rho));
    x[1] = (float)(P.du / U);
    x[2] = (float)(0.5 * log(aL / aR));
    x[3] = (float)log(P.L.rho * P.L.c * P.L.c / aL);
    x[4] = (float)log(P.R.rho * P.R.c * P.R.c / aR);
    x[5] = (float)log((P.pac - plo) / Pn);
    x[6] = (float)(famL - 1);
    x[7] = (float)(famR - 1);
    return true;
}

// Family pairs whose solves take the learned start: a JWL side and no
// Mie-Grueneisen side.  Measured: the JWL isentrope's Riemann invariant is a
// quadrature, so each outer step saved pays for the network (1.24x on
// detonation products / air); with NASG on both sides a step is cheaper than
// the network (0.93x), and with a Mie-Grueneisen side the cost is the length
// of the RK4 walks along the isentrope, which a start beyond p* or a
// rejected candidate lengthens (0.77x on copper / tantalum).
__host__ __device__ constexpr bool learned_pair(int fa, int fb)
{
    return (fa == M2C_EOS_JWL || fb == M2C_EOS_JWL) && fa != M2C_EOS_MG && fb != M2C_EOS_MG;
}

// Near equilibrium (pressures within 1e-3 of the smaller a_K, velocities
// within 1e-3 of the smaller sound speed): the acoustic start is then close
// to exact and the network is not consulted.
__device__ __forceinline__ bool eos_near_equilibrium(const eos::Pair& P)
{
    const double aL = P.L.p - P.base, aR = P.R.p - P.base, du2 = P.du * P.du;
    return fabs(P.L.p - P.R.p) <= 1e-3 * fmin(aL, aR) && du2 <= 1e-6 * fmin(P.L.c * P.L.c, P.R.c * P.R.c);
}

}  // namespace m2c
