"""Independent exact solver for the two-material stiffened-gas Riemann problem
(TEST INFRASTRUCTURE; shares no code with the C oracle).

The paper builds its interface fluxes on exact solutions of one-dimensional
bimaterial Riemann problems (eq. 1DRiemannProblem) and verifies the whole
code against such solutions (section "One-dimensional Riemann problems").
This module computes those solutions by a different route from the oracle's
Newton solver, so that agreement between the two is evidence for both:

* the velocity change across a shock comes from the jump conditions: the
  Hugoniot energy relation e(rho*, p) - e(rho_K, p_K) = (p + p_K)/2 (1/rho_K
  - 1/rho*) is solved for rho* by bracketing, then mass and momentum give
  |du| = sqrt((p - p_K)(1/rho_K - 1/rho*));
* the velocity change across a rarefaction is the integral of dp/(rho c)
  along the isentrope, evaluated by adaptive quadrature;
* the star pressure is found by a derivative-free bracketing root search.

EOS: p = (gamma - 1) rho e - gamma p_c, c^2 = gamma (p + p_c)/rho.
"""
from __future__ import annotations

import math
import warnings

import numpy as np
from scipy import integrate, optimize


def _e(rho, p, g, pc):
    return (p + g * pc) / ((g - 1.0) * rho)


def _isentrope_rho(p, rho0, p0, g, pc):
    # dS = 0 for the stiffened gas: (p + p_c) rho^-gamma is constant
    return rho0 * ((p + pc) / (p0 + pc)) ** (1.0 / g)


def _shock_rho(p, rho0, p0, g, pc):
    def hug(r):
        return _e(r, p, g, pc) - _e(rho0, p0, g, pc) - 0.5 * (p + p0) * (1.0 / rho0 - 1.0 / r)
    lo = rho0
    hi = rho0 * (g + 1.0) / (g - 1.0)
    # hug(lo) > 0 and hug -> -inf as r -> strong-shock limit from below
    hi_in = hi * (1.0 - 1e-14)
    while hug(hi_in) > 0.0:
        hi_in = lo + 0.5 * (hi_in - lo) + 0.5 * (hi - lo)
    return optimize.brentq(hug, lo, hi_in, xtol=1e-300, rtol=1e-15, maxiter=500)


def velocity_change(p, rho0, u0, p0, g, pc):
    """f_K(p): decrease of the velocity from side K's state to the star
    region, positive for compression."""
    if p > p0:
        rs = _shock_rho(p, rho0, p0, g, pc)
        return math.sqrt((p - p0) * (1.0 / rho0 - 1.0 / rs))
    if p == p0:
        return 0.0

    def integrand(pp):
        r = _isentrope_rho(pp, rho0, p0, g, pc)
        return 1.0 / (r * math.sqrt(g * (pp + pc) / r))
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", integrate.IntegrationWarning)
        val, _ = integrate.quad(integrand, p, p0, epsabs=0.0, epsrel=2e-14, limit=400)
    return -val


def star_state(inp, eos):
    """Star state of one problem: returns (p*, u*, rho*_L, rho*_R) or None
    when no admissible star pressure exists (vacuum)."""
    rL, uL, pL, rR, uR, pR = (float(x) for x in inp)
    gL, pcL, gR, pcR = (float(x) for x in eos)
    plo = -min(pcL, pcR)

    def g(p):
        return (velocity_change(p, rL, uL, pL, gL, pcL) +
                velocity_change(p, rR, uR, pR, gR, pcR) + (uR - uL))

    a = plo + 1e-13 * max(pL - plo, pR - plo)
    if g(a) >= 0.0:
        return None
    b = max(pL, pR)
    while g(b) < 0.0:
        b = plo + 2.0 * (b - plo)
    ps = optimize.brentq(g, a, b, xtol=1e-300, rtol=1e-15, maxiter=500)
    us = 0.5 * (uL + uR) + 0.5 * (velocity_change(ps, rR, uR, pR, gR, pcR)
                                  - velocity_change(ps, rL, uL, pL, gL, pcL))
    rsL = _shock_rho(ps, rL, pL, gL, pcL) if ps > pL else _isentrope_rho(ps, rL, pL, gL, pcL)
    rsR = _shock_rho(ps, rR, pR, gR, pcR) if ps > pR else _isentrope_rho(ps, rR, pR, gR, pcR)
    return ps, us, rsL, rsR


def sample(inp, eos, xi):
    """Self-similar exact solution at speeds xi = (x - x0)/t.

    Returns arrays (rho, u, p, side) with side 0 left material, 1 right.
    Fan interiors use the Riemann invariant u +- 2c/(gamma - 1) and the
    isentrope in the shifted pressure p + p_c.
    """
    st = star_state(inp, eos)
    if st is None:
        raise ValueError("vacuum")
    ps, us, rsL, rsR = st
    rL, uL, pL, rR, uR, pR = (float(x) for x in inp)
    gL, pcL, gR, pcR = (float(x) for x in eos)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    side = (xi > us).astype(np.int32)
    cL = math.sqrt(gL * (pL + pcL) / rL)
    cR = math.sqrt(gR * (pR + pcR) / rR)
    for n, s in enumerate(xi):
        if s <= us:                               # left of the contact
            if ps > pL:
                S = (rsL * us - rL * uL) / (rsL - rL)
                vals = (rL, uL, pL) if s < S else (rsL, us, ps)
            else:
                csL = math.sqrt(gL * (ps + pcL) / rsL)
                head, tail = uL - cL, us - csL
                if s < head:
                    vals = (rL, uL, pL)
                elif s > tail:
                    vals = (rsL, us, ps)
                else:
                    J = uL + 2.0 * cL / (gL - 1.0)
                    c = (J - s) * (gL - 1.0) / (gL + 1.0)
                    vals = (rL * (c / cL) ** (2.0 / (gL - 1.0)), s + c,
                            (pL + pcL) * (c / cL) ** (2.0 * gL / (gL - 1.0)) - pcL)
        else:                                     # right of the contact
            if ps > pR:
                S = (rsR * us - rR * uR) / (rsR - rR)
                vals = (rR, uR, pR) if s > S else (rsR, us, ps)
            else:
                csR = math.sqrt(gR * (ps + pcR) / rsR)
                head, tail = uR + cR, us + csR
                if s > head:
                    vals = (rR, uR, pR)
                elif s < tail:
                    vals = (rsR, us, ps)
                else:
                    J = uR - 2.0 * cR / (gR - 1.0)
                    c = (s - J) * (gR - 1.0) / (gR + 1.0)
                    vals = (rR * (c / cR) ** (2.0 / (gR - 1.0)), s - c,
                            (pR + pcR) * (c / cR) ** (2.0 * gR / (gR - 1.0)) - pcR)
        rho[n], u[n], p[n] = vals
    return rho, u, p, side


def cell_averages(inp, eos, x0, t, edges, sub=16):
    """Exact cell averages of rho, u, p over cells with the given edges
    (midpoint rule with ``sub`` points per cell)."""
    edges = np.asarray(edges, dtype=np.float64)
    ncell = len(edges) - 1
    offs = (np.arange(sub) + 0.5) / sub
    x = (edges[:-1, None] + (edges[1:] - edges[:-1])[:, None] * offs[None, :]).reshape(-1)
    rho, u, p, _ = sample(inp, eos, (x - x0) / t)
    return (rho.reshape(ncell, sub).mean(1), u.reshape(ncell, sub).mean(1),
            p.reshape(ncell, sub).mean(1))
