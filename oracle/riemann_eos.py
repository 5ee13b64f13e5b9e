"""Exact two-material Riemann problem with a general convex EOS on each side
(TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg may use this module; it shares no code with the GPU library).

What is computed: the star state (p*, u*, rho*_L, rho*_R) of the
one-dimensional bimaterial Riemann problem of eq. 1DRiemannProblem when each
side obeys its own EOS p = p(rho, e) (section "Equations of state", eq.
eos_all).  Three families are covered, as the paper defines them:

* Noble-Abel stiffened gas, eq. NASG_EOS (parameters gamma, p_c, b, e_c);
* Mie-Grueneisen in the compression / tension form of the appendix on
  equations of state (rho_0, c_0, Gamma_0, s, e_0, eta_min);
* Jones-Wilkins-Lee, eq. JWL_EOS (omega, A_1, A_2, R_1, R_2, rho_0).

The paper cites the solvers it uses for these problems without giving their
steps.  The solution follows from the Euler equations alone, and this module
writes that definition out:

* p* is the root of F(p) = f_L(p) + f_R(p) + u_R - u_L, so that pressure and
  normal velocity are continuous at the interface (eq. interface_cond),
  with u*_L = u_L - f_L(p*) and u*_R = u_R + f_R(p*);
* for p > p_K the K-wave is a shock: the Hugoniot energy relation
  e(rho*, p) - e_K = (p + p_K)/2 (1/rho_K - 1/rho*) gives rho*, and mass and
  momentum give f_K = sqrt((p - p_K)(1/rho_K - 1/rho*));
* for p <= p_K it is a rarefaction: along the isentrope through state K,
  parametrised by s = ln(rho / rho_K), dp/ds = rho c^2 and df/ds = c, with
  c^2 = dp/drho|_e + p dp/de|_rho / rho^2; f_K(p) is f at the s where the
  isentrope reaches p.

Library primitives: scipy's DOP853 integrator (dense output, relative
tolerance 1e-13) for the isentrope and brentq for the three scalar roots
(Hugoniot density, isentrope position, star pressure).  No Newton steps, no
acoustic guesses: every root is bracketed.

Admissible pressures (a reading; the paper states only the MG one): a state
or star pressure must exceed the family's floor -- -p_c for NASG (where its
sound speed vanishes), p_min = K_0 eta_min for MG (the stated minimum
pressure), 0 for JWL.  A problem whose sides separate faster than their
isentropes can follow down to the higher floor has no star state
(cavitation) and returns NaN, as the stiffened-gas solver does.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize

NASG, MG, JWL = 0, 1, 2
NPARAM = 7


class Eos:
    """p(rho, e), its inverse e(rho, p) and the partial derivatives."""

    floor = -math.inf
    rho_max = math.inf

    def c2(self, rho, e):
        return self.p_rho(rho, e) + self.p(rho, e) * self.p_e(rho, e) / (rho * rho)

    def params(self):
        raise NotImplementedError


class Nasg(Eos):
    """Eq. NASG_EOS: p = (gamma - 1) rho (e - e_c) / (1 - rho b) - gamma p_c."""

    def __init__(self, gamma, pc=0.0, b=0.0, ec=0.0):
        self.g, self.pc, self.b, self.ec = float(gamma), float(pc), float(b), float(ec)
        self.floor = -self.pc
        self.rho_max = 1.0 / self.b if self.b > 0 else math.inf

    def p(self, rho, e):
        return (self.g - 1.0) * rho * (e - self.ec) / (1.0 - rho * self.b) - self.g * self.pc

    def e(self, rho, p):
        return (p + self.g * self.pc) * (1.0 - rho * self.b) / ((self.g - 1.0) * rho) + self.ec

    def p_rho(self, rho, e):
        return (self.g - 1.0) * (e - self.ec) / (1.0 - rho * self.b) ** 2

    def p_e(self, rho, e):
        return (self.g - 1.0) * rho / (1.0 - rho * self.b)

    def params(self):
        return (NASG, [self.g, self.pc, self.b, self.ec])


class MieGruneisen(Eos):
    """Appendix on equations of state, Mie-Grueneisen: p = p_R(eta) +
    rho_0 Gamma_0 (e - e_R(eta)), eta = 1 - rho_0/rho, with the reference
    curves of compression (eta > 0), small tension (eta_min <= eta < 0) and
    the tensile cutoff (eta < eta_min).  In compression e_R uses the
    Hugoniot pressure of the reference state, which is p_R itself."""

    def __init__(self, rho0, c0, Gamma0, s, e0=0.0, eta_min=-0.5):
        self.rho0, self.c0, self.G0, self.s = float(rho0), float(c0), float(Gamma0), float(s)
        self.e0, self.eta_min = float(e0), float(eta_min)
        self.K0 = self.rho0 * self.c0 ** 2
        self.pmin = self.K0 * self.eta_min
        self.floor = self.pmin
        self.rho_max = self.rho0 * self.s / (self.s - 1.0) if self.s > 1.0 else math.inf

    def _ref(self, eta):
        """(p_R, e_R, dp_R/deta, de_R/deta)."""
        r0, K0, s = self.rho0, self.K0, self.s
        if eta >= 0.0:
            pR = K0 * eta / (1.0 - s * eta) ** 2
            dpR = K0 * (1.0 + s * eta) / (1.0 - s * eta) ** 3
            return pR, pR * eta / (2.0 * r0) + self.e0, dpR, (dpR * eta + pR) / (2.0 * r0)
        if eta >= self.eta_min:
            return K0 * eta, K0 * eta * eta / (2.0 * r0) + self.e0, K0, K0 * eta / r0
        em = self.eta_min
        return (self.pmin, K0 * em * em / (2.0 * r0) + self.e0 + self.pmin / r0 * (eta - em),
                0.0, self.pmin / r0)

    def p(self, rho, e):
        pR, eR, _, _ = self._ref(1.0 - self.rho0 / rho)
        return pR + self.rho0 * self.G0 * (e - eR)

    def e(self, rho, p):
        pR, eR, _, _ = self._ref(1.0 - self.rho0 / rho)
        return eR + (p - pR) / (self.rho0 * self.G0)

    def p_rho(self, rho, e):
        _, _, dpR, deR = self._ref(1.0 - self.rho0 / rho)
        return (dpR - self.rho0 * self.G0 * deR) * self.rho0 / (rho * rho)

    def p_e(self, rho, e):
        return self.rho0 * self.G0

    def params(self):
        return (MG, [self.rho0, self.c0, self.G0, self.s, self.e0, self.eta_min])


class Jwl(Eos):
    """Eq. JWL_EOS: p = omega rho e + sum_i A_i (1 - omega rho / (R_i rho_0))
    exp(-R_i rho_0 / rho).  The printed equation carries a positive exponent
    in its first term; the temperature law beside it and the standard form
    have the negative one, which is taken here for both terms."""

    floor = 0.0

    def __init__(self, omega, A1, A2, R1, R2, rho0):
        self.w, self.A = float(omega), (float(A1), float(A2))
        self.R, self.rho0 = (float(R1), float(R2)), float(rho0)

    def _terms(self, rho):
        """sum_i A_i (1 - omega rho/(R_i rho_0)) x_i and its rho-derivative,
        x_i = exp(-R_i rho_0 / rho)."""
        t = dt = 0.0
        for A, R in zip(self.A, self.R):
            x = math.exp(-R * self.rho0 / rho)
            a = 1.0 - self.w * rho / (R * self.rho0)
            t += A * a * x
            dt += A * (-self.w / (R * self.rho0) * x + a * x * R * self.rho0 / (rho * rho))
        return t, dt

    def p(self, rho, e):
        return self.w * rho * e + self._terms(rho)[0]

    def e(self, rho, p):
        return (p - self._terms(rho)[0]) / (self.w * rho)

    def p_rho(self, rho, e):
        return self.w * e + self._terms(rho)[1]

    def p_e(self, rho, e):
        return self.w * rho

    def params(self):
        return (JWL, [self.w, self.A[0], self.A[1], self.R[0], self.R[1], self.rho0])


def make_eos(family, params):
    """An Eos from a family id and its parameter list (as in params())."""
    if family == NASG:
        return Nasg(*params[:4])
    if family == MG:
        return MieGruneisen(*params[:6])
    if family == JWL:
        return Jwl(*params[:6])
    raise ValueError(f"unknown EOS family {family}")


def pack(eos_list):
    """[(family, [NPARAM doubles])] of a material list (the table layout the
    library's general-EOS entry points take)."""
    out = []
    for m in eos_list:
        fam, prm = m.params()
        out.append((fam, list(prm) + [0.0] * (NPARAM - len(prm))))
    return out


# An isentrope is followed down to q = p - floor = 1e-12 (p_K - floor) +
# 1e-6 |floor|; star pressures below that count as cavitation.  Closer to
# the floor, p + |floor| is a difference of nearly equal numbers and the
# isentrope is not resolved in FP64.
_FLOOR_MARGIN = 1e-12
_FLOOR_REL = 1e-6
_S_END = -400.0
_MAX_STEPS = 20000


class Side:
    """One side K = (rho, u, p) of the problem and its wave curve f_K(p)."""

    def __init__(self, eos, rho, u, p):
        self.eos, self.rho, self.u, self.p = eos, float(rho), float(u), float(p)
        if not (self.rho > 0 and self.rho < eos.rho_max and self.p > eos.floor):
            raise ValueError("inadmissible state")
        self.e = eos.e(self.rho, self.p)
        c2 = eos.c2(self.rho, self.e)
        if not c2 > 0:
            raise ValueError("state with c^2 <= 0")
        self.c = math.sqrt(c2)
        self._sol = None

    # -- rarefaction: the isentrope through K in s = ln(rho/rho_K) --------------
    def _isentrope(self):
        if self._sol is not None:
            return self._sol
        eos, fl = self.eos, self.eos.floor
        q0 = self.p - fl                              # distance from the floor

        def c2_at(t, q):
            rho = self.rho * math.exp(t)
            return eos.c2(rho, eos.e(rho, fl + q))

        def rhs(s, y):
            c2 = c2_at(s, y[0])
            if not c2 > 0:                      # outside the convex part (trial stages only)
                return [0.0, 0.0]
            return [self.rho * math.exp(s) * c2, math.sqrt(c2)]

        # Stepped by hand so that the run is bounded.  Pressures are carried
        # as the distance q from the floor; where the floor is far below
        # the pressure (large p_c), q is only known to the rounding of p
        # itself, so the absolute tolerance of q is that rounding level.
        # The isentrope ends where q reaches q_stop or where c^2 reaches 0
        # (the EOS is admissible only where it is convex), each located
        # inside the accepted step that passes it.
        st = integrate.DOP853(rhs, 0.0, [q0, 0.0], _S_END, rtol=1e-13,
                              atol=[1e-15 * abs(fl) + 1e-300, 1e-15 * self.c])
        ts, interps = [0.0], []
        q_stop = _FLOOR_MARGIN * q0 + _FLOOR_REL * abs(fl)
        end = None
        while st.status == "running":
            if len(interps) >= _MAX_STEPS:
                raise RuntimeError("isentrope integration exceeded its step budget")
            st.step()
            if st.status == "failed":
                raise RuntimeError("isentrope integration failed")
            ts.append(st.t)
            interps.append(st.dense_output())
            nonconvex = not c2_at(st.t, st.y[0]) > 0
            if not nonconvex and st.y[0] > q_stop:
                continue
            sol = integrate._ivp.common.OdeSolution(ts, interps)
            if nonconvex:
                end = optimize.brentq(lambda t: c2_at(t, sol(t)[0]), ts[-1], ts[-2], xtol=1e-300, rtol=1e-15)
                end = end + 1e-12 * (ts[-2] - end)      # stay on the convex side
            if st.y[0] <= q_stop:
                t_q = optimize.brentq(lambda t: sol(t)[0] - q_stop, ts[-1], ts[-2], xtol=1e-300, rtol=1e-15)
                end = t_q if end is None else max(end, t_q)
            if end is not None:
                break
        sol = integrate._ivp.common.OdeSolution(ts, interps)
        self.s_end = ts[-1] if end is None else end
        y_end = sol(self.s_end)
        self.p_end = fl + float(y_end[0])
        self.f_end = float(y_end[1])
        self._sol = sol
        return sol

    def _rarefaction(self, pstar):
        sol = self._isentrope()
        if pstar < self.p_end:
            return None
        if pstar == self.p_end:
            return self.f_end, self.rho * math.exp(self.s_end)
        if pstar >= self.p:
            return 0.0, self.rho
        q = pstar - self.eos.floor
        s = optimize.brentq(lambda t: sol(t)[0] - q, self.s_end, 0.0, xtol=1e-300, rtol=1e-15, maxiter=500)
        return float(sol(s)[1]), self.rho * math.exp(s)

    # -- shock: the Hugoniot energy relation ------------------------------------
    def _shock(self, pstar):
        eos, rK, pK, eK = self.eos, self.rho, self.p, self.e

        def hug(r):
            return eos.e(r, pstar) - eK - 0.5 * (pstar + pK) * (1.0 / rK - 1.0 / r)
        lo = rK
        if math.isfinite(eos.rho_max):
            hi = eos.rho_max * (1.0 - 1e-15)
        else:
            hi = 2.0 * rK
            while hug(hi) > 0.0:
                lo, hi = hi, 2.0 * hi
        r = optimize.brentq(hug, lo, hi, xtol=1e-300, rtol=1e-15, maxiter=500)
        return math.sqrt((pstar - pK) * (1.0 / rK - 1.0 / r)), r

    def wave(self, pstar):
        """(f_K(p*), rho*_K), or None below the reach of the isentrope."""
        if pstar > self.p:
            return self._shock(pstar)
        return self._rarefaction(pstar)


def star_state(left, right):
    """(p*, u*, rho*_L, rho*_R) of Sides left and right; NaNs when no star
    state exists (cavitation)."""
    nan = (math.nan,) * 4
    du = right.u - left.u

    def F(p):
        a, b = left.wave(p), right.wave(p)
        if a is None or b is None:
            return None
        return a[0] + b[0] + du

    left._isentrope()
    right._isentrope()
    lo = max(left.p_end, right.p_end)
    Flo = F(lo)
    if Flo is None or Flo > 0.0:
        return nan
    fl = max(left.eos.floor, right.eos.floor)
    hi = max(left.p, right.p)
    while F(hi) < 0.0:
        hi = fl + 2.0 * (hi - fl)
    p = optimize.brentq(lambda x: F(x), lo, hi, xtol=1e-300, rtol=1e-15, maxiter=500)
    fL, rL = left.wave(p)
    fR, rR = right.wave(p)
    return p, 0.5 * (left.u - fL + right.u + fR), rL, rR


def solve(inp, mats, eos_list):
    """Star states of n problems: inp [6][n] = (rho_L, u_L, p_L, rho_R, u_R,
    p_R), mats [2][n] material indices into eos_list; returns [4][n]."""
    inp = np.asarray(inp, dtype=np.float64).reshape(6, -1)
    mats = np.asarray(mats).reshape(2, -1)
    n = inp.shape[1]
    out = np.empty((4, n))
    for i in range(n):
        L = Side(eos_list[int(mats[0, i])], inp[0, i], inp[1, i], inp[2, i])
        R = Side(eos_list[int(mats[1, i])], inp[3, i], inp[4, i], inp[5, i])
        out[:, i] = star_state(L, R)
    return out


def eval_eos(eos, rho, e):
    """(p, c) at the given (rho, e) arrays."""
    rho, e = np.asarray(rho, dtype=np.float64), np.asarray(e, dtype=np.float64)
    p = np.array([eos.p(r, x) for r, x in zip(rho.ravel(), e.ravel())]).reshape(rho.shape)
    c = np.array([math.sqrt(eos.c2(r, x)) for r, x in zip(rho.ravel(), e.ravel())]).reshape(rho.shape)
    return p, c
