"""Pins of the general-EOS Riemann oracle (``oracle/riemann_eos.py``).

The oracle solves the two-material Riemann problem of eq. 1DRiemannProblem
with a Noble-Abel stiffened gas (eq. NASG_EOS), Mie-Grueneisen (appendix on
equations of state) or JWL (eq. JWL_EOS) on each side, by bracketed roots
and a DOP853 integration of the isentrope.  Every check here compares it with
something it does not contain:

* the stiffened-gas special case against the C oracle's closed-form Newton
  solver (itself pinned to exact solutions);
* NASG with covolume and energy offset against the closed-form NASG wave
  curves, derived by hand in this file;
* Mie-Grueneisen shocks from the reference state against the linear shock
  velocity / particle velocity relation the compression branch encodes, and
  its sound speed at the reference state against c_0;
* rarefactions against an independent integration of the first law
  de = -p dv in (v, e) with finite-difference wave speeds (uses p(rho, e)
  only), and JWL rarefactions against the closed-form JWL isentropes;
* shocks against the Hugoniot written with p(rho, e) instead of e(rho, p);
* mirror and Galilean invariance, and independence of the NASG energy offset;
* the worked glass / air example the paper prints.

``test_planted_mistakes`` plants plausible mistakes in a copy of the oracle
source and shows that a pin catches each.
"""
from __future__ import annotations

import importlib.util
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, optimize

import oracle
from oracle import riemann_eos as RE_MOD

HERE = os.path.dirname(os.path.abspath(__file__))

# --------------------------------------------------------------- materials ---
# Parameter sets of the kinds the paper's examples use (SI units): air, water
# (stiffened and Noble-Abel), soda lime glass, copper, tantalum, TNT products.


def materials(RE):
    return {
        "air": RE.Nasg(1.4),
        "water_sg": RE.Nasg(6.12, 3.43e8),
        "water_nasg": RE.Nasg(1.19, 7.028e8, 6.61e-4, -1.177788e6),
        "gas_nasg": RE.Nasg(1.6, 0.0, 2.0e-4, 3.0e5),
        "glass": RE.MieGruneisen(2204.0, 2220.0, 0.65, 1.61, 0.0, -0.5),
        "copper": RE.MieGruneisen(8930.0, 3940.0, 2.0, 1.49, 0.0, -0.1),
        "tantalum": RE.MieGruneisen(16650.0, 3414.0, 1.6, 1.2, 1.0e4, -0.05),
        "tnt": RE.Jwl(0.3, 3.712e11, 3.231e9, 4.15, 0.95, 1630.0),
    }


def random_state(rng, name, m):
    """(rho, p) inside the material's admissible range."""
    if name == "air" or name == "gas_nasg":
        return rng.uniform(0.5, 50.0), 10 ** rng.uniform(4.5, 7.5)
    if name.startswith("water"):
        return rng.uniform(950.0, 1100.0), 10 ** rng.uniform(5, 9)
    if name in ("glass", "copper", "tantalum"):
        return m.rho0 * (1.0 + rng.uniform(-0.005, 0.06)), rng.uniform(0.0, 5e9)
    if name == "tnt":
        return rng.uniform(400.0, 1800.0), 10 ** rng.uniform(7, 10)
    raise KeyError(name)


def problems(RE, rng, pairs, per_pair):
    """Sides (left, right) for each pair of material names, velocities drawn
    around the acoustic scale so that shocks and rarefactions both occur."""
    mats = materials(RE)
    out = []
    for a, b in pairs:
        k = 0
        while k < per_pair:
            rl, pl = random_state(rng, a, mats[a])
            rr, pr = random_state(rng, b, mats[b])
            try:
                L = RE.Side(mats[a], rl, 0.0, pl)
                R = RE.Side(mats[b], rr, 0.0, pr)
            except ValueError:
                continue
            du = rng.uniform(-1.0, 0.6) * min(L.c, R.c)
            L.u, R.u = 0.5 * du, -0.5 * du
            out.append((L, R))
            k += 1
    return out


def star(RE, L, R):
    return RE.star_state(L, R)


# ------------------------------------------------------------------ checks ---

def check_stiffened_gas(RE):
    """NASG with b = e_c = 0 is the stiffened gas of the C oracle, whose
    Newton solver uses the closed-form wave curves."""
    rng = np.random.default_rng(11)
    ncav = 0
    for i in range(14):
        g = rng.uniform(1.2, 7.0, 2)
        pc = rng.choice([0.0, 3e8, 6e8], 2)
        rho = rng.uniform(1.0, 1000.0, 2)
        p = 10 ** rng.uniform(4, 9, 2)
        u = rng.normal(0.0, 150.0, 2)
        L = RE.Side(RE.Nasg(g[0], pc[0]), rho[0], u[0], p[0])
        R = RE.Side(RE.Nasg(g[1], pc[1]), rho[1], u[1], p[1])
        s = star(RE, L, R)
        rc, o, _ = oracle.riemann([rho[0], u[0], p[0], rho[1], u[1], p[1]], [g[0], pc[0], g[1], pc[1]])
        if rc != 0:
            assert math.isnan(s[0]), (i, s)
            ncav += 1
            continue
        scale = abs(o[0]) + pc.max()
        assert abs(s[0] - o[0]) <= 1e-11 * scale, (i, s, o)
        assert abs(s[1] - o[1]) <= 1e-11 * max(L.c, R.c), (i, s, o)
        assert abs(s[2] / o[2] - 1) <= 1e-11 and abs(s[3] / o[3] - 1) <= 1e-11, (i, s, o)
    assert ncav < 14


def nasg_wave(m, rho, p, pstar):
    """Closed-form NASG wave curve (derived from e = (p + gamma p_c)(v - b)
    / (gamma - 1) + e_c): shock through the Hugoniot, whose covolume-shifted
    volume ratio is rational in p + p_c; rarefaction through the isentrope
    (p + p_c)(v - b)^gamma = const.  Returns (f, rho*)."""
    g, pc, b = m.g, m.pc, m.b
    qb, qK = pstar + pc, p + pc
    VK = 1.0 / rho - b
    if pstar > p:
        V = VK * ((g - 1) * qb + (g + 1) * qK) / ((g + 1) * qb + (g - 1) * qK)
        return math.sqrt((pstar - p) * (VK - V)), 1.0 / (V + b)
    cK = math.sqrt(g * qK / (rho * (1.0 - b * rho)))
    f = 2.0 * cK * (1.0 - b * rho) / (g - 1.0) * ((qb / qK) ** ((g - 1.0) / (2.0 * g)) - 1.0)
    return f, 1.0 / (VK * (qK / qb) ** (1.0 / g) + b)


def check_nasg_closed_form(RE):
    rng = np.random.default_rng(12)
    pairs = [("water_nasg", "gas_nasg"), ("gas_nasg", "air"), ("water_nasg", "water_sg")]
    for L, R in problems(RE, rng, pairs, 4):
        s = star(RE, L, R)
        mL, mR = L.eos, R.eos
        lo = max(-mL.pc, -mR.pc) * (1 - 1e-9) + 1e-9

        def F(p):
            return nasg_wave(mL, L.rho, L.p, p)[0] + nasg_wave(mR, R.rho, R.p, p)[0] + R.u - L.u
        if F(lo) > 0:
            assert math.isnan(s[0])
            continue
        hi = max(L.p, R.p)
        while F(hi) < 0:
            hi *= 2.0
        p = optimize.brentq(F, lo, hi, xtol=1e-300, rtol=1e-15)
        fL, rL = nasg_wave(mL, L.rho, L.p, p)
        fR, rR = nasg_wave(mR, R.rho, R.p, p)
        scale = abs(p) + max(mL.pc, mR.pc)
        assert abs(s[0] - p) <= 1e-11 * scale, (s, p)
        assert abs(s[1] - (L.u - fL)) <= 1e-11 * max(L.c, R.c), (s, L.u - fL)
        assert abs(s[2] / rL - 1) <= 1e-11 and abs(s[3] / rR - 1) <= 1e-11, (s, rL, rR)


def check_mg_hugoniot(RE):
    """A shock from the Mie-Grueneisen reference state (rho_0, p = 0,
    e = e_0) moves at U_s = c_0 + s u_p: mass conservation gives U_s =
    rho* u_p / (rho* - rho_0), with u_p the velocity jump."""
    for name in ("glass", "copper", "tantalum"):
        m = materials(RE)[name]
        side = RE.Side(m, m.rho0, 0.0, 0.0)
        assert abs(side.e - m.e0) <= 1e-12 * (abs(m.e0) + 1.0)
        for p in (1e7, 1e8, 1e9, 1e10, 4e10):
            up, r = side.wave(p)
            Us = r * up / (r - m.rho0)
            assert abs(Us - (m.c0 + m.s * up)) <= 1e-10 * Us, (name, p, Us, m.c0 + m.s * up)


def check_mg_reference_sound_speed(RE):
    """c_0 is the sound speed at the reference state (appendix on equations
    of state), and p_R, e_R are continuous where the branches meet."""
    for name in ("glass", "copper", "tantalum"):
        m = materials(RE)[name]
        c = math.sqrt(m.c2(m.rho0, m.e0))
        assert abs(c / m.c0 - 1.0) <= 1e-14, (name, c, m.c0)
        e, d = m.e0 + 1e3, 1e-7

        def p_at(eta):
            return m.p(m.rho0 / (1.0 - eta), e)
        for eta in (0.0, m.eta_min):
            assert abs(p_at(eta + d) - p_at(eta - d)) <= 3.0 * m.K0 * d, (name, eta)
        # p_R and its slope K_0 continue across eta = 0
        up, down = (p_at(d) - p_at(0.0)) / d, (p_at(0.0) - p_at(-d)) / d
        assert abs(up / down - 1.0) <= 1e-4 and abs(down / m.K0 - 1.0) <= 0.05, (name, up, down)


def rarefaction_cases(RE):
    mats = materials(RE)
    cases = []
    for name, rho, p, frac in (("glass", 2204.0, 1e5, 0.0), ("glass", 2260.0, 2e9, 0.2),
                               ("copper", 9100.0, 4e9, -0.5), ("tantalum", 16600.0, 1e8, -0.1),
                               ("tnt", 1630.0, 2.1e10, 0.01), ("tnt", 600.0, 1e8, 0.001),
                               ("water_nasg", 1050.0, 3e8, 0.001), ("gas_nasg", 20.0, 1e6, 0.01)):
        m = mats[name]
        cases.append((m, rho, p, m.floor + frac * (p - m.floor) if frac > 0 else p * frac if frac < 0 else 0.0))
    return cases


def check_first_law(RE):
    """Rarefaction end states against an independent integration of
    de/dv = -p(v, e), and f against -int sqrt(-dp/dv|_s) dv with the slope
    of the isentrope taken by central differences of p(rho, e)."""
    for m, rho, p, pstar in rarefaction_cases(RE):
        side = RE.Side(m, rho, 0.0, p)
        f, rs = side.wave(pstar)
        vK, vs = 1.0 / rho, 1.0 / rs

        def slope(v, e):
            d = 1e-6 * v
            pp = m.p(1.0 / v, e)
            return (m.p(1.0 / (v + d), e - pp * d) - m.p(1.0 / (v - d), e + pp * d)) / (2 * d)

        def rhs(v, y):
            return [-m.p(1.0 / v, y[0]), -math.sqrt(max(-slope(v, y[0]), 0.0))]
        sol = integrate.solve_ivp(rhs, (vK, vs), [side.e, 0.0], method="DOP853", rtol=1e-12,
                                  atol=[1e-12 * abs(side.e) + 1e-9, 1e-9 * side.c])
        e_end, f_ind = sol.y[0, -1], sol.y[1, -1]
        assert abs(m.p(rs, e_end) - pstar) <= 1e-8 * (p - m.floor), (type(m).__name__, m.p(rs, e_end), pstar)
        assert abs(f - f_ind) <= 1e-7 * side.c, (type(m).__name__, f, f_ind)


def check_jwl_isentrope(RE):
    """JWL isentropes in closed form: p_s(V) = A_1 exp(-R_1 V) + A_2
    exp(-R_2 V) + C V^-(1+omega), V = rho_0/rho (the curves along which
    de = -p dv for eq. JWL_EOS)."""
    m = materials(RE)["tnt"]
    A1, A2 = m.A
    R1, R2 = m.R
    w, v0 = m.w, 1.0 / m.rho0
    for rho, p, pstar in ((1630.0, 2.1e10, 1e9), (1000.0, 3e9, 1e7), (300.0, 1e8, 2e5)):
        VK = m.rho0 / rho
        C = (p - A1 * math.exp(-R1 * VK) - A2 * math.exp(-R2 * VK)) * VK ** (1 + w)

        def ps(V):
            return A1 * math.exp(-R1 * V) + A2 * math.exp(-R2 * V) + C * V ** -(1 + w)

        def dps_dv(v):
            V = v / v0
            return (-A1 * R1 * math.exp(-R1 * V) - A2 * R2 * math.exp(-R2 * V) - (1 + w) * C * V ** -(2 + w)) / v0
        side = RE.Side(m, rho, 0.0, p)
        f, rs = side.wave(pstar)
        assert abs(ps(m.rho0 / rs) - pstar) <= 1e-10 * p, (rho, ps(m.rho0 / rs), pstar)
        f_ind = -integrate.quad(lambda v: math.sqrt(-dps_dv(v)), 1.0 / rho, 1.0 / rs, epsabs=0, epsrel=1e-13,
                                limit=200)[0]
        assert abs(f - f_ind) <= 1e-10 * side.c, (rho, f, f_ind)


def check_shock_with_p_of_e(RE):
    """Shock end states against the Hugoniot written with p(rho, e):
    p(1/v, e_K + (p* + p_K)(v_K - v)/2) = p*, solved for v by bisection."""
    mats = materials(RE)
    for name, rho, p, pstar in (("tnt", 1630.0, 1e9, 3e10), ("tnt", 500.0, 1e7, 1e9), ("copper", 8930.0, 0.0, 5e10),
                                ("glass", 2200.0, 1e5, 3e9), ("water_nasg", 1000.0, 1e5, 2e9),
                                ("gas_nasg", 1.0, 1e5, 3e7), ("tantalum", 16700.0, 2e9, 6e9)):
        m = mats[name]
        side = RE.Side(m, rho, 0.0, p)
        f, rs = side.wave(pstar)
        vK = 1.0 / rho

        def G(v):
            return m.p(1.0 / v, side.e + 0.5 * (pstar + p) * (vK - v)) - pstar
        lo = vK
        while G(lo) < 0:
            lo *= 0.98
            if math.isfinite(m.rho_max):
                lo = max(lo, 1.0 / m.rho_max * (1 + 1e-12))
        v = optimize.brentq(G, lo, vK, xtol=1e-300, rtol=1e-15)
        assert abs(v * rs - 1.0) <= 1e-11, (name, v, 1.0 / rs)
        assert abs(f - math.sqrt((pstar - p) * (vK - v))) <= 1e-10 * math.sqrt(pstar * vK), (name,)


def check_invariances(RE):
    """Mirror symmetry, Galilean invariance and, for NASG, independence of
    the energy offset e_c."""
    rng = np.random.default_rng(13)
    pairs = [("water_nasg", "copper"), ("tnt", "air"), ("glass", "tantalum"), ("tnt", "water_sg")]
    for L, R in problems(RE, rng, pairs, 2):
        s = star(RE, L, R)
        if math.isnan(s[0]):
            continue
        m = star(RE, RE.Side(R.eos, R.rho, -R.u, R.p), RE.Side(L.eos, L.rho, -L.u, L.p))
        c = max(L.c, R.c)
        ps = abs(s[0]) + max(L.p, R.p)
        assert abs(m[0] - s[0]) <= 1e-11 * ps and abs(m[1] + s[1]) <= 1e-11 * c, (s, m)
        assert abs(m[2] / s[3] - 1) <= 1e-11 and abs(m[3] / s[2] - 1) <= 1e-11, (s, m)
        U = 0.7 * c
        g = star(RE, RE.Side(L.eos, L.rho, L.u + U, L.p), RE.Side(R.eos, R.rho, R.u + U, R.p))
        assert abs(g[0] - s[0]) <= 1e-11 * ps and abs(g[1] - s[1] - U) <= 1e-11 * c, (s, g)
    a = RE.Nasg(1.19, 7.028e8, 6.61e-4, 0.0)
    b = RE.Nasg(1.19, 7.028e8, 6.61e-4, -2.5e6)
    air = RE.Nasg(1.4)
    for u in (-300.0, 50.0):
        s0 = star(RE, RE.Side(a, 1000.0, 0.0, 1e8), RE.Side(air, 1.2, u, 1e5))
        s1 = star(RE, RE.Side(b, 1000.0, 0.0, 1e8), RE.Side(air, 1.2, u, 1e5))
        assert abs(s0[0] - s1[0]) <= 1e-11 * (abs(s0[0]) + 7.028e8) and abs(s0[1] - s1[1]) <= 1e-9, (s0, s1)
        assert abs(s0[2] / s1[2] - 1) <= 1e-11, (s0, s1)


def check_glass_air(RE):
    """The paper's worked example: a glass slab moving away from air."""
    d = json.load(open(os.path.join(HERE, "golden", "riemann_eos_glass_air.json")))
    L = RE.Side(RE.make_eos(RE.NASG, d["left"]["params"]), d["left"]["rho"], d["left"]["u"], d["left"]["p"])
    R = RE.Side(RE.make_eos(RE.MG, d["right"]["params"]), d["right"]["rho"], d["right"]["u"], d["right"]["p"])
    p, u, rL, rR = star(RE, L, R)
    assert round(rR, 2) == d["printed"]["rho_star_glass_kg_m3"], rR
    assert p < L.p and p < R.p and rL > 0.0          # two rarefactions, no cavitation


CHECKS = {f.__name__: f for f in (check_stiffened_gas, check_nasg_closed_form, check_mg_hugoniot,
                                  check_mg_reference_sound_speed, check_first_law, check_jwl_isentrope,
                                  check_shock_with_p_of_e, check_invariances, check_glass_air)}


@pytest.mark.parametrize("name", sorted(CHECKS))
def test_pin(name):
    CHECKS[name](RE_MOD)


def test_solve_array_interface():
    """solve() over arrays equals star_state() per problem; cavitation gives NaN."""
    mats = [RE_MOD.Nasg(1.4), RE_MOD.MieGruneisen(2204.0, 2220.0, 0.65, 1.61)]
    inp = np.array([[1.2, 1.2], [0.0, -3000.0], [1e5, 1e5], [2204.0, 1.2], [100.0, 3000.0], [1e5, 1e5]])
    mat = np.array([[0, 0], [1, 0]])
    out = RE_MOD.solve(inp, mat, mats)
    ref = RE_MOD.star_state(RE_MOD.Side(mats[0], 1.2, 0.0, 1e5), RE_MOD.Side(mats[1], 2204.0, 100.0, 1e5))
    assert np.allclose(out[:, 0], ref, rtol=0, atol=0)
    assert np.isnan(out[:, 1]).all()


# -------------------------------------------------------- planted mistakes ---
MUTANTS = [
    ("nasg dp/drho power", "self.ec) / (1.0 - rho * self.b) ** 2", "self.ec) / (1.0 - rho * self.b)",
     "check_nasg_closed_form"),
    ("mg Hugoniot energy half", "return pR, pR * eta / (2.0 * r0) + self.e0", "return pR, pR * eta / r0 + self.e0",
     "check_mg_hugoniot"),
    ("mg tension de_R", "K0, K0 * eta / r0", "K0, K0 * eta / (2.0 * r0)", "check_first_law"),
    ("jwl exponent sign", "x = math.exp(-R * self.rho0 / rho)", "x = math.exp(R * self.rho0 / rho)",
     "check_jwl_isentrope"),
    ("jwl derivative", "a * x * R * self.rho0 / (rho * rho)", "a * x * R * self.rho0 / rho", "check_jwl_isentrope"),
    ("hugoniot mean pressure", "0.5 * (pstar + pK)", "0.5 * (pstar - pK)", "check_stiffened_gas"),
    ("rarefaction df/ds", "return [self.rho * math.exp(s) * c2, math.sqrt(c2)]",
     "return [self.rho * math.exp(s) * c2, math.sqrt(c2) / self.rho]", "check_stiffened_gas"),
    ("sound speed sign", "+ self.p(rho, e) * self.p_e(rho, e)", "- self.p(rho, e) * self.p_e(rho, e)",
     "check_stiffened_gas"),
    ("star velocity side", "0.5 * (left.u - fL + right.u + fR)", "0.5 * (left.u + fL + right.u - fR)",
     "check_stiffened_gas"),
]


@pytest.mark.parametrize("label,old,new,check", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistakes(label, old, new, check, tmp_path):
    src = open(RE_MOD.__file__).read()
    assert src.count(old) == 1, label
    path = tmp_path / "riemann_eos_mutant.py"
    path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location("riemann_eos_mutant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    with pytest.raises((AssertionError, ValueError, RuntimeError, ZeroDivisionError, OverflowError)):
        CHECKS[check](mod)
