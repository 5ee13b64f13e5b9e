"""Pins of the CPU oracle against things other than itself.

Each check uses a closed form, a conservation law, a physical invariant, an
independent solver or an exact solution -- never a retyped copy of the
oracle's own formula.  ``test_planted_mistakes`` shows that plausible mistakes
planted in the oracle source (on the CPU) make at least one pin fail.
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import exact_riemann as ex

WATER, AIR = W.WATER, W.AIR


# ---------------------------------------------------------------- checks ---
# Each check takes an oracle library handle so the planted-mistake test can
# run it against a mutated build.

def _cons_to_prim(lib, w, g, pc):
    q = np.empty(5)
    lib.ora_cons_to_prim(np.asarray(w, float), g, pc, q)
    return q


def _prim_to_cons(lib, q, g, pc):
    w = np.empty(5)
    lib.ora_prim_to_cons(np.asarray(q, float), g, pc, w)
    return w


def _hllc(lib, qL, qR, g, pc):
    F = np.empty(5)
    lib.ora_hllc(np.asarray(qL, float), np.asarray(qR, float), g, pc, F)
    return F


def _riemann(lib, inp, eos, rtol=1e-12, maxit=50):
    import ctypes
    out = np.empty(4)
    it = ctypes.c_int32(0)
    rc = lib.ora_riemann(np.asarray(inp, float), np.asarray(eos, float), rtol, maxit, out,
                         ctypes.byref(it))
    return rc, out, it.value


def euler_flux_def(q, g, pc):
    """Advective flux along x from its definition (eq. NSEquation_terms),
    with rho E from the stiffened-gas EOS (eq. NASG_EOS, b = e_c = 0)."""
    rho, u, v, w, p = q
    rhoE = (p + g * pc) / (g - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.array([rho * u, rho * u * u + p, rho * u * v, rho * u * w, (rhoE + p) * u])


def _rand_state(rng, mat):
    if mat == 0:   # air-like
        return np.array([rng.uniform(0.1, 10), rng.uniform(-300, 300), rng.uniform(-100, 100),
                         rng.uniform(-100, 100), rng.uniform(1e4, 1e7)])
    return np.array([rng.uniform(900, 1100), rng.uniform(-100, 100), rng.uniform(-50, 50),
                     rng.uniform(-50, 50), rng.uniform(1e4, 1e9)])


def check_eos_roundtrip(lib):
    rng = np.random.default_rng(1)
    for mat, (g, pc) in enumerate([AIR, WATER]):
        for _ in range(200):
            q = _rand_state(rng, mat)
            w = _prim_to_cons(lib, q, g, pc)
            # rho E from the EOS definition, independent of the oracle
            rhoE = (q[4] + g * pc) / (g - 1) + 0.5 * q[0] * (q[1:4] ** 2).sum()
            assert abs(w[4] - rhoE) <= 1e-14 * abs(rhoE)
            q2 = _cons_to_prim(lib, w, g, pc)
            amp = (g * pc + abs(q[4])) / abs(q[4])       # cancellation factor
            assert np.allclose(q2[:4], q[:4], rtol=1e-14, atol=1e-12)
            assert abs(q2[4] - q[4]) <= 8e-16 * amp * abs(q[4]) * 8


def check_sound_speed(lib):
    """c^2 = p_rho + Gamma p / rho (appendix "Flux Jacobians") with the
    partial derivatives of p(rho, e) taken by central differences of the
    oracle's own EOS inversion."""
    rng = np.random.default_rng(2)
    for mat, (g, pc) in enumerate([AIR, WATER]):
        for _ in range(50):
            q = _rand_state(rng, mat)
            q[1:4] = 0.0
            rho, p = q[0], q[4]
            e = (p + g * pc) / ((g - 1) * rho)

            def P(r, ee):
                return _cons_to_prim(lib, [r, 0, 0, 0, r * ee], g, pc)[4]
            dr, de = 1e-4 * rho, 1e-4 * e
            p_rho = (P(rho + dr, e) - P(rho - dr, e)) / (2 * dr)
            Gam = (P(rho, e + de) - P(rho, e - de)) / (2 * de) / rho
            c_fd = math.sqrt(p_rho + Gam * p / rho)
            c = lib.ora_sound_speed(rho, p, g, pc)
            assert abs(c - c_fd) <= 1e-6 * c


def check_mc_limiter(lib):
    a = 1.2
    rng = np.random.default_rng(3)
    for _ in range(500):
        d = rng.normal() * 10 ** rng.uniform(-3, 3)
        # linear data: the slope is the common difference (phi(1) = 1)
        assert lib.ora_mc_slope(d, d, a) == pytest.approx(d, rel=1e-15)
        # local extremum: zero slope
        assert lib.ora_mc_slope(d, -abs(rng.normal()) * np.sign(d), a) == 0.0
        assert lib.ora_mc_slope(0.0, d, a) == 0.0
        assert lib.ora_mc_slope(d, 0.0, a) == 0.0
        # monotone data: the slope is the MC bound min(a|dm|, |dm+dp|/2, a|dp|)
        dm = d
        dp = np.sign(d) * abs(rng.normal()) * 10 ** rng.uniform(-3, 3)
        ref = np.sign(d) * min(a * abs(dm), 0.5 * abs(dm + dp), a * abs(dp))
        assert lib.ora_mc_slope(dm, dp, a) == pytest.approx(ref, rel=1e-13, abs=1e-300)
    # alpha = 0 gives constant reconstruction
    assert lib.ora_mc_slope(1.0, 1.0, 0.0) == 0.0


def check_hllc_properties(lib):
    rng = np.random.default_rng(4)
    for mat, (g, pc) in enumerate([AIR, WATER]):
        for _ in range(300):
            q = _rand_state(rng, mat)
            # consistency: Phi(W, W) = F(W) . n
            F = _hllc(lib, q, q, g, pc)
            Fd = euler_flux_def(q, g, pc)
            c = math.sqrt(g * (q[4] + pc) / q[0])
            rhoE = (q[4] + g * pc) / (g - 1) + 0.5 * q[0] * (q[1:4] ** 2).sum()
            # the star branch forms F + S (U* - U) with U* - U = 0 up to
            # rounding of U, so the bound scales with |U| times the wave speed
            scale = np.abs(Fd).max() + (rhoE + q[0] * np.abs(q[1:4]).max()) * (abs(q[1]) + c)
            assert np.all(np.abs(F - Fd) <= 1e-14 * scale)
            # isolated contact (equal u and p, any rho, v, w): exact upwind flux
            q2 = _rand_state(rng, mat)
            q2[1] = q[1]
            q2[4] = q[4]
            F = _hllc(lib, q, q2, g, pc)
            up = q if q[1] >= 0 else q2
            Fd = euler_flux_def(up, g, pc)
            Fd[1] = up[0] * q[1] ** 2 + q[4]
            c = math.sqrt(g * (q[4] + pc) / min(q[0], q2[0]))
            rhoE = (q[4] + g * pc) / (g - 1) + 0.5 * max(q[0], q2[0]) * 3e4
            scale = np.abs(Fd).max() + (rhoE + max(q[0], q2[0]) * 300) * (abs(q[1]) + c)
            assert np.all(np.abs(F - Fd) <= 1e-14 * scale)
            # mirror symmetry: swapping sides and reversing normal velocities
            # reverses every flux component except the normal momentum
            qa, qb = _rand_state(rng, mat), _rand_state(rng, mat)
            F1 = _hllc(lib, qa, qb, g, pc)
            ma, mb = qa.copy(), qb.copy()
            ma[1] *= -1
            mb[1] *= -1
            F2 = _hllc(lib, mb, ma, g, pc)
            sgn = np.array([-1, 1, -1, -1, -1])
            scale = np.abs(F1).max() + max(qa[4], qb[4])
            assert np.all(np.abs(F2 - sgn * F1) <= 1e-12 * scale)
    # supersonic states: pure upwinding
    g, pc = AIR
    qL = np.array([1.0, 2000.0, 10.0, 5.0, 1e5])
    qR = np.array([0.5, 1900.0, -3.0, 1.0, 2e5])
    assert np.allclose(_hllc(lib, qL, qR, g, pc), euler_flux_def(qL, g, pc), rtol=1e-14)
    qL[1], qR[1] = -2000.0, -2100.0
    assert np.allclose(_hllc(lib, qL, qR, g, pc), euler_flux_def(qR, g, pc), rtol=1e-14)


def _llf(lib, qL, qR, g, pc):
    F = np.empty(5)
    lib.ora_llf(np.asarray(qL, float), np.asarray(qR, float), g, pc, F)
    return F


def check_van_albada(lib):
    """Van Albada slopes (appendix "Slope limiters"): for k = 2 the textbook
    symmetric form d- d+ (d- + d+) / (d-^2 + d+^2); symmetric in (d-, d+)
    for every k; exact on linear data; a hand-evaluated value for k = 4; the
    modified limiter keeps the slope where phi >= 0 and zeroes it elsewhere."""
    rng = np.random.default_rng(21)
    for _ in range(2000):
        a, b = rng.normal(size=2) * 10.0 ** rng.uniform(-3, 3, size=2)
        s2 = lib.ora_va_slope(a, b, 2, 0)
        ref = a * b * (a + b) / (a * a + b * b)
        assert abs(s2 - ref) <= 1e-14 * (abs(a) + abs(b))
        for k in (2, 4):
            assert abs(lib.ora_va_slope(a, b, k, 0) - lib.ora_va_slope(b, a, k, 0)) <= 1e-14 * (abs(a) + abs(b))
            sk, sm = lib.ora_va_slope(a, b, k, 0), lib.ora_va_slope(a, b, k, 1)
            assert sm == (sk if sk * b >= 0 else 0.0)
    for d in (1e-3, 2.5, -7.0):
        for k in (2, 4):
            assert lib.ora_va_slope(d, d, k, 0) == pytest.approx(d, rel=1e-15)
    # theta = 2, k = 4: phi = (16 + 2) / (16 + 1)
    assert lib.ora_va_slope(2.0, 1.0, 4, 0) == pytest.approx(18.0 / 17.0, rel=1e-15)
    assert lib.ora_va_slope(1.0, 0.0, 2, 0) == 0.0


def check_llf_properties(lib):
    """Local Lax-Friedrichs (appendix "Local Lax-Friedrichs flux"):
    consistency, mirror symmetry, and the stationary contact, where the two
    physical fluxes are (0, p, 0, 0, 0) and only the dissipation acts:
    mass flux -max(c_L, c_R) (rho_R - rho_L) / 2."""
    rng = np.random.default_rng(5)
    for mat, (g, pc) in enumerate([AIR, WATER]):
        for _ in range(300):
            q = _rand_state(rng, mat)
            F = _llf(lib, q, q, g, pc)
            Fd = euler_flux_def(q, g, pc)
            assert np.all(np.abs(F - Fd) <= 1e-13 * np.abs(Fd).max())
            qa, qb = _rand_state(rng, mat), _rand_state(rng, mat)
            F1 = _llf(lib, qa, qb, g, pc)
            ma, mb = qa.copy(), qb.copy()
            ma[1] *= -1
            mb[1] *= -1
            F2 = _llf(lib, mb, ma, g, pc)
            sgn = np.array([-1, 1, -1, -1, -1])
            assert np.all(np.abs(F2 - sgn * F1) <= 1e-12 * (np.abs(F1).max() + max(qa[4], qb[4])))
            # stationary contact
            qL, qR = _rand_state(rng, mat), _rand_state(rng, mat)
            qL[1:4] = 0.0
            qR[1:4] = 0.0
            qR[4] = qL[4]
            F = _llf(lib, qL, qR, g, pc)
            cmax = max(math.sqrt(g * (qL[4] + pc) / qL[0]), math.sqrt(g * (qR[4] + pc) / qR[0]))
            assert F[0] == pytest.approx(-0.5 * cmax * (qR[0] - qL[0]), rel=1e-13, abs=1e-12 * cmax * qR[0])
            assert F[1] == pytest.approx(qL[4], rel=1e-14)
            assert F[2] == 0.0 and F[3] == 0.0


def check_riemann_vs_independent(lib, nprob=150, seed=11):
    inp, eos = W.riemann_problem_set(seed, nprob)
    nvac = 0
    for i in range(nprob):
        st = ex.star_state(inp[i], eos[i])
        rc, out, it = _riemann(lib, inp[i], eos[i])
        if st is None:
            nvac += 1
            assert rc == oracle.ERR_RIEMANN
            continue
        assert rc == oracle.OK and it > 0
        plo = -min(eos[i, 1], eos[i, 3])
        uscale = abs(inp[i, 1]) + abs(inp[i, 4]) + math.sqrt((st[0] - plo) / min(inp[i, 0], inp[i, 3]))
        assert abs(out[0] - st[0]) <= 1e-11 * (st[0] - plo)
        assert abs(out[1] - st[1]) <= 1e-11 * uscale
        assert abs(out[2] - st[2]) <= 1e-11 * st[2]
        assert abs(out[3] - st[3]) <= 1e-11 * st[3]
    assert nvac < nprob // 4


def _rhoE(rho, u, p, g, pc):
    return (p + g * pc) / (g - 1) + 0.5 * rho * u * u


def check_riemann_jump_conditions(lib, nprob=300, seed=12):
    """Shock sides satisfy the Rankine-Hugoniot conditions of mass,
    momentum and energy; rarefaction sides keep (p + p_c) rho^-gamma and the
    Riemann invariant u -+ 2c/(gamma - 1)."""
    inp, eos = W.riemann_problem_set(seed, nprob)
    nshock = nrare = 0
    for i in range(nprob):
        rc, out, _ = _riemann(lib, inp[i], eos[i])
        if rc != oracle.OK:
            continue
        ps, us, rsL, rsR = out
        for side in (0, 1):
            r, u, p = inp[i, 3 * side: 3 * side + 3]
            g, pc = eos[i, 2 * side: 2 * side + 2]
            rs = rsL if side == 0 else rsR
            if ps > p * (1 + 1e-9):
                nshock += 1
                S = (rs * us - r * u) / (rs - r)
                mom = (rs * us * us + ps) - (r * u * u + p) - S * (rs * us - r * u)
                Es, E0 = _rhoE(rs, us, ps, g, pc), _rhoE(r, u, p, g, pc)
                en = us * (Es + ps) - u * (E0 + p) - S * (Es - E0)
                assert abs(mom) <= 1e-10 * (abs(ps - p) + r * u * u + rs * us * us)
                assert abs(en) <= 1e-9 * (abs(us) + abs(u) + abs(S)) * (abs(Es) + abs(E0) + ps + p)
            elif ps < p * (1 - 1e-9):
                nrare += 1
                assert abs((ps + pc) / rs ** g / ((p + pc) / r ** g) - 1) <= 1e-11
                cs, c0 = math.sqrt(g * (ps + pc) / rs), math.sqrt(g * (p + pc) / r)
                sg = 1.0 if side == 0 else -1.0
                J0 = u + sg * 2 * c0 / (g - 1)
                Js = us + sg * 2 * cs / (g - 1)
                assert abs(Js - J0) <= 1e-10 * (abs(J0) + c0)
    assert nshock > 20 and nrare > 20


def check_riemann_special_cases(lib):
    # identical states: p* = p, u* = u, no waves
    for (g, pc), r, u, p in [(AIR, 1.2, 30.0, 2e5), (WATER, 1000.0, -5.0, 3e7)]:
        rc, out, _ = _riemann(lib, [r, u, p, r, u, p], [g, pc, g, pc])
        assert rc == 0
        assert out[0] == pytest.approx(p, rel=1e-13)
        assert out[1] == pytest.approx(u, rel=1e-12, abs=1e-9)
        assert out[2] == pytest.approx(r, rel=1e-12) and out[3] == pytest.approx(r, rel=1e-12)
    # mirror-symmetric collision of equal states: contact at rest
    rc, out, _ = _riemann(lib, [1000, 40, 1e6, 1000, -40, 1e6], [*WATER, *WATER])
    assert rc == 0 and abs(out[1]) <= 1e-9 and out[2] == pytest.approx(out[3], rel=1e-12)
    # uniform u and p across two materials (the interface condition of eq.
    # interface_cond is already met): the star state is the data
    rc, out, _ = _riemann(lib, [1000, 12, 5e5, 1.0, 12, 5e5], [*WATER, *AIR])
    assert rc == 0 and out[0] == pytest.approx(5e5, rel=1e-12)
    assert out[1] == pytest.approx(12, rel=1e-10)
    assert out[2] == pytest.approx(1000, rel=1e-12) and out[3] == pytest.approx(1.0, rel=1e-12)
    # strongly separating air: vacuum detected
    rc, _, _ = _riemann(lib, [1.0, -2000, 1e5, 1.0, 2000, 1e5], [*AIR, *AIR])
    assert rc == oracle.ERR_RIEMANN
    # maxit = 1 forces the bisection fallback; same star pressure to rtol
    inp = [1000, 0, 4e8, 1.0, 0, 1e5]
    rc1, o1, it1 = _riemann(lib, inp, [*WATER, *AIR])
    rc2, o2, it2 = _riemann(lib, inp, [*WATER, *AIR], maxit=1)
    assert rc1 == rc2 == 0 and it1 > 1 and it2 < 0
    assert o2[0] == pytest.approx(o1[0], rel=1e-11)


def check_ls_derivative(lib):
    rng = np.random.default_rng(5)
    h = 0.37
    for _ in range(100):
        c = rng.normal(size=4)
        x0 = rng.normal()
        xs = x0 + h * np.arange(-2, 3)
        f = c[0] + c[1] * xs + c[2] * xs ** 2 + c[3] * xs ** 3
        exact = c[1] + 2 * c[2] * x0 + 3 * c[3] * x0 ** 2
        scale = np.abs(f).max() / h + abs(exact)
        for v in (1.0, -1.0):
            assert abs(lib.ora_ls_derivative(f, v, h) - exact) <= 1e-13 * scale
        assert lib.ora_ls_derivative(f, 0.0, h) == 0.0
    # quartic data: the one-sided stencils are not exact (third order only)
    xs = h * np.arange(-2, 3)
    f = xs ** 4
    assert lib.ora_ls_derivative(f, 1.0, h) != 0.0


def _sim(problem, lib, **kw):
    return oracle.OracleSim(problem, lib_handle=lib, **kw)


def check_dt_uniform(lib):
    p = W.periodic_box(0, n=(8, 6, 4))
    g, pc = p.gamma[0], p.pc[0]
    p.prim[:] = 0
    p.prim[0], p.prim[1], p.prim[2], p.prim[3], p.prim[4], p.prim[5] = 1.3, 40.0, -25.0, 10.0, 2e5, 1.0
    s = _sim(p, lib)
    c = math.sqrt(g * (2e5 + pc) / 1.3)
    lam = (40 + c) * 8 + (25 + c) * 6 + (10 + c) * 4
    assert s.dt() == pytest.approx(p.cfl / lam, rel=1e-14)


def check_conservation_periodic(lib):
    for seed, mat, order in [(0, 0, 2), (1, 1, 2), (3, 0, 3)]:
        p = W.periodic_box(seed, material=mat, n=(12, 10, 8))
        s = _sim(p, lib, rk_order=order)
        c0 = s.cons().reshape(6, -1)
        assert s.step(15) == 0
        c1 = s.cons().reshape(6, -1)
        for v in range(5):
            tot0, tot1 = c0[v].sum(), c1[v].sum()
            scale = np.abs(c0[v]).sum()
            assert abs(tot1 - tot0) <= 64 * 15 * np.finfo(float).eps * scale, v


def check_rk_temporal_order(lib):
    """Forward Euler, TVD-RK2 and TVD-RK3 (section "Time integration")
    converge at orders 1, 2 and 3 in dt on a linear semi-discrete system: a
    uniform flow carrying a smooth level set (every face sees the same two
    states, so the fluid residual is exactly zero, and the level-set
    operator is linear in phi)."""
    n = 32
    p = W.periodic_box(0, n=(n, 1, 1))
    x = (np.arange(n) + 0.5) / n
    p.prim[0], p.prim[1], p.prim[2], p.prim[3], p.prim[4] = 1000.0, 1.0, 0.0, 0.0, 1e5
    p.prim[5] = (2.0 + np.sin(2.0 * np.pi * x)).reshape(1, 1, n)
    T = 0.5 / n                                  # half a cell at u = 1

    def run(order, steps):
        s = _sim(p, lib, rk_order=order)
        assert s.step_dt(steps, T / steps) == 0
        out = s.cons()
        assert np.all(out[1] == out[1].ravel()[0])   # the flow stays exactly uniform
        return out[5].ravel()

    ref = run(3, 1280)
    for order in (1, 2, 3):
        e = [np.max(np.abs(run(order, m) - ref)) for m in (10, 20, 40)]
        rates = [math.log2(e[0] / e[1]), math.log2(e[1] / e[2])]
        assert all(abs(r - order) < 0.25 for r in rates), (order, e, rates)


def check_conservation_wall(lib):
    p = W.periodic_box(2, material=0, n=(10, 8, 6), bc=W.BC_WALL)
    s = _sim(p, lib)
    c0 = s.cons().reshape(6, -1)
    assert s.step(15) == 0
    c1 = s.cons().reshape(6, -1)
    for v in (0, 4):
        scale = np.abs(c0[v]).sum()
        assert abs(c1[v].sum() - c0[v].sum()) <= 64 * 15 * np.finfo(float).eps * scale


def check_uniform_translation(lib):
    """Two materials in uniform velocity and pressure: FIVER keeps u and p
    uniform and the interface moves with the flow."""
    for axis in (0, 1, 2):
        p = W.uniform_translation(n=100, axis=axis, velocity=50.0, pressure=1e5)
        s = _sim(p, lib)
        for _ in range(6):
            assert s.step(10) == 0
            q, chi = s.prim()
            assert np.max(np.abs(q[1 + axis] - 50.0)) <= 1e-9 * 50
            assert np.max(np.abs(q[4] - 1e5)) <= 1e-8 * 1e5
        t = s.stats()["t"]
        water = (chi.reshape(-1) == 1)
        x = (np.arange(100) + 0.5) / 100
        lo_edge = x[water].min() - 0.005
        assert abs(lo_edge - (0.25 + 50.0 * t)) <= 1.0 / 100 + 1e-12
        assert s.stats()["flips"] > 0 and s.stats()["orphans"] == 0


def check_axis_permutation(lib):
    res = []
    for axis in (0, 1, 2):
        p = W.uniform_translation(n=80, axis=axis, velocity=0.0, pressure=1e5, periodic=False)
        # a pressure jump inside the water slab drives waves through the interface
        prim = p.prim.reshape(6, -1)
        s_coord = (np.arange(80) + 0.5) / 80
        prim[4] = np.where(s_coord < 0.5, 5e8, 1e5)
        p.prim = prim.reshape(p.prim.shape)
        s = _sim(p, lib)
        assert s.step(40) == 0
        q, _ = s.prim()
        res.append((q[0].reshape(-1).copy(), q[1 + axis].reshape(-1).copy(), q[4].reshape(-1).copy()))
    for k in range(3):
        assert np.array_equal(res[0][k], res[1][k]) and np.array_equal(res[0][k], res[2][k])


def _run_to_time(s, T, max_steps=5000):
    t = 0.0
    for _ in range(max_steps):
        dt = s.dt()
        assert dt > 0.0 and math.isfinite(dt)
        if t + dt >= T:
            assert s.step_dt(1, T - t) == 0
            return
        assert s.step(1) == 0
        t += dt
    raise AssertionError("time target not reached")


def check_shock_tube_exact(lib, seeds=(0, 1, 2), Ns=(250, 1000), **opts):
    """The scheme converges to the exact two-material solution (section
    "One-dimensional Riemann problems"): L1 errors of u and p against exact
    cell averages shrink with the grid and are small at 1000 cells."""
    T = 2.0e-5
    for seed in seeds:
        errs = []
        for N in Ns:
            p = W.shock_tube_1d(seed, nx=N)
            s = _sim(p, lib, **opts)
            _run_to_time(s, T)
            q, _ = s.prim()
            inp = [1000.0, 0.0, p.meta["pL"], 1.0, 0.0, 1e5]
            ra, ua, pa = ex.cell_averages(inp, [*WATER, *AIR], 0.5, T, np.linspace(0, 1, N + 1))
            eu = np.mean(np.abs(q[1, 0, 0] - ua)) / max(np.abs(ua).max(), 1e-30)
            ep = np.mean(np.abs(q[4, 0, 0] - pa)) / np.abs(pa).max()
            errs.append((eu, ep))
        assert errs[-1][0] < 1.5e-2 and errs[-1][1] < 1.5e-2, errs
        assert errs[0][0] > 2.0 * errs[-1][0] and errs[0][1] > 2.0 * errs[-1][1], errs


def check_interface_faces_listing(lib):
    p = W.shock_bubble(0, n=16)
    s = _sim(p, lib)
    f = s.interface_faces()
    chi = (p.prim[5] < 0).astype(np.uint8).reshape(-1)
    n = 16
    ref = []
    for c in range(n ** 3):
        i, j, k = c % n, (c // n) % n, c // (n * n)
        for d, (ok, nb) in enumerate([(i + 1 < n, c + 1), (j + 1 < n, c + n), (k + 1 < n, c + n * n)]):
            if ok and chi[c] != chi[nb]:
                ref.append(3 * c + d)
    assert np.array_equal(f, np.array(ref, dtype=np.int32))


CHECKS = {
    "eos_roundtrip": check_eos_roundtrip,
    "sound_speed": check_sound_speed,
    "mc_limiter": check_mc_limiter,
    "hllc_properties": check_hllc_properties,
    "riemann_vs_independent": check_riemann_vs_independent,
    "riemann_jump_conditions": check_riemann_jump_conditions,
    "riemann_special_cases": check_riemann_special_cases,
    "ls_derivative": check_ls_derivative,
    "dt_uniform": check_dt_uniform,
    "conservation_periodic": check_conservation_periodic,
    "conservation_wall": check_conservation_wall,
    "rk_temporal_order": check_rk_temporal_order,
    "uniform_translation": check_uniform_translation,
    "axis_permutation": check_axis_permutation,
    "shock_tube_exact": check_shock_tube_exact,
    "shock_tube_exact_llf_van_albada": lambda lib: check_shock_tube_exact(
        lib, seeds=(0, 2), limiter=oracle.LIM_VA, limiter_k=2, flux=oracle.FLUX_LLF),
    "shock_tube_exact_modified_van_albada": lambda lib: check_shock_tube_exact(
        lib, seeds=(1,), limiter=oracle.LIM_VA_MOD, limiter_k=4),
    "van_albada": check_van_albada,
    "llf_properties": check_llf_properties,
    "interface_faces_listing": check_interface_faces_listing,
}


@pytest.mark.parametrize("name", list(CHECKS))
def test_oracle_pin(name, oracle_lib):
    CHECKS[name](oracle_lib)


def test_narrow_band_level_set():
    """Narrow band (section "Level set method"): phi is held outside the band
    and the run equals the whole-grid run when the band covers everything."""
    p = W.shock_bubble(5, nxyz=(20, 18, 16), radius=0.25, p_shock=1e9, shock_x=0.3)
    band = 2.5 * min(p.dx())
    full = oracle.OracleSim(p)
    wide = oracle.OracleSim(p, ls_band=1e9)
    narrow = oracle.OracleSim(p, ls_band=band)
    for s in (full, wide, narrow):
        assert s.step(12) == 0
    assert np.array_equal(full.cons(), wide.cons())
    phi0 = p.prim[5]
    out = np.abs(phi0) >= band
    wn, wf = narrow.cons(), full.cons()
    assert out.any() and np.array_equal(wn[5][out], phi0[out])
    assert not np.array_equal(wf[5][out], phi0[out])          # the whole-grid run moves them
    inner = np.abs(phi0) < band
    assert not np.array_equal(wn[5][inner], phi0[inner])


# ------------------------------------------------------ planted mistakes ---
# (source fragment, replacement) pairs: each plants a plausible mistake in a
# private copy of the oracle; the pins must catch every one.
MUTANTS = [
    ("star energy sign", "(Ss - uL) * (Ss + pL", "(Ss + uL) * (Ss + pL"),
    ("Davis speed", "double SR = fmax(uL + cL, uR + cR);", "double SR = fmax(uL + cL, uR);"),
    ("shock wave function", "return (p - s->p) * q;", "return (p - s->p) * q * 1.0001;"),
    ("rarefaction exponent", "(pow(r, (g - 1.0) / (2.0 * g)) - 1.0)", "(pow(r, (g - 1.0) / (g)) - 1.0)"),
    ("FIVER argument order", "num_flux(&s->c, sb, qb, xb, Fr_u)", "num_flux(&s->c, qb, sb, xb, Fr_u)"),
    ("FIVER EOS side", "num_flux(&s->c, qa, sa, xa, Fr_l)", "num_flux(&s->c, qa, sa, xb, Fr_l)"),
    ("MC limiter middle term", "B / (A + 1.0) * (theta + 1.0)", "B / A * (theta + 1.0)"),
    ("face value half slope", "la[v] = qa[v] + 0.5 * sa;", "la[v] = qa[v] + sa;"),
    ("level-set stencil", "(2.0 * f[3] + 3.0 * f[2] - 6.0 * f[1] + f[0])", "(2.0 * f[3] + 3.0 * f[2] - 6.0 * f[1] + 2.0 * f[0])"),
    ("flux difference order", "R[v][c] += (FL[i + 1][v] - FU[i][v]) / s->h[d];", "R[v][c] += (FU[i + 1][v] - FL[i][v]) / s->h[d];"),
    ("RK2 weight", "0.5 * W0[v][c] + 0.5 * (W1[v][c] + dt * R[v][c])", "0.5 * W0[v][c] + 0.5 * (W1[v][c] + 0.9 * dt * R[v][c])"),
    ("Van Albada numerator", "B * (tk + theta) / (tk + A)", "B * (tk - theta) / (tk + A)"),
    ("LLF dissipation sign", "- 0.5 * lmax * (UR[v] - UL[v])", "+ 0.5 * lmax * (UR[v] - UL[v])"),
    ("LLF state jump", "UL[1] = qL[0] * qL[1];", "UL[1] = qL[1];"),
    ("RK3 middle weight", "0.75 * W0[v][c] + 0.25 * W1[v][c]", "0.75 * W0[v][c] + 0.26 * W1[v][c]"),
    ("RK3 level-set last weight", "phi0[c] / 3.0 + 2.0 / 3.0 * phi2[c] + 2.0 / 3.0 * dt * L[c]",
     "phi0[c] / 3.0 + 2.0 / 3.0 * phi2[c] + 0.6 * dt * L[c]"),
    ("EOS gamma p_c term", "q[4] = (gamma - 1.0) * rho * e - gamma * pc;", "q[4] = (gamma - 1.0) * rho * e - pc;"),
    ("HLLC contact speed numerator", "rL * uL * (SL - uL) - rR * uR * (SR - uR)) /",
     "rL * uL * (SL - uL) + rR * uR * (SR - uR)) /"),
    # the zero-slope rule next to an interface (reading of section "Spatial
    # discretization": the projected states of eq. 1DRiemannProblem are the
    # cell states), dropped on both sides or on one
    ("slope across the interface, both cells",
     ("int flat_a = s->X[pa - stride] != xa || s->X[pa + stride] != xa;",
      "int flat_b = s->X[pb - stride] != xb || s->X[pb + stride] != xb;"),
     ("int flat_a = 0;", "int flat_b = 0;")),
    ("slope across the interface, upper cell",
     "int flat_b = s->X[pb - stride] != xb || s->X[pb + stride] != xb;", "int flat_b = 0;"),
    ("slope across the interface, lower cell",
     "int flat_a = s->X[pa - stride] != xa || s->X[pa + stride] != xa;", "int flat_a = 0;"),
    # the phase update (outline step 6 of section "Code structure")
    ("phase update keeps the old normal velocity", "q[1 + d] = r->ustar;",
     "q[1 + d] = side ? r->VR[d] : r->VL[d];"),
    ("phase update takes the other side's star density", "q[0] = side ? r->rhoR : r->rhoL;",
     "q[0] = side ? r->rhoL : r->rhoR;"),
    ("phase update takes the other side's velocity", "for (int a = 0; a < 3; ++a) q[1 + a] = side ? r->VR[a] : r->VL[a];",
     "for (int a = 0; a < 3; ++a) q[1 + a] = side ? r->VL[a] : r->VR[a];"),
]


@pytest.fixture(scope="module")
def mutant_dir():
    d = tempfile.mkdtemp(prefix="oracle_mut_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


def _all_checks():
    """The pins of this file, then the high-precision brute-force pins
    (slower; a mutant is reported caught at its first failing check)."""
    from tests import test_oracle_bruteforce as BF
    return [*CHECKS.items(), *BF.CHECKS.items()]


@pytest.mark.parametrize("label,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistakes(label, old, new, mutant_dir):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "m2c_oracle.c")).read()
    olds, news = (old, new) if isinstance(old, tuple) else ((old,), (new,))
    for o, n in zip(olds, news):
        assert src.count(o) == 1, (label, o)
        src = src.replace(o, n)
    mdir = os.path.join(mutant_dir, label.replace(" ", "_").replace("'", ""))
    os.makedirs(mdir, exist_ok=True)
    shutil.copy(os.path.join(os.path.dirname(oracle.__file__), "m2c_oracle.h"), mdir)
    with open(os.path.join(mdir, "m2c_oracle.c"), "w") as f:
        f.write(src)
    so = os.path.join(mdir, "libmut.so")
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-o", so,
                    os.path.join(mdir, "m2c_oracle.c"), "-lm"], check=True)
    lib = oracle.load(so)
    caught = None
    for name, chk in _all_checks():
        try:
            chk(lib)
        except (AssertionError, ValueError):
            caught = name
            break
    assert caught, f"planted mistake '{label}' passed every pin"
