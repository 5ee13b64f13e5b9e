"""High-precision brute-force pins of the oracle: single-face fluxes, the
zero-slope rule next to a material interface and the phase update.

Every reference value here is computed with mpmath at 30 significant digits
straight from the paper's statements, not from the oracle's formulas:

* the stiffened-gas EOS (eq. NASG_EOS with b = e_c = 0) and its sound speed;
* the MC limiter in its printed phi(theta) form (appendix "Slope limiters",
  eqs. theta and AB with uniform widths);
* the four-case HLLC flux of appendix "HLLC flux" with the Davis speeds and
  contact speed as printed and the star energy of the cited source (Toro);
* the two-material Riemann problem of eq. 1DRiemannProblem, solved from its
  jump conditions (Hugoniot energy relation by bisection on the density,
  mass and momentum for the velocity jump) and, across rarefactions, by
  quadrature of dp / (rho c) along the isentrope, with a bracketed root
  search for the star pressure -- the oracle uses closed-form wave curves
  and Newton's method instead.

The grid checks follow one forward-Euler step of the scheme by hand on a 1D
two-material line: primitive reconstruction whose slope vanishes in a cell
with an axis neighbour of the other material (so that the states projected
into eq. 1DRiemannProblem are the cell states), HLLC at single-material
faces, the two one-sided FIVER fluxes at the interface face ordered along the
face normal, the conservative update of eq. NS_discretized, the third-order
upwind level-set update, and the phase update of step 6 of the time-step
outline (section "Code structure and workflow"): a flipped cell takes the
star state of its new material's side -- density rho*_B, normal velocity u*,
pressure p*, the B cell's tangential velocity.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import exact_riemann as ex

WATER, AIR = W.WATER, W.AIR
mp.mp.dps = 30
M = mp.mpf


# ------------------------------------------------------------ references ---

def mp_rhoE(q, g, pc):
    """rho E of a primitive state (rho, u, v, w, p): rho e = (p + g p_c)/(g - 1)."""
    r, u, v, w, p = q
    return (p + g * pc) / (g - 1) + r * (u * u + v * v + w * w) / 2


def mp_prim(wc, g, pc):
    """Primitive state of a conservative one (rho, rho u, rho v, rho w, rho E)."""
    r = wc[0]
    u, v, w = wc[1] / r, wc[2] / r, wc[3] / r
    p = (g - 1) * (wc[4] - r * (u * u + v * v + w * w) / 2) - g * pc
    return [r, u, v, w, p]


def mp_cons(q, g, pc):
    r, u, v, w, p = q
    return [r, r * u, r * v, r * w, mp_rhoE(q, g, pc)]


def mp_c(r, p, g, pc):
    return mp.sqrt(g * (p + pc) / r)


def mp_phys_flux(q, E):
    r, u, v, w, p = q
    return [r * u, r * u * u + p, r * u * v, r * u * w, (E + p) * u]


def mp_hllc(qL, qR, g, pc):
    """Appendix "HLLC flux", face frame (rho, u_n, v_t1, v_t2, p); returns the
    flux and a per-component magnitude of the terms it sums."""
    qL = [M(x) for x in qL]
    qR = [M(x) for x in qR]
    g, pc = M(g), M(pc)
    rL, uL, pL = qL[0], qL[1], qL[4]
    rR, uR, pR = qR[0], qR[1], qR[4]
    cL, cR = mp_c(rL, pL, g, pc), mp_c(rR, pR, g, pc)
    EL, ER = mp_rhoE(qL, g, pc), mp_rhoE(qR, g, pc)
    SL = min(uL - cL, uR - cR)
    SR = max(uL + cL, uR + cR)
    Ss = (pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR)) / (rL * (SL - uL) - rR * (SR - uR))

    def star_flux(q, E, S):
        r, u, v, w, p = q
        fac = r * (S - u) / (S - Ss)
        Es = E / r + (Ss - u) * (Ss + p / (r * (S - u)))
        Us = [fac, fac * Ss, fac * v, fac * w, fac * Es]
        U = [r, r * u, r * v, r * w, E]
        F = mp_phys_flux(q, E)
        return [F[k] + S * (Us[k] - U[k]) for k in range(5)]

    if 0 <= SL:
        F = mp_phys_flux(qL, EL)
    elif SL <= 0 <= Ss:
        F = star_flux(qL, EL, SL)
    elif Ss <= 0 <= SR:
        F = star_flux(qR, ER, SR)
    else:
        F = mp_phys_flux(qR, ER)
    UL, UR = mp_cons(qL, g, pc), mp_cons(qR, g, pc)
    FL, FR = mp_phys_flux(qL, EL), mp_phys_flux(qR, ER)
    Smax = max(abs(SL), abs(SR))
    scale = [abs(FL[k]) + abs(FR[k]) + Smax * (abs(UL[k]) + abs(UR[k])) for k in range(5)]
    return F, scale


def mp_mc(dm, dp, alpha):
    """phi(theta) (w_{i+1} - w_i), eq. theta with A = B = 1 (uniform grid)."""
    dm, dp, alpha = M(dm), M(dp), M(alpha)
    if dp == 0:
        return M(0)
    th = dm / dp
    A = B = M(1)
    phi = max(M(0), min(alpha * th, B / (A + 1) * (th + 1), alpha))
    return phi * dp


def _bisect(f, a, b, iters=120):
    fa = f(a)
    for _ in range(iters):
        m = (a + b) / 2
        fm = f(m)
        if (fm < 0) == (fa < 0):
            a, fa = m, fm
        else:
            b = m
    return (a + b) / 2


def mp_shock_rho(p, r0, p0, g, pc):
    """Density behind a shock of pressure p from (r0, p0): root of the
    Hugoniot energy relation e(r, p) - e(r0, p0) = (p + p0)/2 (1/r0 - 1/r)."""
    def e(r, pp):
        return (pp + g * pc) / ((g - 1) * r)

    def hug(r):
        return e(r, p) - e(r0, p0) - (p + p0) / 2 * (1 / r0 - 1 / r)
    hi = r0 * (g + 1) / (g - 1)
    return _bisect(hug, r0, hi * (1 - M(10) ** -25))


def mp_isentrope_rho(p, r0, p0, g, pc):
    return r0 * ((p + pc) / (p0 + pc)) ** (1 / g)


def mp_wave(p, r0, u0, p0, g, pc):
    """Velocity decrease from side state 0 to the star region at pressure p
    (positive through a shock)."""
    if p > p0:
        rs = mp_shock_rho(p, r0, p0, g, pc)
        return mp.sqrt((p - p0) * (1 / r0 - 1 / rs))
    if p == p0:
        return M(0)

    def integrand(pp):
        r = mp_isentrope_rho(pp, r0, p0, g, pc)
        return 1 / (r * mp_c(r, pp, g, pc))
    return -mp.quad(integrand, [p, p0])


def mp_star(qL, qR, eosL, eosR):
    """Star state (p*, u*, rho*_L, rho*_R) of eq. 1DRiemannProblem for
    (rho, u, p) on each side."""
    rL, uL, pL = (M(x) for x in qL)
    rR, uR, pR = (M(x) for x in qR)
    gL, pcL = (M(x) for x in eosL)
    gR, pcR = (M(x) for x in eosR)
    plo = -min(pcL, pcR)

    def gfun(p):
        return mp_wave(p, rL, uL, pL, gL, pcL) + mp_wave(p, rR, uR, pR, gR, pcR) + (uR - uL)
    a = plo + (max(pL, pR) - plo) * M(10) ** -20
    assert gfun(a) < 0, "vacuum"
    b = max(pL, pR)
    while gfun(b) < 0:
        b = plo + 2 * (b - plo)
    ps = mp.findroot(gfun, (a, b), solver="anderson", tol=M(10) ** -26, maxsteps=200)
    us = (uL + uR) / 2 + (mp_wave(ps, rR, uR, pR, gR, pcR) - mp_wave(ps, rL, uL, pL, gL, pcL)) / 2
    rsL = mp_shock_rho(ps, rL, pL, gL, pcL) if ps > pL else mp_isentrope_rho(ps, rL, pL, gL, pcL)
    rsR = mp_shock_rho(ps, rR, pR, gR, pcR) if ps > pR else mp_isentrope_rho(ps, rR, pR, gR, pcR)
    return ps, us, rsL, rsR


def mp_ls_derivative(f, V, h):
    """Third-order upwind-biased difference of the level set (reading of
    section "Level set method": four-point stencils exact on cubics, upwinded
    by the cell velocity)."""
    if V > 0:
        return (2 * f[3] + 3 * f[2] - 6 * f[1] + f[0]) / (6 * h)
    if V < 0:
        return (-f[4] + 6 * f[3] - 3 * f[2] - 2 * f[1]) / (6 * h)
    return M(0)


def mp_fe_step_1d(W0, mat, eos, h, dt, alpha=1.2):
    """One forward-Euler step of the scheme on a line of cells with
    transmissive ends (two zero-gradient images per end), written out by
    hand.  W0: (6, n) conservative state and phi as doubles; mat: material
    ids; eos: ((gamma, p_c) of material 0, of material 1)."""
    n = W0.shape[1]
    h, dt = M(h), M(dt)
    q = [mp_prim([M(W0[v, i]) for v in range(5)], M(eos[mat[i]][0]), M(eos[mat[i]][1])) for i in range(n)]
    phi = [M(W0[5, i]) for i in range(n)]

    def img(i):                       # transmissive image index
        return min(max(i, 0), n - 1)

    def slope(i, v):
        a, b, c = img(i - 1), img(i), img(i + 1)
        if mat[a] != mat[b] or mat[c] != mat[b]:
            return M(0)               # no stencil crosses the interface
        return mp_mc(q[b][v] - q[a][v], q[c][v] - q[b][v], alpha)

    # flux seen by the cell below (FL) and above (FU) face m, m = 0..n, the
    # face between cells m-1 and m
    FL, FU = [], []
    for m in range(n + 1):
        a, b = img(m - 1), img(m)
        if mat[a] == mat[b]:
            la = [q[a][v] + slope(m - 1, v) / 2 for v in range(5)]
            rb = [q[b][v] - slope(m, v) / 2 for v in range(5)]
            F, _ = mp_hllc(la, rb, *eos[mat[a]])
            FL.append(F)
            FU.append(F)
        else:
            ps, us, rsa, rsb = mp_star((q[a][0], q[a][1], q[a][4]), (q[b][0], q[b][1], q[b][4]),
                                       eos[mat[a]], eos[mat[b]])
            sa = [rsa, us, q[a][2], q[a][3], ps]
            sb = [rsb, us, q[b][2], q[b][3], ps]
            FL.append(mp_hllc(q[a], sa, *eos[mat[a]])[0])
            FU.append(mp_hllc(sb, q[b], *eos[mat[b]])[0])
    out = np.empty((6, n), dtype=object)
    for i in range(n):
        w = [M(W0[v, i]) for v in range(5)]
        for v in range(5):
            out[v, i] = w[v] - dt * (FL[i + 1][v] - FU[i][v]) / h
        f = [phi[img(i + s)] for s in (-2, -1, 0, 1, 2)]
        V = q[i][1]
        out[5, i] = phi[i] - dt * V * mp_ls_derivative(f, V, h)
    return out


# ---------------------------------------------------------------- checks ---
# Each check takes an oracle library handle, so that the planted-mistake test
# of tests/test_oracle_pins.py can run it on a mutated build.

def _rand_face_state(rng, material, fast=False):
    if material == 0:      # air
        u = rng.uniform(-300, 300) + (rng.choice([-1, 1]) * rng.uniform(400, 900) if fast else 0.0)
        return [rng.uniform(0.05, 20), u, rng.uniform(-100, 100), rng.uniform(-100, 100),
                math.exp(rng.uniform(math.log(1e3), math.log(1e8)))]
    u = rng.uniform(-200, 200) + (rng.choice([-1, 1]) * rng.uniform(1500, 3000) if fast else 0.0)
    return [rng.uniform(900, 1200), u, rng.uniform(-50, 50), rng.uniform(-50, 50),
            math.exp(rng.uniform(math.log(1e4), math.log(2e9)))]


def check_hllc_bruteforce(lib, n=600, seed=31):
    """Single-face HLLC fluxes against the appendix transcription at 30
    digits, over subsonic and supersonic pairs of both materials (every one
    of the four cases is hit)."""
    rng = np.random.default_rng(seed)
    cases = set()
    for t in range(n):
        mat = t % 2
        g, pc = (AIR, WATER)[mat]
        fast = (t // 2) % 4 == 3
        qL = _rand_face_state(rng, mat, fast)
        qR = _rand_face_state(rng, mat, fast and rng.uniform() < 0.5)
        F = np.empty(5)
        lib.ora_hllc(np.asarray(qL, float), np.asarray(qR, float), g, pc, F)
        Fm, scale = mp_hllc(qL, qR, g, pc)
        for v in range(5):
            err = abs(M(F[v]) - Fm[v])
            assert err <= M("1e-13") * scale[v], (t, v, qL, qR, float(err / scale[v]))
        # which case of the appendix applies
        cL = math.sqrt(g * (qL[4] + pc) / qL[0])
        cR = math.sqrt(g * (qR[4] + pc) / qR[0])
        SL, SR = min(qL[1] - cL, qR[1] - cR), max(qL[1] + cL, qR[1] + cR)
        cases.add(0 if SL >= 0 else (3 if SR <= 0 else 1))
    assert cases == {0, 1, 3}


def check_mc_bruteforce(lib, n=4000, seed=32):
    """MC slopes against phi(theta) (w_{i+1} - w_i) evaluated at 30 digits:
    equal to within two rounding errors, with exact zeros where phi = 0."""
    rng = np.random.default_rng(seed)
    for t in range(n):
        alpha = (1.2, 1.0, 2.0, 1.5, 0.0)[t % 5]
        dm = rng.normal() * 10.0 ** rng.integers(-3, 4)
        dp = rng.normal() * 10.0 ** rng.integers(-3, 4)
        if t % 17 == 0:
            dp = dm * rng.choice([1.0, -1.0, 0.5, 2.0, 1.0 / 1.2])
        s = lib.ora_mc_slope(dm, dp, alpha)
        ref = mp_mc(dm, dp, alpha)
        if ref == 0:
            assert s == 0.0, (dm, dp, alpha, s)
        else:
            assert abs(M(s) - ref) <= M("4.5e-16") * abs(ref), (dm, dp, alpha, s, float(ref))


def _line_problem(n, mats, prims, phi):
    """A 1D two-material problem on [0, 1] from per-cell primitive states."""
    prim = np.zeros((6, 1, 1, n))
    for i in range(n):
        prim[:5, 0, 0, i] = prims[i]
        prim[5, 0, 0, i] = phi[i]
    return W.Problem(name="line", n=(n, 1, 1), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                     gamma=(AIR[0], WATER[0]), pc=(AIR[1], WATER[1]), bc=(0,) * 6, cfl=0.4,
                     steps=1, prim=prim)


def _two_material_line(seed, n=12):
    """Water (material 1) on the left half, air on the right half, each cell
    with its own random state, so that every limiter regime occurs."""
    rng = np.random.default_rng(seed)
    x = (np.arange(n) + 0.5) / n
    prims, mats = [], []
    for i in range(n):
        if x[i] < 0.5:
            mats.append(1)
            prims.append([rng.uniform(980, 1020), rng.uniform(-5, 5), rng.uniform(-3, 3), rng.uniform(-3, 3),
                          rng.uniform(1e6, 3e6)])
        else:
            mats.append(0)
            prims.append([rng.uniform(1.0, 1.5), rng.uniform(-10, 10), rng.uniform(-3, 3), rng.uniform(-3, 3),
                          rng.uniform(1e5, 2e5)])
    return _line_problem(n, mats, prims, x - 0.5), mats


def check_fe_step_two_material_bruteforce(lib, seeds=(0, 1, 2)):
    """One forward-Euler step of a 1D water/air line against the
    hand-written step at 30 digits (conservative state and phi), including
    the cells next to the interface whose slopes vanish and the interface
    face's FIVER fluxes."""
    for seed in seeds:
        p, mats = _two_material_line(seed)
        s = oracle.OracleSim(p, lib_handle=lib, rk_order=1)
        W0 = s.cons().reshape(6, -1)
        q0, _ = s.prim()
        lam = max(abs(q0[1].reshape(-1)) + np.sqrt(np.where(np.array(mats) == 1, WATER[0], AIR[0])
                                                    * (q0[4].reshape(-1) + np.where(np.array(mats) == 1,
                                                                                     WATER[1], AIR[1]))
                                                    / q0[0].reshape(-1)))
        h = 1.0 / p.n[0]
        dt = 0.4 * h / lam
        assert s.step_dt(1, dt) == 0
        W1 = s.cons().reshape(6, -1)
        ref = mp_fe_step_1d(W0, mats, (AIR, WATER), h, dt)
        for v in range(6):
            scale = max(abs(ref[v, i]) for i in range(p.n[0]))
            err = max(abs(M(W1[v, i]) - ref[v, i]) for i in range(p.n[0]))
            assert err <= M("1e-13") * scale, (seed, v, float(err / scale))


def _flip_line(direction, n=12):
    """Water moving into air: exactly one air cell (phi = +eps) is overrun
    by the level set in one forward-Euler step.  direction +1: water on the
    left moving right; -1: the mirror image."""
    h = 1.0 / n
    water = [1000.0, 50.0 * direction, 3.0, -2.0, 1.0e6]
    air = [1.2, 20.0 * direction, 0.0, 0.0, 1.0e5]
    cw = math.sqrt(WATER[0] * (water[4] + WATER[1]) / water[0])
    dt = 0.4 * h / (cw + 50.0)
    eps = 20.0 * dt / 3.0
    x = (np.arange(n) + 0.5) * h
    if direction > 0:
        flip = n // 2
        x0 = x[flip] - eps
        phi = x - x0                     # water (phi < 0) left of x0
    else:
        flip = n // 2 - 1
        x0 = x[flip] + eps
        phi = x0 - x                     # water right of x0
    mats = [1 if f < 0 else 0 for f in phi]
    prims = [water if m == 1 else air for m in mats]
    return _line_problem(n, mats, prims, phi), flip, dt


def check_phase_update_flip(lib):
    """Phase update (outline step 6 of section "Code structure and
    workflow"): the one cell that changes material in a forward-Euler step
    takes the new material's star state of the interface face it shared
    with its water neighbour -- rho*_water, u*, p* of the independent
    exact solver on the two step-start cell states, and the water cell's
    tangential velocity."""
    for direction in (1, -1):
        p, flip, dt = _flip_line(direction)
        s = oracle.OracleSim(p, lib_handle=lib, rk_order=1)
        q0, chi0 = s.prim()
        q0 = q0.reshape(6, -1)
        nb = flip - direction                  # the water neighbour (material B)
        assert s.step_dt(1, dt) == 0
        st = s.stats()
        q1, chi1 = s.prim()
        q1 = q1.reshape(6, -1)
        chi1 = chi1.reshape(-1)
        assert st["flips"] == 1 and st["orphans"] == 0, st
        assert chi0.reshape(-1)[flip] == 0 and chi1[flip] == 1
        lo, hi = (nb, flip) if direction > 0 else (flip, nb)
        inp = [q0[0, lo], q0[1, lo], q0[4, lo], q0[0, hi], q0[1, hi], q0[4, hi]]
        eos = [*((WATER, AIR)[0 if direction > 0 else 1]), *((AIR, WATER)[0 if direction > 0 else 1])]
        ps, us, rsL, rsR = ex.star_state(inp, eos)
        rs_water = rsL if direction > 0 else rsR
        assert abs(q1[0, flip] - rs_water) <= 1e-11 * rs_water, (direction, q1[0, flip], rs_water)
        assert abs(q1[1, flip] - us) <= 1e-11 * max(abs(us), 1.0), (direction, q1[1, flip], us)
        assert abs(q1[4, flip] - ps) <= 1e-11 * ps, (direction, q1[4, flip], ps)
        for a in (2, 3):
            assert abs(q1[a, flip] - q0[a, nb]) <= 1e-13 * abs(q0[a, nb]), (direction, a)


def check_riemann_mp_vs_oracle(lib, n=12, seed=33):
    """The oracle's Newton star states against the 30-digit jump-condition
    and quadrature solution (water/air in both orders, shocks and
    rarefactions on either side)."""
    rng = np.random.default_rng(seed)
    for t in range(n):
        qw = [rng.uniform(950, 1050), rng.uniform(-50, 50), math.exp(rng.uniform(math.log(1e5), math.log(1e9)))]
        qa = [rng.uniform(0.5, 5.0), rng.uniform(-50, 50), math.exp(rng.uniform(math.log(1e4), math.log(1e7)))]
        if t % 2:
            inp, eos = [*qw, *qa], [*WATER, *AIR]
        else:
            inp, eos = [*qa, *qw], [*AIR, *WATER]
        import ctypes
        out = np.empty(4)
        it = ctypes.c_int32(0)
        rc = lib.ora_riemann(np.asarray(inp, float), np.asarray(eos, float), 1e-12, 50, out, ctypes.byref(it))
        assert rc == 0
        ps, us, rsL, rsR = mp_star(inp[:3], inp[3:], eos[:2], eos[2:])
        plo = -min(eos[1], eos[3])
        assert abs(M(out[0]) - ps) <= M("1e-11") * (ps - plo), t
        assert abs(M(out[1]) - us) <= M("1e-11") * max(abs(us), 1), t
        assert abs(M(out[2]) - rsL) <= M("1e-11") * rsL, t
        assert abs(M(out[3]) - rsR) <= M("1e-11") * rsR, t


CHECKS = {
    "hllc_bruteforce": check_hllc_bruteforce,
    "mc_bruteforce": check_mc_bruteforce,
    "riemann_mp_vs_oracle": check_riemann_mp_vs_oracle,
    "fe_step_two_material_bruteforce": check_fe_step_two_material_bruteforce,
    "phase_update_flip": check_phase_update_flip,
}


@pytest.mark.parametrize("name", list(CHECKS))
def test_bruteforce_pin(name, oracle_lib):
    CHECKS[name](oracle_lib)
