"""Pins of the oracle's general-EOS time step (``oracle/m2c_oracle.c`` with
``eos_general`` set; interface star states from ``oracle/riemann_eos.py``).

Checks against what the equations fix, not against a retyped copy:

* the C closed forms p(rho, e), e(rho, p), c^2(rho, p) of NASG,
  Mie-Grueneisen and JWL agree with the separately written ones of the
  Riemann oracle, and c^2 is the derivative of p along an isentrope (first
  law de = p/rho^2 drho), taken by central differences;
* NASG with b = e_c = 0 is the stiffened gas: a general run of a
  water/air shock tube reproduces the stiffened-gas run;
* a two-material contact in uniform velocity and pressure (Mie-Grueneisen
  against JWL) keeps u and p uniform;
* a JWL/NASG shock tube reaches the exact star state of the Riemann
  problem between its waves, with the shock at the speed the jump
  conditions give and the rarefaction head at u_L - c_L;
* a single-material periodic box of a solid conserves its totals.

``test_planted_mistakes`` plants mistakes in a copy of the C oracle.
"""
from __future__ import annotations

import math
import os
import subprocess

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import riemann_eos as RE

MATERIALS = ["air", "gas_nasg", "water_nasg", "glass", "copper", "tantalum", "tnt"]


def _states(name, n, seed):
    """Admissible (rho, p) samples of a material over its sampling ranges."""
    rng = np.random.default_rng(seed)
    spec = W.EOS_MATERIALS[name]
    eos = RE.make_eos(*W._eos_of(name))
    out = []
    while len(out) < n:
        (rl, rh, rlog), (pl, ph, plog) = spec[2], spec[3]
        u, v = rng.random(2)
        rho = math.exp(math.log(rl) + u * math.log(rh / rl)) if rlog else rl + u * (rh - rl)
        p = math.exp(math.log(pl) + v * math.log(ph / pl)) if plog else pl + v * (ph - pl)
        if p > eos.floor and eos.c2(rho, eos.e(rho, p)) > 0:
            out.append((rho, p))
    return out


def check_eos_closed_forms(lib):
    for name in MATERIALS:
        fam, prm = W._eos_of(name)
        py = RE.make_eos(fam, prm)
        e_struct = oracle.eos_struct(fam, prm)
        for rho, p in _states(name, 40, 3):
            e = lib.ora_eos_e(e_struct, rho, p)
            scale = abs(py.e(rho, p)) + abs(p) / rho
            assert abs(e - py.e(rho, p)) <= 1e-13 * scale, (name, rho, p)
            assert abs(lib.ora_eos_p(e_struct, rho, e) - p) <= 1e-12 * (abs(p) + abs(py.floor) + 1.0), (name, rho, p)
            c2 = lib.ora_eos_c2(e_struct, rho, p)
            assert abs(c2 - py.c2(rho, py.e(rho, p))) <= 1e-11 * c2, (name, rho, p)
        assert lib.ora_eos_floor(e_struct) == py.floor


def check_c2_isentropic(lib):
    """c^2 = dp/drho along de = p/rho^2 drho (central differences)."""
    for name in MATERIALS:
        fam, prm = W._eos_of(name)
        m = oracle.eos_struct(fam, prm)
        for rho, p in _states(name, 12, 5):
            e = lib.ora_eos_e(m, rho, p)
            d = 1e-5 * rho
            # second-order step of de/drho = p/rho^2 from (rho, e) both ways
            def walk(sign):
                r1 = rho + 0.5 * sign * d
                p1 = p + 0.5 * sign * d * lib.ora_eos_c2(m, rho, p)
                e1 = e + sign * d * p1 / (r1 * r1)
                return lib.ora_eos_p(m, rho + sign * d, e1)
            fd = (walk(1) - walk(-1)) / (2 * d)
            c2 = lib.ora_eos_c2(m, rho, p)
            assert abs(fd - c2) <= 2e-5 * c2, (name, rho, p, fd, c2)


def _nasg_as_sg(problem):
    """The same problem with its stiffened gases given as NASG (b = e_c = 0)."""
    import dataclasses
    eos = tuple((0, [problem.gamma[m], problem.pc[m], 0.0, 0.0, 0.0, 0.0, 0.0]) for m in range(2))
    return dataclasses.replace(problem, eos=eos)


def check_nasg_reduces_to_sg(lib):
    p = W.shock_tube_1d(3, nx=120, steps=25)
    a = oracle.OracleSim(p, lib_handle=lib)
    b = oracle.OracleSim(_nasg_as_sg(p), lib_handle=lib)
    assert a.step(25) == 0 and b.step(25) == 0
    wa, wb = a.cons(), b.cons()
    for k in range(6):
        scale = np.abs(wa[k]).max() + (1.0 if k in (1, 2, 3) else 0.0) * np.abs(wa[0]).max() * 10.0
        assert np.abs(wa[k] - wb[k]).max() <= 1e-10 * scale, k
    assert a.stats()["flips"] == b.stats()["flips"]


def contact_problem(u0=1500.0, p0=1e8, nx=60, steps=30):
    return W.eos_shock_tube_1d("copper", "tnt", (8930.0, u0, p0), (1630.0, u0, p0), nx=nx, steps=steps)


def check_uniform_contact(lib):
    import dataclasses
    u0, p0 = 1500.0, 1e8
    p = dataclasses.replace(contact_problem(u0, p0), bc=(2,) * 6)
    o = oracle.OracleSim(p, lib_handle=lib)
    assert o.step(30) == 0
    q, _ = o.prim()
    assert np.abs(q[4] / p0 - 1.0).max() <= 1e-10, np.abs(q[4] / p0 - 1.0).max()
    assert np.abs(q[1] / u0 - 1.0).max() <= 1e-10
    assert o.stats()["flips"] > 0


TUBE = dict(left="tnt", right="water_nasg", L=(1630.0, 0.0, 2e10), R=(1000.0, 0.0, 1e5))


def check_tube_star_state(lib):
    nx, steps = 200, 60
    p = W.eos_shock_tube_1d(TUBE["left"], TUBE["right"], TUBE["L"], TUBE["R"], nx=nx, steps=steps)
    o = oracle.OracleSim(p, lib_handle=lib)
    assert o.step(steps) == 0
    t = o.stats()["t"]
    q, chi = o.prim()
    x = (np.arange(nx) + 0.5) / nx
    pr, u = q[4, 0, 0], q[1, 0, 0]
    mL, mR = RE.make_eos(*p.eos[1]), RE.make_eos(*p.eos[0])
    L, R = RE.Side(mL, *TUBE["L"]), RE.Side(mR, *TUBE["R"])
    ps, us, rl, rr = RE.star_state(L, R)
    # shock speed from mass conservation across it, rarefaction head speed
    S = (rr * us - TUBE["R"][0] * TUBE["R"][1]) / (rr - TUBE["R"][0])
    head = TUBE["L"][1] - L.c
    xc, xs, xh = 0.5 + us * t, 0.5 + S * t, 0.5 + head * t
    plateau = (x > xc + 0.25 * (xs - xc)) & (x < xs - 0.25 * (xs - xc))
    assert plateau.sum() >= 5
    assert abs(np.median(pr[plateau]) / ps - 1.0) <= 0.01, (np.median(pr[plateau]), ps)
    assert abs(np.median(u[plateau]) / us - 1.0) <= 0.01
    # shock: where p crosses the mean of p* and p_R
    i = np.flatnonzero(pr > 0.5 * (ps + TUBE["R"][2]))[-1]
    assert abs(x[i] - xs) <= 3.0 / nx, (x[i], xs)
    # rarefaction head: the first cell whose pressure fell by 1 % (the
    # scheme smears the head over about two cells ahead of it)
    j = np.flatnonzero(pr < TUBE["L"][2] * (1 - 1e-2))[0]
    assert abs(x[j] - xh) <= 3.0 / nx, (x[j], xh)


def check_solid_box_conservation(lib):
    import dataclasses
    base = W.periodic_box(2, n=(8, 7, 6), steps=8, material=1)
    prim = base.prim.copy()
    prim[0] = 8930.0 * (1.0 + 0.01 * (prim[0] - 1000.0) / 50.0)
    prim[4] = 1e9 + 5e8 * (prim[4] - 1e6) / 3e5
    p = dataclasses.replace(base, prim=prim, eos=(W._eos_of("tnt"), W._eos_of("copper")))
    o = oracle.OracleSim(p, lib_handle=lib)
    w0 = o.cons()
    assert o.step(8) == 0
    w1 = o.cons()
    for k in range(5):
        scale = np.abs(w0[k]).sum() if k in (0, 4) else np.abs(w0[0]).sum() * 100.0
        assert abs(w1[k].sum() - w0[k].sum()) <= 1e-13 * scale, k
    assert np.abs(w1[0] - w0[0]).max() > 1e-6 * 8930.0


CHECKS = {f.__name__: f for f in (check_eos_closed_forms, check_c2_isentropic, check_nasg_reduces_to_sg,
                                  check_uniform_contact, check_tube_star_state, check_solid_box_conservation)}


def _bind(lib):
    import ctypes as C
    for name in ("ora_eos_p", "ora_eos_e", "ora_eos_c2"):
        getattr(lib, name).restype = C.c_double
        getattr(lib, name).argtypes = [C.POINTER(oracle.EosC), C.c_double, C.c_double]
    lib.ora_eos_floor.restype = C.c_double
    lib.ora_eos_floor.argtypes = [C.POINTER(oracle.EosC)]
    return lib


@pytest.mark.parametrize("name", sorted(CHECKS))
def test_pin(name):
    CHECKS[name](_bind(oracle.lib()))


MUTANTS = [
    ("sound speed energy term", "return p_rho + p * p_e / (rho * rho);", "return p_rho + p * p_e / rho;",
     "check_c2_isentropic"),
    ("MG compression energy", "*eR = *pR * eta / (2.0 * r0) + e0;", "*eR = *pR * eta / r0 + e0;",
     "check_eos_closed_forms"),
    ("JWL exponent", "double x = exp(-R * r0 / rho);", "double x = exp(-R * rho / r0);", "check_eos_closed_forms"),
    ("NASG covolume", "/ (1.0 - a[2] * rho) - a[0] * a[1];", "/ (1.0 + a[2] * rho) - a[0] * a[1];",
     "check_eos_closed_forms"),
    ("general flux energy", "double EL = ora_eos_e(e, qL[0], qL[4]) + 0.5 *", "double EL = ora_eos_e(e, qL[0], qL[4]) + 0.25 *",
     "check_tube_star_state"),
    ("general sound speed in HLLC", "double cL = sqrt(ora_eos_c2(e, qL[0], qL[4]))",
     "double cL = 0.5 * sqrt(ora_eos_c2(e, qL[0], qL[4]))", "check_nasg_reduces_to_sg"),
    ("general primitive -> conservative energy", "double e = ora_eos_e(&c->eos[m], rho, q[4]);",
     "double e = ora_eos_e(&c->eos[m], rho, q[4]) * 1.0001;", "check_uniform_contact"),
    ("general conservative -> primitive pressure", "q[4] = ora_eos_p(&c->eos[m], rho, e);",
     "q[4] = ora_eos_p(&c->eos[m], rho, 1.0001 * e);", "check_uniform_contact"),
    ("interface materials swapped", "s->c.riemann(xa, xb, in, out)", "s->c.riemann(xb, xa, in, out)",
     "check_tube_star_state"),
]


@pytest.fixture(scope="module")
def mutant_dir(tmp_path_factory):
    return str(tmp_path_factory.mktemp("eos_step_mutants"))


@pytest.mark.parametrize("label,old,new,check", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistakes(label, old, new, check, mutant_dir):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "m2c_oracle.c")).read()
    assert src.count(old) == 1, label
    d = os.path.join(mutant_dir, label.replace(" ", "_"))
    os.makedirs(d, exist_ok=True)
    c_path, so = os.path.join(d, "m.c"), os.path.join(d, "m.so")
    open(c_path, "w").write(src.replace(old, new))
    inc = os.path.dirname(oracle.__file__)
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-I", inc, "-o", so,
                    c_path, "-lm"], check=True)
    lib = _bind(oracle.load(so))
    with pytest.raises(AssertionError):
        CHECKS[check](lib)
