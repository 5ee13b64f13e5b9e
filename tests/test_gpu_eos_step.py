"""The time step with a general EOS per material on the GPU against the
oracle (``oracle/m2c_oracle.c`` with ``eos_general``; interface star states
from ``oracle/riemann_eos.py``), through the C ABI.

Bar: the FP64 bar of the stiffened-gas runs (e_k <= 1e-9, no material-id
mismatch).  The library integrates Mie-Grueneisen isentropes by RK4 at
ds = 0.01 (error about 1e-10 of the star state, measured against the same
oracle); NASG and JWL wave curves are closed forms on both sides up to the
oracle's quadrature tolerance, so the interface fluxes agree to about 1e-10
and the states, to which they contribute through dt/h, closer still.

Every case prints its name before it runs.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

import oracle
import workloads as W
from tests.parity import TOL_FP64, compare_runs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m2c():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_16387_amd as m
    m.lib()
    return m


def _run(m2c, problem, steps, **kw):
    print(problem.name, problem.meta, problem.n, "steps", steps, kw, flush=True)
    oracle.build(force=False)
    o = oracle.OracleSim(problem, **{k: v for k, v in kw.items() if k in ("rk_order", "limiter", "limiter_k",
                                                                           "flux", "ls_band")})
    g = m2c.Sim(m2c.config_for(problem, **kw), problem.prim)
    assert o.step(steps) == 0
    assert g.step(steps) == 0
    e = compare_runs(g, o, problem)
    print({k: (f"{v:.2e}" if isinstance(v, float) else v) for k, v in e.items()}, o.stats()["flips"], flush=True)
    assert e["id_mismatch"] == 0
    for k in ("rho", "rhou", "rhov", "rhow", "rhoE", "phi"):
        assert e[k] <= TOL_FP64, (k, e[k])
    return g, o


TUBES = {
    # detonation products against water: strong shock into NASG water
    "tnt-water": ("tnt", "water_nasg", (1630.0, 0.0, 2e10), (1000.0, 0.0, 1e5)),
    # copper plate striking detonation products at rest
    "copper-tnt": ("copper", "tnt", (8930.0, 600.0, 1e5), (1630.0, 0.0, 1e9)),
    # glass against water, separating: rarefactions on the Mie-Grueneisen side
    "glass-water": ("glass", "water_nasg", (2220.0, -150.0, 2e9), (1000.0, 150.0, 1e8)),
    # NASG gas (covolume, e_c) against NASG water
    "gas-water": ("gas_nasg", "water_nasg", (5.0, 0.0, 5e6), (1000.0, 0.0, 1e5)),
    # detonation products expanding into air seven decades less dense
    "tnt-air-1e7": ("tnt", "air", (1630.0, 0.0, 2e10), (1.63e-4, 0.0, 10.0)),
}


@pytest.mark.parametrize("name", sorted(TUBES))
def test_eos_shock_tube_matches_oracle(m2c, name):
    left, right, L, R = TUBES[name]
    p = W.eos_shock_tube_1d(left, right, L, R, nx=160, steps=40)
    g, o = _run(m2c, p, 40)
    assert o.stats()["riemann_solves"] > 0
    # each material's density against its own scale (the light side spans
    # seven decades below the heavy one in the density-jump case)
    wg, wo = g.get_conserved()[0].reshape(-1), o.cons()[0].reshape(-1)
    _, chi = o.prim()
    for m in (0, 1):
        sel = chi.reshape(-1) == m
        err = np.abs(wg[sel] - wo[sel]).max() / np.abs(wo[sel]).max()
        print("material", m, "density error", err, flush=True)
        assert err <= TOL_FP64


def test_eos_options_match_oracle(m2c):
    """RK3, Van Albada (k = 4) and local Lax-Friedrichs with general EOS."""
    left, right, L, R = TUBES["tnt-water"]
    p = W.eos_shock_tube_1d(left, right, L, R, nx=120, steps=25)
    _run(m2c, p, 25, rk_order=3, limiter=oracle.LIM_VA, limiter_k=4, flux=oracle.FLUX_LLF)


def test_eos_charge_3d_matches_oracle(m2c):
    """A sphere of detonation products in NASG water on a 3D grid (interface
    faces along all three axes, cells flipping as the sphere grows)."""
    p = W.eos_charge(4, n=(11, 10, 9), steps=4)
    g, o = _run(m2c, p, 4)
    assert o.stats()["iface_faces_last"] > 50


@pytest.mark.parametrize("inner,outer,p_in,rho_in,rho_out,p_out", [
    ("copper", "tnt", 1e5, 8930.0, 1630.0, 5e9),      # copper ball struck by detonation products
    ("air", "glass", 1e5, 1.2, 2204.0, 1e9),          # air pore in compressed glass
], ids=["copper-in-tnt", "air-in-glass"])
def test_eos_mie_grueneisen_3d_matches_oracle(m2c, inner, outer, p_in, rho_in, rho_out, p_out):
    """3D runs with a Mie-Grueneisen material on one side of the interface
    (RK4 isentropes in the library, adaptive ones in the oracle)."""
    p = W.eos_charge(6, n=(10, 9, 8), steps=3, inner=inner, outer=outer, p_inner=p_in, rho_inner=rho_in,
                     rho_outer=rho_out, p_outer=p_out)
    g, o = _run(m2c, p, 3)
    assert o.stats()["iface_faces_last"] > 50


# one 3D case per ordered pair of families (material 0 = outer, material 1 =
# the sphere): the interface kernels are compiled per family pair and the
# stage kernels per family set, so each of them runs at least once here
FAMILY_PAIRS = {
    # (outer, inner, p_inner, rho_inner, rho_outer, p_outer)
    "nasg-nasg": ("water_nasg", "gas_nasg", 5e6, 5.0, 1000.0, 1e5),
    "nasg-mg": ("water_nasg", "glass", 1e5, 2220.0, 1000.0, 1e9),
    "nasg-jwl": ("water_nasg", "tnt", 5e9, 1630.0, 1000.0, 1e5),
    "mg-nasg": ("glass", "air", 1e5, 1.2, 2204.0, 1e9),
    "mg-mg": ("copper", "tantalum", 5e9, 16650.0, 8930.0, 1e5),
    "mg-jwl": ("copper", "tnt", 5e9, 1630.0, 8930.0, 1e5),
    "jwl-nasg": ("tnt", "water_nasg", 1e5, 1000.0, 1630.0, 1e9),
    "jwl-mg": ("tnt", "copper", 1e5, 8930.0, 1630.0, 5e9),
    "jwl-jwl": ("tnt", "tnt", 5e9, 1630.0, 1630.0, 1e9),
}


@pytest.mark.parametrize("name", sorted(FAMILY_PAIRS))
def test_eos_every_family_pair_3d_matches_oracle(m2c, name):
    outer, inner, p_in, rho_in, rho_out, p_out = FAMILY_PAIRS[name]
    p = W.eos_charge(9, n=(10, 9, 8), steps=3, inner=inner, outer=outer, p_inner=p_in, rho_inner=rho_in,
                     rho_outer=rho_out, p_outer=p_out)
    g, o = _run(m2c, p, 3)
    assert g.tile()[:2] == (16, 15)
    assert o.stats()["iface_faces_last"] > 50


def test_eos_3d_walls_band_and_options_match_oracle(m2c):
    """The run-time option kernels with a general EOS in 3D: wall boundaries,
    a narrow-band level set, RK3, modified Van Albada and LLF."""
    p = W.eos_charge(8, n=(10, 9, 8), steps=3)
    p = dataclasses.replace(p, bc=(1, 1, 1, 1, 1, 1))
    g, o = _run(m2c, p, 3, rk_order=3, limiter=oracle.LIM_VA_MOD, limiter_k=2, flux=oracle.FLUX_LLF,
                ls_band=0.15)
    assert o.stats()["iface_faces_last"] > 50


def test_eos_autotune_restores_state(m2c):
    """The tile autotuner on a general-EOS context tries only the compiled
    general-EOS tiles and restores the state (and marks the interface queue
    stale): the run that follows matches the oracle."""
    p = W.eos_charge(4, n=(11, 10, 9), steps=4)
    print("autotune on the general-EOS charge", flush=True)
    g = m2c.Sim(m2c.config_for(p), p.prim)
    tile, ms = g.autotune(2)
    print("tile", tile, "ms", ms, flush=True)
    assert tile[:2] == (16, 15)
    o = oracle.OracleSim(p)
    assert g.step(4) == 0 and o.step(4) == 0
    e = compare_runs(g, o, p)
    print(e, flush=True)
    assert e["id_mismatch"] == 0
    for k in ("rho", "rhou", "rhov", "rhow", "rhoE", "phi"):
        assert e[k] <= TOL_FP64, (k, e[k])


def test_nasg_as_stiffened_gas_matches_stiffened_gas_path(m2c):
    """NASG with b = e_c = 0 is the stiffened gas: the general-EOS kernels
    reproduce the stiffened-gas kernels on a shock-bubble run (no oracle)."""
    p = W.shock_bubble(5, n=24, steps=20, radius=0.2, p_shock=1e9, shock_x=0.3)
    eos = tuple((0, [p.gamma[m], p.pc[m], 0.0, 0.0, 0.0, 0.0, 0.0]) for m in range(2))
    q = dataclasses.replace(p, eos=eos)
    print("shock bubble 24^3 as NASG", flush=True)
    a = m2c.Sim(m2c.config_for(p), p.prim)
    b = m2c.Sim(m2c.config_for(q), p.prim)
    assert a.step(20) == 0 and b.step(20) == 0
    wa, wb = a.get_conserved(), b.get_conserved()
    for k in range(6):
        scale = np.abs(wa[k]).max() + (np.abs(wa[0]).max() * 100.0 if k in (1, 2, 3) else 0.0)
        err = np.abs(wa[k] - wb[k]).max() / scale
        print(k, err, flush=True)
        assert err <= 1e-10, (k, err)
    assert np.array_equal(a.get_state()[1], b.get_state()[1])


def test_eos_rejects_unsupported_forms(m2c):
    left, right, L, R = TUBES["tnt-water"]
    p = W.eos_shock_tube_1d(left, right, L, R, nx=64, steps=5)
    cfg = m2c.config_for(p, precision=m2c.M2C_PREC_MIXED)
    with pytest.raises(m2c.M2CError):
        m2c.Sim(cfg)
    cfg = m2c.config_for(p)
    cfg.eos[0].prm[0] = 0.5                      # NASG gamma <= 1
    with pytest.raises(m2c.M2CError):
        m2c.Sim(cfg)
