"""The benchmark configurations at their real size and length on the GPU,
checked against the oracle at the last step (needs an MI355X).

* 128^3 shock-bubble: all 100 steps, whole grid, against the all-core oracle
  build (bit-identical to the serial one), each side with its own CFL steps.
* 384^3 bubble cloud (FP64 and mixed), the 64-run batch (FP64 and mixed)
  and the 128^3 general-EOS charge: the GPU state one step before the end is
  downloaded, blocks of it around sampled cells are stepped by the oracle
  with the GPU's dt, and the block centres are compared with the GPU's last
  step.  One step of a cell depends only on the cells within four of it
  (two Runge-Kutta stages of a two-cell stencil) plus one for the phase
  update, so half-width 6 suffices; a block cut by the domain edge has the
  domain's own transmissive boundary there.
* The general-EOS step on grids of several tiles in every direction (the
  in-plane tile halos with JWL and Mie-Grueneisen materials), whole grid.
* The mixed form's error after all 50 steps of the 384^3 cloud, per
  conserved variable and for the pressure, against the FP64 path (which
  the sampled checks tie to the oracle at every step checked).

Every case prints its name, sizes and errors.
"""
from __future__ import annotations

import copy
import os

import numpy as np
import pytest

import oracle
import workloads as W
from tests.parity import TOL_FP64, compare_runs

pytestmark = pytest.mark.gpu
R = 6
TOL_MIXED = 1e-3


@pytest.fixture(scope="module")
def m2c():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_16387_amd as m
    m.lib()
    return m


def _say(*a):
    print(*a, flush=True)


def _cons_block(p, w, k, j, i):
    """The block of half-width R around cell (k, j, i) of conserved state w
    as a problem of its own, plus the centre's index inside it."""
    nx, ny, nz = p.n
    h = p.dx()
    lo_idx = (max(i - R, 0), max(j - R, 0), max(k - R, 0))
    hi_idx = (min(i + R + 1, nx), min(j + R + 1, ny), min(k + R + 1, nz))
    wb = w[:, lo_idx[2]:hi_idx[2], lo_idx[1]:hi_idx[1], lo_idx[0]:hi_idx[0]].copy()
    b = copy.copy(p)
    b.n = tuple(hi_idx[d] - lo_idx[d] for d in range(3))
    b.lo = tuple(p.lo[d] + lo_idx[d] * h[d] for d in range(3))
    b.hi = tuple(b.lo[d] + b.n[d] * h[d] for d in range(3))
    b.prim = None
    return b, wb, (k - lo_idx[2], j - lo_idx[1], i - lo_idx[0])


def _samples(p, w, nrand, niface, seed):
    rng = np.random.default_rng(seed)
    nx, ny, nz = p.n
    near = np.argwhere(np.abs(w[5]) < 1.5 * min(p.dx()))
    out = [tuple(int(v) for v in near[q]) for q in rng.choice(len(near), min(niface, len(near)), replace=False)]
    out += [(int(rng.integers(nz)), int(rng.integers(ny)), int(rng.integers(nx))) for _ in range(nrand)]
    out += [(0, 0, 0), (nz - 1, ny - 1, nx - 1)]
    return out


def _rho_c_max(p):
    """max rho c over the initial state (the scale of the momentum floor of
    the parity metric)."""
    q = p.prim.reshape(6, -1)
    mat = (q[5] < 0).astype(int)
    if getattr(p, "eos", None) is None:
        g = np.asarray(p.gamma)[mat]
        pc = np.asarray(p.pc)[mat]
        return float(np.max(q[0] * np.sqrt(g * (q[4] + pc) / q[0])))
    from oracle import riemann_eos as RE
    mats = [RE.make_eos(f, prm) for f, prm in p.eos]
    best = 0.0
    for m in (0, 1):
        sel = np.flatnonzero(mat == m)
        if sel.size == 0:
            continue
        # the densest and the highest-pressure cells of the material bound rho c
        for i in {int(sel[np.argmax(q[0][sel])]), int(sel[np.argmax(q[4][sel])])}:
            r, pr = q[0][i], q[4][i]
            best = max(best, r * np.sqrt(max(mats[m].c2(r, mats[m].e(r, pr)), 0.0)))
    return best


def _check_last_step(p, w_prev, w_last, dt, samples, tol, label):
    """Oracle blocks of w_prev stepped once with dt against w_last, errors
    relative to each field's maximum with the floors of the parity metric
    (1 kg/m^3, 1e-3 max(rho c) for the momenta, the smallest cell width)."""
    fm = 1e-3 * _rho_c_max(p)
    scale = np.maximum(np.max(np.abs(w_last.reshape(6, -1)), axis=1), [1.0, fm, fm, fm, 1.0, min(p.dx())])
    worst = np.zeros(6)
    for (k, j, i) in samples:
        b, wb, (ck, cj, ci) = _cons_block(p, w_prev, k, j, i)
        o = oracle.OracleSim(b)
        assert o.set_cons(wb) == 0
        assert o.step_dt(1, dt) == 0, (label, (k, j, i))
        worst = np.maximum(worst, np.abs(w_last[:, k, j, i] - o.cons()[:, ck, cj, ci]) / scale)
    _say(label, "samples", len(samples), "max rel err per field (rho, rho u, rho v, rho w, rho E, phi)", worst)
    assert np.all(worst <= tol), (label, worst)
    return worst


def test_shock_bubble_128_all_100_steps_vs_openmp_oracle(m2c):
    p = W.shock_bubble(0, n=128)
    _say("shock_bubble 128^3, 100 steps, seed 0")
    g = m2c.Sim(m2c.config_for(p), p.prim)
    assert g.step(100) == 0
    oracle.build(force=False, openmp=True)
    o = oracle.OracleSim(p, lib_handle=oracle.lib_openmp())
    assert o.step(100) == 0
    e = compare_runs(g, o, p)
    st_g, st_o = g.stats(), o.stats()
    _say({k: (f"{v:.2e}" if isinstance(v, float) else v) for k, v in e.items()},
         "t gpu", st_g["t"], "t oracle", st_o["t"], "solves", st_g["riemann_solves"], st_o["riemann_solves"])
    assert e["id_mismatch"] == 0
    assert abs(st_g["t"] - st_o["t"]) <= 1e-12 * st_o["t"]
    assert st_g["riemann_solves"] == st_o["riemann_solves"]
    for k in ("rho", "rhou", "rhov", "rhow", "rhoE", "phi"):
        assert e[k] <= TOL_FP64, (k, e[k])


@pytest.fixture(scope="module")
def cloud():
    return W.bubble_cloud(0)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_bubble_cloud_384_last_step_sampled(m2c, cloud, prec):
    p = cloud
    _say("bubble_cloud 384^3, steps 1..50, precision", prec)
    g = m2c.Sim(m2c.config_for(p, precision=prec), p.prim)
    assert g.step(p.steps - 1) == 0
    w_prev = g.get_conserved()
    assert g.step(1) == 0
    dt = g.stats()["dt_last"]
    w_last = g.get_conserved()
    _check_last_step(p, w_prev, w_last, dt, _samples(p, w_prev, 8, 14, seed=50 + prec),
                     TOL_FP64 if prec == 0 else TOL_MIXED, f"cloud prec {prec} step {p.steps}")


def test_bubble_cloud_384_mixed_error_after_50_steps(m2c, cloud):
    """Error of the mixed form after the whole workload, per conserved
    variable (relative to the variable's maximum, with the parity floors)
    and for the pressure (relative to max |p| over the cells, and to p + p_c
    cell by cell), against the FP64 path."""
    p = cloud
    out = {}
    for prec in (0, 1):
        g = m2c.Sim(m2c.config_for(p, precision=prec), p.prim)
        assert g.step(p.steps) == 0
        out[prec] = (g.get_conserved(), *g.get_state())
        g.close()
    (w64, q64, x64), (wmx, qmx, xmx) = out[0], out[1]
    from tests.parity import conserved_errors
    e = conserved_errors(wmx, w64, q64, p.gamma, p.pc, x64, min(p.dx()))
    pc = np.where(x64 == 1, p.pc[1], p.pc[0])
    dp = np.abs(qmx[4] - q64[4])
    e["p_rel_max"] = float(dp.max() / np.abs(q64[4]).max())
    e["p_rel_cellwise_pbar"] = float((dp / (q64[4] + pc)).max())
    e["id_mismatch"] = int(np.count_nonzero(xmx != x64))
    _say("mixed vs FP64 after 50 steps of the 384^3 cloud:", {k: (f"{v:.2e}" if isinstance(v, float) else v)
                                                               for k, v in e.items()})
    assert e["id_mismatch"] == 0
    for k in ("rho", "rhou", "rhov", "rhow", "rhoE", "phi", "p_rel_max"):
        assert e[k] <= TOL_MIXED, (k, e[k])


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_batch_64_runs_last_step_sampled(m2c, prec):
    probs = W.batched_shock_bubbles(0)
    steps = probs[0].steps
    _say("batch of", len(probs), "runs,", sum(q.ncells for q in probs), "cells, steps 1 ..", steps, "precision", prec)
    b = m2c.Batch([m2c.config_for(q, precision=prec) for q in probs], [q.prim for q in probs])
    assert b.step(steps - 1) == 0
    w_prev = [b.get_conserved(k) for k in range(len(probs))]
    assert b.step(1) == 0
    worst = np.zeros(6)
    for k, q in enumerate(probs):
        st = b.stats(k)
        assert st["steps"] == steps, (k, st)
        w_last = b.get_conserved(k)
        worst = np.maximum(worst, _check_last_step(q, w_prev[k], w_last, st["dt_last"],
                                                   _samples(q, w_prev[k], 2, 3, seed=100 + k),
                                                   TOL_FP64 if prec == 0 else TOL_MIXED, f"run {k} {q.n}"))
    _say("batch worst over runs", worst)
    b.close()


def test_eos_charge_128_last_step_sampled(m2c):
    """The 128^3 sphere of detonation products (JWL, 5 GPa) in NASG water,
    as the benchmark runs it: steps 1..20, the last one checked."""
    p = W.eos_charge(0, n=(128, 128, 128), steps=20)
    _say("eos_charge 128^3, steps 1..20")
    g = m2c.Sim(m2c.config_for(p), p.prim)
    assert g.step(p.steps - 1) == 0
    w_prev = g.get_conserved()
    assert g.step(1) == 0
    dt = g.stats()["dt_last"]
    _check_last_step(p, w_prev, g.get_conserved(), dt, _samples(p, w_prev, 2, 5, seed=7), TOL_FP64,
                     "eos charge step 20")


@pytest.mark.parametrize("case", ["tnt_in_water_nasg", "copper_in_tnt"])
def test_eos_charge_multi_tile(m2c, case):
    """General-EOS step on 40 x 36 x 9 cells: three 16 x 16 tiles per
    in-plane axis with ragged edges and two z-blocks of the 8-plane march,
    so that every tile halo (x, y and the z window) carries JWL / NASG /
    Mie-Grueneisen states.  One step: the oracle's interface solves (adaptive
    isentropes in Python) dominate the test time."""
    if case == "tnt_in_water_nasg":
        p = W.eos_charge(11, n=(40, 36, 9), steps=1)
    else:
        p = W.eos_charge(12, n=(40, 36, 9), steps=1, inner="copper", outer="tnt", p_inner=1e5,
                         rho_inner=8930.0, rho_outer=1630.0, p_outer=1e9)
    _say(case, p.n, "steps", p.steps)
    o = oracle.OracleSim(p)
    g = m2c.Sim(m2c.config_for(p), p.prim)
    assert g.tile()[:2] == (16, 15)
    assert o.step(p.steps) == 0
    assert g.step(p.steps) == 0
    e = compare_runs(g, o, p)
    _say({k: (f"{v:.2e}" if isinstance(v, float) else v) for k, v in e.items()}, "interface faces",
         o.stats()["iface_faces_last"])
    assert o.stats()["iface_faces_last"] > 100
    assert e["id_mismatch"] == 0
    for k in ("rho", "rhou", "rhov", "rhow", "rhoE", "phi"):
        assert e[k] <= TOL_FP64, (k, e[k])
