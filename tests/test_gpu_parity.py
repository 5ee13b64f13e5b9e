"""GPU path vs the CPU oracle, through the C ABI (needs an MI355X).

Every case prints its name before it runs.  Inputs come from the seeded
``workloads`` generators; expected values come only from ``oracle``.
"""
from __future__ import annotations

import math

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


def _pair(m2c, problem, precision=0, **kw):
    oracle.build(force=False)
    o = oracle.OracleSim(problem)
    g = m2c.Sim(m2c.config_for(problem, precision=precision, **kw), problem.prim)
    return g, o


def _assert_close(e, tol=TOL_FP64):
    print({k: (f"{v:.2e}" if isinstance(v, float) else v) for k, v in e.items()}, flush=True)
    assert e["id_mismatch"] == 0
    for k in ("rho", "rhou", "rhov", "rhow", "rhoE", "phi"):
        assert e[k] <= tol, (k, e[k])


# ---- point kernels ---------------------------------------------------------

def _random_faces(rng, n, mat):
    g, pc = (W.WATER if mat == 1 else W.AIR)
    rho = (1000.0 if mat == 1 else 1.0) * np.exp(rng.uniform(-0.3, 0.3, n))
    c = np.sqrt(g * (1e5 + pc) / rho)
    q = np.empty((5, n))
    q[0] = rho
    q[1] = rng.uniform(-2, 2, n) * c
    q[2] = rng.uniform(-1, 1, n) * c
    q[3] = rng.uniform(-1, 1, n) * c
    q[4] = np.exp(rng.uniform(math.log(1e4), math.log(1e8), n))
    return q, g, pc


@pytest.mark.parametrize("mat", [0, 1])
def test_hllc_points(m2c, mat):
    import torch
    rng = np.random.default_rng(100 + mat)
    n = 3000
    qL, g, pc = _random_faces(rng, n, mat)
    qR, _, _ = _random_faces(rng, n, mat)
    F = m2c.eval_hllc(torch.tensor(qL, device="cuda"), torch.tensor(qR, device="cuda"), g, pc).cpu().numpy()
    ref = np.stack([oracle.hllc(qL[:, i].copy(), qR[:, i].copy(), g, pc) for i in range(n)], axis=1)
    scale = np.max(np.abs(ref), axis=1, keepdims=True)
    err = np.max(np.abs(F - ref) / scale)
    print("hllc max rel err", err)
    assert err < 1e-12


def test_riemann_points(m2c):
    import torch
    inp, eos = W.riemann_problem_set(7, 4000)
    out, iters, rc = m2c.riemann_solve(torch.tensor(inp.T.copy(), device="cuda"),
                                       torch.tensor(eos.T.copy(), device="cuda"))
    out = out.cpu().numpy()
    iters = iters.cpu().numpy()
    nbad = 0
    for i in range(inp.shape[0]):
        rcs, ref, _ = oracle.riemann(inp[i], eos[i])
        if rcs != oracle.OK:
            assert iters[i] == 0
            nbad += 1
            continue
        assert iters[i] != 0
        plo = -min(eos[i, 1], eos[i, 3])
        assert abs(out[0, i] - ref[0]) <= 1e-10 * (ref[0] - plo)
        us = max(abs(inp[i, 1]), abs(inp[i, 4]), math.sqrt(eos[i, 0] * (inp[i, 2] + eos[i, 1]) / inp[i, 0]))
        assert abs(out[1, i] - ref[1]) <= 1e-9 * us
        assert abs(out[2, i] - ref[2]) <= 1e-10 * ref[2]
        assert abs(out[3, i] - ref[3]) <= 1e-10 * ref[3]
    assert (rc == m2c.M2C_ERR_RIEMANN) == (nbad > 0)


# ---- interface work queue (bit-exact) ---------------------------------------

def test_queue_shock_bubble(m2c):
    p = W.shock_bubble(1, n=40)
    g, o = _pair(m2c, p)
    q = g.interface_faces()
    ref = o.interface_faces()
    assert q.size > 0
    assert np.array_equal(q, ref)


# (9,7,5): byte path of the compaction; (8,6,5), (4,3,3), (12,1,7): 32-bit
# word path (nx a multiple of 4), with the periodic wrap of the last word of
# a row, a 4-cell row and an inactive axis
@pytest.mark.parametrize("dims", [(9, 7, 5), (8, 6, 5), (4, 3, 3), (12, 1, 7)])
def test_queue_checkerboard_periodic(m2c, dims):
    p = W.periodic_box(3, n=dims)
    nx, ny, nz = p.n
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    p.prim[5] = np.where((i + j + k) % 2 == 0, 1.0, -1.0)
    p.prim[4] = np.where(p.prim[5] < 0, 1e6, 1e5)
    p.prim[0] = np.where(p.prim[5] < 0, 1000.0, 1.0)
    g, o = _pair(m2c, p)
    assert np.array_equal(g.interface_faces(), o.interface_faces())


@pytest.mark.parametrize("dims", [(20, 12, 10), (21, 12, 10), (64, 3, 2)])
def test_queue_random_materials(m2c, dims):
    """Random material ids (transmissive boundaries): every face class."""
    p = W.shock_bubble(5, nxyz=dims, radius=0.3)
    rng = np.random.default_rng(sum(dims))
    phi = np.where(rng.random(p.prim[5].shape) < 0.35, -1.0, 1.0)
    p.prim[5] = phi
    p.prim[0] = np.where(phi < 0, 1.0, 1000.0)
    p.prim[1:4] = 0.0
    p.prim[4] = 1e5
    g, o = _pair(m2c, p)
    q = g.interface_faces()
    assert q.size > 0
    assert np.array_equal(q, o.interface_faces())


def test_queue_empty(m2c):
    p = W.periodic_box(4, n=(8, 8, 8))
    g, o = _pair(m2c, p)
    assert g.interface_faces().size == 0 == o.interface_faces().size


# ---- whole steps -------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_shock_tube_full(m2c, seed):
    """1000x1x1 water/air shock tube, 200 steps (full size)."""
    p = W.shock_tube_1d(seed)
    g, o = _pair(m2c, p)
    assert g.step(p.steps) == 0
    assert o.step(p.steps) == 0
    _assert_close(compare_runs(g, o, p))
    sg, so = g.stats(), o.stats()
    assert sg["steps"] == so["steps"] == p.steps
    assert abs(sg["t"] - so["t"]) <= 1e-12 * so["t"]
    assert sg["riemann_solves"] == so["riemann_solves"]
    assert sg["flips"] == so["flips"]


@pytest.mark.parametrize("bc", [W.BC_PERIODIC, W.BC_WALL, W.BC_TRANSMISSIVE])
def test_single_material_box(m2c, bc):
    p = W.periodic_box(5, n=(37, 21, 11), bc=bc)
    g, o = _pair(m2c, p)
    assert g.step(15) == 0 and o.step(15) == 0
    _assert_close(compare_runs(g, o, p))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_uniform_translation(m2c, axis):
    p = W.uniform_translation(n=150, axis=axis, steps=60)
    g, o = _pair(m2c, p)
    assert g.step(p.steps) == 0 and o.step(p.steps) == 0
    _assert_close(compare_runs(g, o, p))
    prim, _ = g.get_state()
    u = prim[1 + axis]
    assert np.max(np.abs(u - 50.0)) < 1e-9 * 50.0
    assert np.max(np.abs(prim[4] - 1e5)) < 1e-9 * 1e5


@pytest.mark.parametrize("tile", [None, (32, 8, 8), (16, 15, 3), (16, 16, 5), (32, 8, 16), (64, 2, 1)])
def test_shock_bubble_small(m2c, tile):
    """3D shock-bubble on a 45x38x33 grid (ragged in every tile shape)."""
    p = W.shock_bubble(2, nxyz=(45, 38, 33), radius=0.2, p_shock=1e9, shock_x=0.25)
    g, o = _pair(m2c, p, tile=tile)
    assert g.step(12) == 0 and o.step(12) == 0
    e = compare_runs(g, o, p)
    _assert_close(e)
    assert g.stats()["riemann_solves"] == o.stats()["riemann_solves"]


# forward Euler and TVD-RK3 (section "Time integration"): the stage kernels
# of the first, middle and last kinds with their blend weights
@pytest.mark.parametrize("order,steps,cfl", [(1, 8, 0.15), (3, 25, 0.4)])
@pytest.mark.parametrize("prec", [0, 1])
def test_rk_orders(m2c, order, steps, cfl, prec):
    p = W.shock_bubble(7, nxyz=(24, 20, 18), radius=0.22, p_shock=1e9, shock_x=0.25, cfl=cfl)
    o = oracle.OracleSim(p, rk_order=order)
    g = m2c.Sim(m2c.config_for(p, precision=prec, rk_order=order), p.prim)
    assert g.step(steps) == 0 and o.step(steps) == 0
    e = compare_runs(g, o, p)
    print("rk", order, prec, e)
    assert e["id_mismatch"] == 0
    tol = TOL_FP64 if prec == 0 else 1e-3
    for k in ("rho", "rhou", "rhov", "rhow", "rhoE", "phi"):
        assert e[k] <= tol, (k, e[k])
    st = g.stats()
    assert st["steps"] == steps and st["riemann_solves"] == o.stats()["riemann_solves"]


# limiters and numerical fluxes other than MC + HLLC: the option kernels
# (run-time choice), with the same choice in the FIVER one-sided fluxes; a
# zero MC parameter gives constant reconstruction in the default kernels
@pytest.mark.parametrize("lim,k,flux,alpha,order,tile", [
    (oracle.LIM_VA, 2, oracle.FLUX_HLLC, 1.2, 2, None),
    (oracle.LIM_VA_MOD, 4, oracle.FLUX_HLLC, 1.2, 2, (32, 7, 4)),
    (oracle.LIM_MC, 2, oracle.FLUX_LLF, 1.2, 2, None),
    (oracle.LIM_VA, 6, oracle.FLUX_LLF, 1.2, 3, (16, 15, 3)),
    (oracle.LIM_MC, 2, oracle.FLUX_HLLC, 0.0, 2, None),
])
@pytest.mark.parametrize("prec", [0, 1])
def test_limiter_and_flux_options(m2c, lim, k, flux, alpha, order, tile, prec):
    p = W.shock_bubble(8, nxyz=(26, 21, 17), radius=0.22, p_shock=1e9, shock_x=0.3)
    o = oracle.OracleSim(p, limiter=lim, limiter_k=k, flux=flux, alpha=alpha, rk_order=order)
    g = m2c.Sim(m2c.config_for(p, precision=prec, limiter=lim, limiter_k=k, flux=flux, alpha=alpha,
                               rk_order=order, tile=tile), p.prim)
    assert g.step(20) == 0 and o.step(20) == 0
    e = compare_runs(g, o, p)
    print("opts", lim, k, flux, alpha, order, prec, e)
    assert e["id_mismatch"] == 0
    tol = TOL_FP64 if prec == 0 else 1e-3
    for name in ("rho", "rhou", "rhov", "rhow", "rhoE", "phi"):
        assert e[name] <= tol, (name, e[name])
    assert g.stats()["riemann_solves"] == o.stats()["riemann_solves"]


@pytest.mark.parametrize("prec", [0, 1])
def test_narrow_band_level_set(m2c, prec):
    """Level set advanced only where |phi| < band (section "Level set
    method"): parity with the oracle, phi held outside the band."""
    p = W.shock_bubble(5, nxyz=(27, 22, 19), radius=0.25, p_shock=1e9, shock_x=0.3)
    band = 3.0 * min(p.dx())
    o = oracle.OracleSim(p, ls_band=band)
    g = m2c.Sim(m2c.config_for(p, precision=prec, ls_band=band), p.prim)
    assert g.step(20) == 0 and o.step(20) == 0
    e = compare_runs(g, o, p)
    print("band", prec, e)
    assert e["id_mismatch"] == 0
    tol = TOL_FP64 if prec == 0 else 1e-3
    for name in ("rho", "rhou", "rhov", "rhow", "rhoE", "phi"):
        assert e[name] <= tol, (name, e[name])
    out = np.abs(p.prim[5]) >= band
    assert np.array_equal(g.get_conserved()[5][out], p.prim[5][out])


@pytest.mark.parametrize("prec", [0, 1])
def test_bubble_next_to_rigid_wall(m2c, prec):
    """The paper's shock-induced collapse of a bubble near a rigid wall:
    walls on every side, bubble 0.04 from the +x wall, a 1 GPa shock; FIVER
    faces meet wall images.  FP64 at the oracle bar, mixed at its bound."""
    p = W.shock_bubble(6, nxyz=(40, 24, 22), radius=0.2, p_shock=1e9, shock_x=0.52, centre_x=0.76,
                       bc=(W.BC_WALL,) * 6)
    g, o = _pair(m2c, p, precision=prec)
    assert g.step(80) == 0 and o.step(80) == 0
    assert o.stats()["flips"] > 0                    # the shock has reached the bubble
    e = compare_runs(g, o, p)
    print("wall", prec, e)
    assert e["id_mismatch"] == 0
    tol = TOL_FP64 if prec == 0 else 1e-3
    for k in ("rho", "rhou", "rhov", "rhow", "rhoE", "phi"):
        assert e[k] <= tol, (k, e[k])


def test_shock_bubble_interaction_flips(m2c):
    """Shock reaches the bubble: cells change material (phase update)."""
    p = W.shock_bubble(0, n=32, radius=0.3, p_shock=1e9, shock_x=0.2)
    g, o = _pair(m2c, p)
    assert g.step(40) == 0 and o.step(40) == 0
    e = compare_runs(g, o, p)
    _assert_close(e)
    sg, so = g.stats(), o.stats()
    print(sg, so)
    assert sg["flips"] == so["flips"]
    assert sg["orphans"] == so["orphans"]


def test_shock_bubble_128_one_step(m2c):
    """Full 128^3 shock-bubble grid, two steps in the benchmark's launch shape."""
    p = W.shock_bubble(0, n=128)
    g, o = _pair(m2c, p)
    assert g.step(2) == 0 and o.step(2) == 0
    _assert_close(compare_runs(g, o, p))


def test_profiling_samples_steps(m2c):
    """m2c_set_profiling(every): kernel classes timed on one step in `every`."""
    p = W.shock_bubble(2, nxyz=(24, 20, 18))
    s = m2c.Sim(m2c.config_for(p), p.prim)
    s.set_profiling(3)
    s.step(10)                                   # steps 0, 3, 6, 9 are timed
    st = s.stats()
    assert st["stage_launches"] == 8 and st["fiver_launches"] == 8
    assert st["ms_stage"] > 0.0 and st["ms_fiver"] > 0.0
    s.set_profiling(0)
    s.reset_stats()
    s.step(2)
    assert s.stats()["stage_launches"] == 0


def test_determinism(m2c):
    p = W.shock_bubble(1, n=40, radius=0.25, p_shock=1e9, shock_x=0.2)
    a = m2c.Sim(m2c.config_for(p), p.prim)
    b = m2c.Sim(m2c.config_for(p), p.prim)
    a.step(25)
    b.step(25)
    assert np.array_equal(a.get_conserved(), b.get_conserved())


def test_checkpoint_roundtrip(m2c):
    p = W.shock_bubble(1, n=24, radius=0.25, p_shock=1e9, shock_x=0.2)
    a = m2c.Sim(m2c.config_for(p), p.prim)
    a.step(10)
    w = a.get_conserved()
    a.step(10)
    b = m2c.Sim(m2c.config_for(p))
    b.set_conserved(w)
    b.step(10)
    assert np.array_equal(a.get_conserved(), b.get_conserved())


def test_set_state_rejects_nonphysical(m2c):
    p = W.periodic_box(6, n=(8, 8, 8))
    prim = p.prim.copy()
    prim[0, 3, 2, 1] = -1.0
    g = m2c.Sim(m2c.config_for(p))
    rc = g.set_state(prim, check=False)
    assert rc == m2c.M2C_ERR_NONPHYSICAL
    assert g.step(1, check=False) == m2c.M2C_ERR_STATE
    prim[0, 3, 2, 1] = 1.0
    assert g.set_state(prim) == 0


def test_blowup_is_transactional(m2c):
    """CFL far above the stability limit: the step that fails is rolled back."""
    p = W.shock_tube_1d(3, nx=200)
    p.cfl = 5.0
    g = m2c.Sim(m2c.config_for(p), p.prim)
    rc = None
    for _ in range(200):
        w_before = g.get_conserved()
        rc = g.step(1, check=False)
        if rc != 0:
            break
    assert rc in (m2c.M2C_ERR_NONPHYSICAL, m2c.M2C_ERR_RIEMANN)
    assert np.array_equal(g.get_conserved(), w_before)
    assert g.stats()["err_code"] == rc


def test_mixed_precision_error_stated(m2c):
    """Mixed form (FP32 bulk reconstruction and HLLC): error vs the FP64 oracle."""
    p = W.shock_bubble(2, nxyz=(40, 36, 30), radius=0.2, p_shock=1e8, shock_x=0.2)
    g, o = _pair(m2c, p, precision=1)
    assert g.step(20) == 0 and o.step(20) == 0
    e = compare_runs(g, o, p)
    print("mixed", e)
    assert e["id_mismatch"] == 0
    for k in ("rho", "rhou", "rhov", "rhow", "rhoE", "phi"):
        assert e[k] < 1e-3, (k, e[k])


def test_interface_queue_rebuilt_after_state_replacement(m2c):
    """The interface queue is kept across steps that flip no cell; a state
    replaced between steps (set_state, set_conserved) must rebuild it.  A run
    continued on a different bubble has to match the oracle started on that
    bubble."""
    a = W.shock_bubble(1, nxyz=(24, 22, 20), radius=0.2, p_shock=1e8, shock_x=0.1)
    b = W.shock_bubble(2, nxyz=(24, 22, 20), radius=0.3, p_shock=1e8, shock_x=0.1, centre_x=0.4)
    print("queue rebuild: bubble A then bubble B", flush=True)
    g = m2c.Sim(m2c.config_for(a), a.prim)
    assert g.step(4) == 0
    g.set_state(b.prim)
    assert g.step(4) == 0
    o = oracle.OracleSim(b)
    assert o.step(4) == 0
    _assert_close(compare_runs(g, o, b))
    # the same through the conservative checkpoint entry point
    g2 = m2c.Sim(m2c.config_for(a), a.prim)
    assert g2.step(4) == 0
    o2 = oracle.OracleSim(b)
    g2.set_conserved(o2.cons())
    assert g2.step(4) == 0 and o2.step(4) == 0
    _assert_close(compare_runs(g2, o2, b))
