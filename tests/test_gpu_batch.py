"""Batched form (persistent stage kernel over many runs, hipGraph replay)
and the tile autotuner, through the C ABI (needs an MI355X)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads as W
from tests.parity import TOL_FP64, compare_runs, conserved_errors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m2c():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_16387_amd as m
    m.lib()
    return m


def _runs():
    """Uneven shock-bubble grids (ragged in every tile shape) and a 1D tube."""
    out = []
    for k, dims in enumerate([(24, 20, 18), (33, 17, 12), (16, 16, 16), (40, 12, 9)]):
        out.append(W.shock_bubble(10 + k, nxyz=dims, radius=0.22, p_shock=1e9, shock_x=0.25))
    out.append(W.shock_tube_1d(4, nx=300))
    return out


# Batched vs single-grid contexts.  The mixed forms run the same stage code
# and agree bit for bit.  In FP64 the single-grid kernel reads the material
# parameters from an LDS table while the batched kernel (tighter register
# budget) selects them from scalars; the two compile to different
# instruction sequences whose results differ in the last bits of a few
# cells (measured: first difference one ulp of rho E in one cell after six
# steps), so FP64 is held to 1e-12 on the parity metric, 1000 times below
# the oracle bar, with identical material ids and counters.
TOL_BATCH_FP64 = 1e-12


def assert_batch_matches(b, k, sim, problem):
    """FP64 run k of batch b against the single-grid context sim."""
    wb, ws = b.get_conserved(k), sim.get_conserved()
    prim, chi = sim.get_state()
    e = conserved_errors(wb, ws, prim, problem.gamma, problem.pc, chi, min(problem.dx()))
    assert max(e.values()) <= TOL_BATCH_FP64, (k, e)
    assert np.array_equal(b.get_state(k)[1], chi), k


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("tile", [(16, 16, 8), (32, 8, 4), (16, 15, 3)])
def test_batch_equals_standalone(m2c, prec, tile):
    probs = _runs()
    cfgs = [m2c.config_for(p, precision=prec, tile=tile) for p in probs]
    b = m2c.Batch(cfgs, [p.prim for p in probs])
    assert b.tile() == tile
    b.step(12)
    for k, p in enumerate(probs):
        s = m2c.Sim(m2c.config_for(p, precision=prec, tile=tile), p.prim)
        s.step(12)
        if prec == 1:
            assert np.array_equal(b.get_conserved(k), s.get_conserved()), k
        else:
            assert_batch_matches(b, k, s, p)
        sb, ss = b.stats(k), s.stats()
        assert sb["steps"] == ss["steps"] == 12
        assert abs(sb["t"] - ss["t"]) <= 1e-12 * ss["t"]
        assert sb["riemann_solves"] == ss["riemann_solves"]


def test_batch_vs_oracle(m2c):
    probs = _runs()[:3]
    b = m2c.Batch([m2c.config_for(p) for p in probs], [p.prim for p in probs])
    b.step(10)
    for k, p in enumerate(probs):
        o = oracle.OracleSim(p)
        assert o.step(10) == 0

        class _View:
            def get_conserved(self, k=k):
                return b.get_conserved(k)

            def get_state(self, k=k):
                return b.get_state(k)
        e = compare_runs(_View(), o, p)
        print(k, e)
        assert e["id_mismatch"] == 0
        for name in ("rho", "rhou", "rhov", "rhow", "rhoE", "phi"):
            assert e[name] <= TOL_FP64, (k, name, e[name])


def test_batch_failure_is_isolated(m2c):
    """One run with a CFL far above the limit fails; the others keep stepping
    and match their standalone runs; the failed run keeps its last good state."""
    probs = _runs()[:3]
    cfgs = [m2c.config_for(p) for p in probs]
    cfgs[1].cfl = 5.0
    b = m2c.Batch(cfgs, [p.prim for p in probs])
    rc = b.step(30, check=False)
    assert rc in (m2c.M2C_ERR_NONPHYSICAL, m2c.M2C_ERR_RIEMANN)
    st = b.stats(1)
    assert st["err_code"] == rc and st["steps"] < 30
    s1 = m2c.Sim(cfgs[1], probs[1].prim)
    s1.step(st["steps"])
    assert_batch_matches(b, 1, s1, probs[1])
    for k in (0, 2):
        s = m2c.Sim(cfgs[k], probs[k].prim)
        s.step(30)
        assert b.stats(k)["steps"] == 30
        assert_batch_matches(b, k, s, probs[k])


def test_batch_autotune_keeps_state(m2c, tmp_path):
    probs = _runs()[:4]
    cfgs = [m2c.config_for(p) for p in probs]
    b = m2c.Batch(cfgs, [p.prim for p in probs])
    b.step(3)
    w_before = [b.get_conserved(k) for k in range(len(probs))]
    t_before = [b.stats(k)["t"] for k in range(len(probs))]
    tile, ms = b.autotune(steps=2, cache=str(tmp_path / "tiles.json"), key="unit")
    assert ms > 0
    for k in range(len(probs)):
        assert np.array_equal(b.get_conserved(k), w_before[k])
        assert b.stats(k)["t"] == t_before[k]
    b.step(4)
    # the same sequence without the autotuner: 3 steps on the default tile,
    # 4 on the chosen one (different tiles may round a few cells' energy
    # differently in the last bit, so the reference switches where b did)
    ref = m2c.Batch(cfgs, [p.prim for p in probs])
    ref.step(3)
    ref.set_tile(*tile)
    ref.step(4)
    for k in range(len(probs)):
        assert np.array_equal(b.get_conserved(k), ref.get_conserved(k))
    # the cached tile is reused
    b2 = m2c.Batch(cfgs, [p.prim for p in probs])
    assert b2.autotune(cache=str(tmp_path / "tiles.json"), key="unit")[0] == tile
    assert b2.tile() == tile


def test_single_autotune_keeps_state(m2c):
    p = W.shock_bubble(3, nxyz=(36, 30, 26), radius=0.2, p_shock=1e9, shock_x=0.2)
    s = m2c.Sim(m2c.config_for(p), p.prim)
    s.step(2)
    w = s.get_conserved()
    tile, ms = s.autotune(steps=2)
    assert ms > 0 and s.tile() == tile
    assert np.array_equal(s.get_conserved(), w)
    s.step(3)
    r = m2c.Sim(m2c.config_for(p, tile=tile), p.prim)
    r.step(5)
    assert np.array_equal(s.get_conserved(), r.get_conserved())
