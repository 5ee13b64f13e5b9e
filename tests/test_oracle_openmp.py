"""The all-core (OpenMP) build of the oracle gives bit-identical results to
the serial build: the same states, material ids, counters and error cells.
It is what the CPU baseline times on all host cores."""
import os

import numpy as np
import pytest

import oracle
import workloads as W


@pytest.fixture(scope="module")
def libs():
    oracle.build(force=False)
    oracle.build(force=False, openmp=True)
    serial = oracle.load()
    par = oracle.load(os.path.join(os.path.dirname(oracle.__file__), "liboracle_omp.so"))
    assert serial.ora_num_threads() == 1
    return serial, par


def _run(lib, problem, steps, **kw):
    s = oracle.OracleSim(problem, lib_handle=lib, **kw)
    rc = s.step(steps)
    q, chi = s.prim()
    return rc, s.cons(), chi, s.stats()


@pytest.mark.parametrize("case", ["shock_bubble_rk2", "shock_bubble_rk3_va_llf", "cloud_fe"])
def test_openmp_build_bit_identical(libs, case):
    if case == "shock_bubble_rk2":
        p, kw, steps = W.shock_bubble(3, nxyz=(26, 22, 20), radius=0.25, p_shock=1e9, shock_x=0.3), {}, 25
    elif case == "shock_bubble_rk3_va_llf":
        p = W.shock_bubble(4, nxyz=(20, 17, 15), radius=0.22, p_shock=5e8, shock_x=0.3)
        kw, steps = dict(rk_order=3, limiter=oracle.LIM_VA, limiter_k=2, flux=oracle.FLUX_LLF), 15
    else:
        p, kw, steps = W.bubble_cloud(2, n=24, nbubbles=6), dict(rk_order=1), 20
    a = _run(libs[0], p, steps, **kw)
    b = _run(libs[1], p, steps, **kw)
    assert a[0] == b[0] == 0
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])
    assert a[3] == b[3]
    if case == "shock_bubble_rk2":
        assert a[3]["flips"] > 0 and a[3]["riemann_solves"] > 0


def test_openmp_build_same_failure(libs):
    """Two materials pulled apart faster than any admissible star state:
    both builds stop on the same step with the same error and cell."""
    p = W.uniform_translation(n=40, axis=1, velocity=0.0, pressure=1e5, periodic=False)
    prim = p.prim.reshape(6, -1)
    s_coord = (np.arange(40) + 0.5) / 40
    prim[2] = np.where(s_coord < 0.5, -3000.0, 3000.0)
    p.prim = prim.reshape(p.prim.shape)
    a = _run(libs[0], p, 5)
    b = _run(libs[1], p, 5)
    assert a[0] != 0 and a[0] == b[0]
    assert a[3] == b[3] and a[3]["err_cell"] >= 0
    assert np.array_equal(a[1], b[1])
