"""General-EOS two-material Riemann solver and EOS evaluation on the GPU
against the oracle (``oracle/riemann_eos.py``), through the C ABI.

Numerics bar.  The oracle integrates isentropes with DOP853 at relative
tolerance 1e-13 and brackets every root; the library integrates them with
RK4 over ln(p - floor) at steps of at most ds (Mie-Grueneisen; NASG and
JWL isentropes are closed forms, the JWL Riemann-invariant integral by
Gauss-Legendre quadrature) and stops its Newton iterations
at |dp| <= rtol (p - floor).  Both are FP64, so the difference is the RK4
truncation error plus the two stopping rules.  Errors are measured as:
u* relative to the larger sound speed of the two initial states; p* as the
velocity change its difference amounts to across the two star impedances
(|dp| (1/(rho* c*)_L + 1/(rho* c*)_R)), on the same scale -- near
cavitation p* is many decades below the pressures of the problem and is
fixed by the velocities; rho* relative.  TOL_EOS bounds all three at the
default ds = 0.01; the test of the step size shows that the RK4 part of the
error shrinks at fourth order.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import riemann_eos as RE

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL_EOS = 1e-9


@pytest.fixture(scope="module")
def m2c():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_16387_amd as m
    m.lib()
    return m


def _gpu(m2c, inp, mat, mats, ds=0.0, rtol=1e-12):
    import torch
    ti = torch.tensor(np.ascontiguousarray(inp), dtype=torch.float64, device="cuda")
    tm = torch.tensor(np.ascontiguousarray(mat), dtype=torch.int32, device="cuda")
    out, it, rc = m2c.riemann_solve_eos(ti, tm, mats, rtol=rtol, ds=ds)
    torch.cuda.synchronize()
    return out.cpu().numpy(), it.cpu().numpy(), rc


def _errors(inp, mat, eos, ref, got):
    """Per-problem (p, u, rho) errors on the scales of the module docstring."""
    n = inp.shape[1]
    e = np.zeros((3, n))
    for i in range(n):
        mL, mR = eos[mat[0, i]], eos[mat[1, i]]
        cL = RE.Side(mL, inp[0, i], inp[1, i], inp[2, i]).c
        cR = RE.Side(mR, inp[3, i], inp[4, i], inp[5, i]).c
        # the velocity change that the p* difference amounts to across the
        # two star impedances rho* c*
        p, rL, rR = ref[0, i], ref[2, i], ref[3, i]
        zinv = 1.0 / (rL * np.sqrt(mL.c2(rL, mL.e(rL, p)))) + 1.0 / (rR * np.sqrt(mR.c2(rR, mR.e(rR, p))))
        e[0, i] = abs(got[0, i] - p) * zinv / max(cL, cR)
        e[1, i] = abs(got[1, i] - ref[1, i]) / max(cL, cR)
        e[2, i] = max(abs(got[2, i] / ref[2, i] - 1), abs(got[3, i] / ref[3, i] - 1))
    return e


def _compare(inp, mat, mats, got, it, label):
    eos = [RE.make_eos(f, p) for f, p in mats]
    ref = RE.solve(inp, mat, eos)
    bad_ref, bad_got = np.isnan(ref[0]), np.isnan(got[0])
    assert np.array_equal(bad_ref, bad_got), (label, np.flatnonzero(bad_ref != bad_got))
    assert np.all(it[bad_got] == 0) and np.all(it[~bad_got] != 0), label
    ok = ~bad_ref
    e = _errors(inp[:, ok], mat[:, ok], eos, ref[:, ok], got[:, ok])
    print(label, "n", ok.sum(), "cavitation", bad_ref.sum(), "max err p,u,rho", e.max(axis=1),
          "iters", np.abs(it[ok]).mean(), flush=True)
    return e, ok


@pytest.mark.parametrize("pair", W.EOS_PAIRS, ids=["-".join(p) for p in W.EOS_PAIRS])
def test_riemann_eos_matches_oracle(m2c, pair):
    inp, mat, mats, names = W.general_eos_problem_set(100 + W.EOS_PAIRS.index(pair), 40, pairs=[pair])
    got, it, rc = _gpu(m2c, inp, mat, mats)
    e, ok = _compare(inp, mat, mats, got, it, pair)
    assert rc == (m2c.M2C_OK if ok.all() else m2c.M2C_ERR_RIEMANN)
    assert ok.sum() >= 30
    assert e.max() <= TOL_EOS, e.max(axis=1)


def test_riemann_eos_jwl_both_sides_matches_oracle(m2c):
    """Detonation products on both sides (the JWL / JWL kernel)."""
    inp, mat, mats, names = W.general_eos_problem_set(140, 40, pairs=[("tnt", "tnt")])
    got, it, rc = _gpu(m2c, inp, mat, mats)
    e, ok = _compare(inp, mat, mats, got, it, "tnt-tnt")
    assert ok.sum() >= 30
    assert e.max() <= TOL_EOS, e.max(axis=1)


@pytest.mark.parametrize("pair", [("air", "glass"), ("copper", "tnt"), ("tnt", "water_sg")],
                         ids=["air-glass", "copper-tnt", "tnt-water_sg"])
def test_riemann_eos_mirror_symmetry(m2c, pair):
    """Reflection x -> -x of every problem (sides swapped, velocities
    negated) gives p* unchanged, u* negated and the star densities swapped,
    bit for bit: each problem is solved with the lower family on the left,
    so a problem and its mirror image take the same arithmetic."""
    inp, mat, mats, _ = W.general_eos_problem_set(150 + len(pair[0]), 500, pairs=[pair])
    mir = np.stack([inp[3], -inp[4], inp[5], inp[0], -inp[1], inp[2]])
    got, it, rc = _gpu(m2c, inp, mat, mats)
    gm, im, rcm = _gpu(m2c, np.ascontiguousarray(mir), np.ascontiguousarray(mat[::-1]), mats)
    assert rc == rcm and np.array_equal(it, im)
    ok = np.isfinite(got[0])
    assert ok.sum() >= 400
    assert np.array_equal(got[0][ok], gm[0][ok])
    assert np.array_equal(got[1][ok], -gm[1][ok])
    assert np.array_equal(got[2][ok], gm[3][ok]) and np.array_equal(got[3][ok], gm[2][ok])


def test_rk4_step_size_order(m2c):
    """Rarefaction-dominated Mie-Grueneisen problems (the family whose
    isentropes are integrated by RK4; NASG and JWL use closed forms) at two
    step sizes: the error against the oracle falls by about 2^4 when ds
    halves."""
    inp, mat, mats, _ = W.general_eos_problem_set(7, 24, pairs=[("glass", "water_nasg"), ("copper", "tantalum")])
    inp[1], inp[4] = -np.abs(inp[1]), np.abs(inp[4])       # separating: both waves rarefactions
    eos = [RE.make_eos(f, p) for f, p in mats]
    ref = RE.solve(inp, mat, eos)
    ok = ~np.isnan(ref[0])
    errs = []
    # (at ds = 0.2 and 0.1 the glass isentropes are still pre-asymptotic)
    for ds in (0.04, 0.02):
        got, it, _ = _gpu(m2c, inp, mat, mats, ds=ds, rtol=1e-14)
        e = _errors(inp[:, ok], mat[:, ok], eos, ref[:, ok], got[:, ok])
        errs.append(e[1].max())
    print("ds 0.04 / 0.02 u errors", errs, flush=True)
    assert errs[0] > 1e-10, errs                      # the truncation error is visible at ds = 0.04
    assert 8.0 <= errs[0] / errs[1] <= 32.0, errs


def test_glass_air_worked_example(m2c):
    d = json.load(open(os.path.join(HERE, "golden", "riemann_eos_glass_air.json")))
    inp = np.array([[d["left"]["rho"]], [d["left"]["u"]], [d["left"]["p"]],
                    [d["right"]["rho"]], [d["right"]["u"]], [d["right"]["p"]]])
    mat = np.array([[0], [1]], dtype=np.int32)
    mats = [(RE.NASG, d["left"]["params"]), (RE.MG, d["right"]["params"])]
    got, it, rc = _gpu(m2c, inp, mat, mats)
    assert rc == m2c.M2C_OK
    assert round(got[3, 0], 2) == d["printed"]["rho_star_glass_kg_m3"]
    e, ok = _compare(inp, mat, mats, got, it, "glass-air")
    assert e.max() <= TOL_EOS


def test_cavitation_and_inadmissible_inputs(m2c):
    """No star state, an index outside the table and a pressure below the
    floor give NaN and iters = 0 for those problems only."""
    mats = [(RE.NASG, [1.4, 0.0, 0.0, 0.0]), (RE.NASG, [6.12, 3.43e8, 0.0, 0.0])]
    inp = np.array([[1.2, 1.2, 1.2, 1000.0, 1.2],
                    [-2000.0, 0.0, 0.0, 0.0, -10.0],
                    [1e5, 1e5, 1e5, -3.5e8, 1e5],
                    [1.2, 1.2, 1.2, 1.2, 1000.0],
                    [2000.0, 0.0, 0.0, 0.0, 10.0],
                    [1e5, 1e5, 1e5, 1e5, 1e6]])
    mat = np.array([[0, 0, 5, 1, 0], [0, 0, 0, 0, 1]], dtype=np.int32)
    got, it, rc = _gpu(m2c, inp, mat, mats)
    assert rc == m2c.M2C_ERR_RIEMANN
    assert np.isnan(got[:, [0, 2, 3]]).all() and (it[[0, 2, 3]] == 0).all()
    assert np.isfinite(got[:, [1, 4]]).all() and (it[[1, 4]] != 0).all()
    assert abs(got[0, 1] - 1e5) <= 1e-12 * 1e5 and abs(got[1, 1]) <= 1e-12   # equal states
    eos = [RE.make_eos(f, p) for f, p in mats]
    ref = RE.solve(inp[:, [4]], mat[:, [4]], eos)
    assert _errors(inp[:, [4]], mat[:, [4]], eos, ref, got[:, [4]]).max() <= TOL_EOS


def test_near_equal_states(m2c):
    """States a few ulps apart (as two cells at rest in pressure equilibrium
    become after some steps): a shock too weak for the specific volume to
    change in FP64 is a valid wave, and p* is the common pressure."""
    names = ["water_sg", "air", "copper", "tnt", "glass", "water_nasg"]
    mats = [W._eos_of(k) for k in names]
    rows = []
    for a, b, ra, rb, p0 in ((0, 1, 1000.0, 1.0, 1e5), (2, 3, 8930.0, 1630.0, 1e9), (4, 5, 2204.0, 1000.0, 1e8)):
        for dl, dr in ((0, 1), (0, -1), (2, 1), (-3, 4), (1e3, 0)):
            pl = p0 + dl * math.ulp(p0)
            pr = p0 + dr * math.ulp(p0)
            rows.append(((ra, 0.0, pl, rb * (1 + 4e-16), 0.0, pr), (a, b)))
    inp = np.array([r[0] for r in rows]).T.copy()
    mat = np.array([r[1] for r in rows], dtype=np.int32).T.copy()
    got, it, rc = _gpu(m2c, inp, mat, mats)
    print("near-equal p*", got[0], "iters", it, flush=True)
    assert rc == m2c.M2C_OK and (it != 0).all()
    assert np.all(np.abs(got[0] / inp[2] - 1.0) <= 1e-12)
    _compare(inp, mat, mats, got, it, "near-equal")


def test_eos_eval_matches_oracle(m2c):
    import torch
    names = sorted(W.EOS_MATERIALS)
    mats = [(W.EOS_MATERIALS[k][0], W.EOS_MATERIALS[k][1]) for k in names]
    eos = [RE.make_eos(f, p) for f, p in mats]
    rng = np.random.default_rng(5)
    rho, e, mid, pref = [], [], [], []
    for i, k in enumerate(names):
        _, _, rr, pr, _ = W.EOS_MATERIALS[k]
        for _ in range(32):
            r = rng.uniform(rr[0], rr[1])
            p = rng.uniform(pr[0], pr[1])
            rho.append(r)
            e.append(eos[i].e(r, p))
            mid.append(i)
            pref.append(p)
    t = lambda a, dt: torch.tensor(a, dtype=dt, device="cuda")
    p, c = m2c.eos_eval(t(rho, torch.float64), t(e, torch.float64), t(mid, torch.int32), mats)
    p, c = p.cpu().numpy(), c.cpu().numpy()
    for j in range(len(rho)):
        m = eos[mid[j]]
        pr = m.p(rho[j], e[j])
        cr = math.sqrt(m.c2(rho[j], e[j]))
        scale = abs(pref[j]) + abs(m.floor) + 1e5
        assert abs(p[j] - pr) <= 1e-12 * scale, (names[mid[j]], p[j], pr)
        assert abs(c[j] / cr - 1) <= 1e-10, (names[mid[j]], c[j], cr)


def test_large_batch_sampled(m2c):
    """2^20 mixed problems (the benchmark's set) in one launch; 32 sampled
    problems against the oracle."""
    n = 1 << 20
    inp, mat, mats, _ = W.general_eos_problem_set(2024, n)
    got, it, rc = _gpu(m2c, inp, mat, mats)
    assert rc in (m2c.M2C_OK, m2c.M2C_ERR_RIEMANN)
    finite = np.isfinite(got[0])
    assert finite.mean() > 0.9
    idx = np.random.default_rng(1).choice(n, 32, replace=False)
    e, ok = _compare(inp[:, idx], mat[:, idx], mats, got[:, idx], it[idx], "sampled")
    assert e.max() <= TOL_EOS
