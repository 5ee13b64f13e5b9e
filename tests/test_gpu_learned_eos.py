"""Learned start of the general-EOS Riemann solver on the GPU, through the
C ABI: the feature map against its written definition (oracle sound speeds
and floors), the star states against the acoustic start and the oracle,
fewer outer Newton steps on held-out problems, and the acoustic start kept
for Mie-Grueneisen problems and near equilibrium.

The learned start only decides where the outer iteration begins; both
starts iterate to the same tolerance, so their star states agree to the
stopping rule (p* to 1e-10 of p* - p_lo, u* to 1e-9 of the larger sound
speed) and both meet the oracle bar of ``tests/test_gpu_riemann_eos.py``.
"""
from __future__ import annotations

import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import riemann_eos as RE

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NASG, MG, JWL = 0, 1, 2
NO_MG = [pr for pr in W.EOS_PAIRS if all(W.EOS_MATERIALS[m][0] != MG for m in pr)]
JWL_NO_MG = [pr for pr in NO_MG if any(W.EOS_MATERIALS[m][0] == JWL for m in pr)]


@pytest.fixture(scope="module")
def m2c():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_16387_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def net(m2c):
    return m2c.Mlp(np.load(os.path.join(ROOT, "paper_2508_16387_amd", "learned_guess_eos.npy")))


def _dev(inp, mat):
    import torch
    return (torch.tensor(np.ascontiguousarray(inp), dtype=torch.float64, device="cuda"),
            torch.tensor(np.ascontiguousarray(mat), dtype=torch.int32, device="cuda"))


def _features_ref(inp, mat, mats):
    """The feature map written out from its definition in include/m2c.h,
    with the oracle's sound speeds and floors."""
    eos = [RE.make_eos(f, p) for f, p in mats]
    n = inp.shape[1]
    X = np.zeros((8, n))
    plo_all, P_all = np.zeros(n), np.ones(n)
    for i in range(n):
        a, b = int(mat[0, i]), int(mat[1, i])
        q = inp[:, i].copy()
        if mats[a][0] > mats[b][0]:                     # lower family on the left, mirrored
            a, b = b, a
            q = np.array([q[3], -q[4], q[5], q[0], -q[1], q[2]])
        mL, mR = eos[a], eos[b]
        rL, uL, pL, rR, uR, pR = q
        cL, cR = RE.Side(mL, rL, uL, pL).c, RE.Side(mR, rR, uR, pR).c
        flL, flR = mL.floor, mR.floor
        pfl = max(flL + 1e-12 * (pL - flL) + 1e-6 * abs(flL), flR + 1e-12 * (pR - flR) + 1e-6 * abs(flR))
        plo = max(flL, flR)
        zL, zR = rL * cL, rR * cR
        pac = (zR * pL + zL * pR - zL * zR * (uR - uL)) / (zL + zR)
        if not pac > pfl:
            pac = pfl + 0.5 * (min(pL, pR) - pfl)
        aL, aR = pL - plo, pR - plo
        P = math.sqrt(aL * aR)
        U = math.sqrt(P / math.sqrt(rL * rR))
        X[:, i] = [0.5 * math.log(rL / rR), (uR - uL) / U, 0.5 * math.log(aL / aR), math.log(rL * cL * cL / aL),
                   math.log(rR * cR * cR / aR), math.log((pac - plo) / P), mats[a][0] - 1, mats[b][0] - 1]
        plo_all[i], P_all[i] = plo, P
    return X, plo_all, P_all


def _floor_and_speed(inp, mat, mats):
    """Higher floor and larger initial sound speed of every problem (oracle EOS)."""
    eos = [RE.make_eos(f, p) for f, p in mats]
    fl = np.array([max(eos[a].floor, eos[b].floor) for a, b in zip(mat[0], mat[1])])
    cmax = np.array([max(RE.Side(eos[a], *inp[0:3, i]).c, RE.Side(eos[b], *inp[3:6, i]).c)
                     for i, (a, b) in enumerate(zip(mat[0], mat[1]))])
    return fl, cmax


def test_features_match_their_definition(m2c):
    inp, mat, mats, _ = W.general_eos_problem_set(5100, 300)
    ti, tm = _dev(inp, mat)
    out, it, _ = m2c.riemann_solve_eos(ti, tm, mats)
    X, t = m2c.mlp_features_eos(ti, tm, mats, pstar=out[0].contiguous())
    Xg, tg, ps = X.cpu().numpy(), t.cpu().numpy(), out[0].cpu().numpy()
    Xr, plo, P = _features_ref(inp, mat, mats)
    ok = np.isfinite(ps)
    assert ok.sum() > 250
    err = np.abs(Xg[:, ok] - Xr[:, ok]) / (1.0 + np.abs(Xr[:, ok]))
    print("max feature error per row", err.max(axis=1))
    assert err.max() <= 2e-6
    tr = np.log((ps[ok] - plo[ok]) / P[ok])
    assert np.max(np.abs(tg[ok] - tr) / (1.0 + np.abs(tr))) <= 2e-6


def test_learned_start_keeps_the_star_state(m2c, net):
    """Problems of the pairs the network is consulted for: the learned and
    the acoustic start give the same star states (to the stopping rule) and
    meet the oracle bar on a sample."""
    inp, mat, mats, _ = W.general_eos_problem_set(5200, 4096, pairs=NO_MG)
    ti, tm = _dev(inp, mat)
    oa, ia, ra, _ = m2c.riemann_solve_eos_learned(None, ti, tm, mats)
    ol, il, rl, nfb = m2c.riemann_solve_eos_learned(net, ti, tm, mats)
    oa, ol, ia, il = oa.cpu().numpy(), ol.cpu().numpy(), ia.cpu().numpy(), il.cpu().numpy()
    assert ra == rl
    assert np.array_equal(np.isnan(oa[0]), np.isnan(ol[0])) and np.array_equal(ia == 0, il == 0)
    ok = ia != 0
    fl, cmax = _floor_and_speed(inp, mat, mats)
    dp = np.abs(ol[0] - oa[0])[ok] / (oa[0][ok] - fl[ok])
    du = np.abs(ol[1] - oa[1])[ok] / cmax[ok]
    print("max p* difference / (p* - p_lo)", dp.max(), "max u* difference / c", du.max(), "acoustic starts", nfb)
    assert dp.max() <= 1e-10 and du.max() <= 1e-9
    assert 0 < nfb < ok.sum()
    from tests.test_gpu_riemann_eos import TOL_EOS, _compare
    idx = np.random.default_rng(3).choice(inp.shape[1], 40, replace=False)
    e, okc = _compare(inp[:, idx], mat[:, idx], mats, ol[:, idx], il[idx], "learned start")
    assert e.max() <= TOL_EOS


def test_learned_start_takes_fewer_outer_steps(m2c, net):
    inp, mat, mats, _ = W.general_eos_problem_set(5300, 1 << 16, pairs=JWL_NO_MG)
    ti, tm = _dev(inp, mat)
    _, ia, _, _ = m2c.riemann_solve_eos_learned(None, ti, tm, mats)
    _, il, _, nfb = m2c.riemann_solve_eos_learned(net, ti, tm, mats)
    ia, il = ia.cpu().numpy(), il.cpu().numpy()
    ok = (ia != 0) & (il != 0)
    sa, sl = np.abs(ia[ok]).mean(), np.abs(il[ok]).mean()
    print(f"outer Newton steps: acoustic {sa:.3f}, learned {sl:.3f}, acoustic starts {nfb} of {ok.sum()}")
    assert sl <= 0.85 * sa


@pytest.mark.parametrize("pairs", [[("copper", "tantalum"), ("air", "glass")], [("water_nasg", "gas_nasg")],
                                   [("tnt", "air"), ("copper", "tnt")]],
                         ids=["mie_grueneisen", "nasg_both_sides", "jwl_beside_mie_grueneisen"])
def test_sets_that_take_the_acoustic_start(m2c, net, pairs):
    """Sets the network is not consulted for (Mie-Grueneisen problems,
    NASG on both sides, JWL problems in a set with Mie-Grueneisen ones) run
    the acoustic kernels: the same bits as the plain solver, every solve an
    acoustic start."""
    inp, mat, mats, _ = W.general_eos_problem_set(5400, 2000, pairs=pairs)
    ti, tm = _dev(inp, mat)
    o0, i0, r0 = m2c.riemann_solve_eos(ti, tm, mats)
    ol, il, rl, nfb = m2c.riemann_solve_eos_learned(net, ti, tm, mats)
    assert r0 == rl
    o0, ol, i0, il = o0.cpu().numpy(), ol.cpu().numpy(), i0.cpu().numpy(), il.cpu().numpy()
    assert np.array_equal(i0, il)
    assert np.array_equal(o0, ol, equal_nan=True)
    assert nfb == int((il != 0).sum())


def test_untrained_network_keeps_the_star_state(m2c):
    """Random weights: the judge keeps the answer (only the steps change)."""
    raw = m2c.Mlp(seed=11)
    inp, mat, mats, _ = W.general_eos_problem_set(5500, 4096, pairs=NO_MG)
    ti, tm = _dev(inp, mat)
    oa, ia, _, _ = m2c.riemann_solve_eos_learned(None, ti, tm, mats)
    ol, il, _, _ = m2c.riemann_solve_eos_learned(raw, ti, tm, mats)
    oa, ol, ia, il = oa.cpu().numpy(), ol.cpu().numpy(), ia.cpu().numpy(), il.cpu().numpy()
    ok = (ia != 0) & (il != 0)
    assert np.array_equal(ia == 0, il == 0)
    fl, cmax = _floor_and_speed(inp, mat, mats)
    assert (np.abs(ol[0] - oa[0])[ok] / (oa[0][ok] - fl[ok])).max() <= 1e-10
    assert (np.abs(ol[1] - oa[1])[ok] / cmax[ok]).max() <= 1e-9


def test_learned_start_in_the_general_eos_step(m2c, net):
    """The grid step with a general EOS per material and the learned start
    at interface faces (JWL products in NASG water): the state after the
    steps matches the oracle at the FP64 bar and the acoustic-start run to
    the stopping rule, with fewer outer steps per interface solve."""
    import oracle
    from tests.parity import TOL_FP64, compare_runs
    p = W.eos_charge(21, n=(20, 18, 16), steps=8)
    print(p.name, p.n, "steps", p.steps, flush=True)
    o = oracle.OracleSim(p)
    assert o.step(p.steps) == 0
    runs = {}
    for name, guess in (("acoustic", None), ("learned", net)):
        g = m2c.Sim(m2c.config_for(p), p.prim)
        if guess is not None:
            g.set_guess(guess)
        assert g.step(p.steps) == 0
        st = g.stats()
        e = compare_runs(g, o, p)
        print(name, {k: (f"{v:.2e}" if isinstance(v, float) else v) for k, v in e.items()},
              "outer steps per solve", st["newton_iters"] / st["riemann_solves"], "acoustic starts",
              st["mlp_fallbacks"], "of", st["riemann_solves"], flush=True)
        assert e["id_mismatch"] == 0
        for k in ("rho", "rhou", "rhov", "rhow", "rhoE", "phi"):
            assert e[k] <= TOL_FP64, (name, k, e[k])
        runs[name] = (g.get_conserved(), st)
        g.close()
    (wa, sa), (wl, sl) = runs["acoustic"], runs["learned"]
    assert sa["riemann_solves"] == sl["riemann_solves"]
    assert sl["newton_iters"] < sa["newton_iters"]
    assert 0 < sl["mlp_fallbacks"] < sl["riemann_solves"]
    scale = np.maximum(np.abs(wa).max(axis=1, keepdims=True), 1e-30)
    assert np.max(np.abs(wl - wa) / scale) <= 1e-10
