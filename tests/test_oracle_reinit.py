"""Pins of the level-set reinitialization oracle (``oracle/reinit.py``).

Checks against what the equation and its upwind discretisation fix, not
against a retyped copy of the oracle:

* in 1D the steady state of the upwind scheme is known exactly: away from
  the frozen first-layer cells phi grows by exactly one cell width per cell
  on each side of the interface;
* a signed-distance plane is a fixed point;
* on a sphere whose level set is far from a distance (phi_0 = 3 (r^2 -
  R^2), slope 6R at the interface) the result approaches r - R near the
  interface, with the error falling as the grid is refined;
* the sign of phi (the material ids) and the first-layer values never
  change, and cells outside the narrow band keep phi_0;
* the smoothed sign S(phi_0) = phi_0 / sqrt(phi_0^2 + eps^2) is odd and
  bounded by 1.

``test_planted_mistakes`` plants mistakes in a copy of the oracle.
"""
from __future__ import annotations

import importlib.util

import numpy as np
import pytest

from oracle import reinit as RI_MOD

T, W, P = 0, 1, 2


def field_1d(n, x0, f):
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    return f(x - x0).reshape(1, 1, n), (h, 1.0, 1.0)


def check_1d_steady_state(RI):
    for x0, f in ((0.4137, lambda d: 3.0 * d), (0.61, lambda d: d * (2.0 + np.sin(5.0 * d))),
                  (0.5003, lambda d: np.sinh(4.0 * d) / 4.0)):
        phi0, h = field_1d(64, x0, f)
        phi = RI.reinit(phi0, h, (T,) * 6, iters=400)[0, 0]
        p0 = phi0[0, 0]
        i = int(np.argmax(p0 >= 0.0))          # first non-negative cell
        assert phi[i - 1] == p0[i - 1] and phi[i] == p0[i]       # first layer fixed
        # downwind of the first layer the steady state is a ramp of slope 1
        ref_r = p0[i] + h[0] * np.arange(0, 64 - i)
        ref_l = p0[i - 1] - h[0] * np.arange(0, i)
        assert np.allclose(phi[i:], ref_r, rtol=0, atol=1e-12), (x0, np.abs(phi[i:] - ref_r).max())
        assert np.allclose(phi[:i][::-1], ref_l, rtol=0, atol=1e-12), (x0, np.abs(phi[:i][::-1] - ref_l).max())


def check_plane_fixed_point(RI):
    n = (20, 12, 10)
    h = (1.0 / n[0], 1.0 / n[1], 1.0 / n[2])
    x = (np.arange(n[0]) + 0.5) * h[0]
    phi0 = np.broadcast_to(x - 0.437, (n[2], n[1], n[0])).copy()
    phi = RI.reinit(phi0, h, (T, T, P, P, P, P), iters=60)
    assert np.abs(phi - phi0).max() <= 1e-14


def sphere(n, R=0.3):
    h = 1.0 / n
    c = (np.arange(n) + 0.5) * h - 0.5
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    r = np.sqrt(x * x + y * y + z * z)
    return 3.0 * (r * r - R * R), r - R, (h, h, h)


def check_sphere_converges(RI):
    errs = []
    for n in (32, 64):
        phi0, dist, h = sphere(n)
        phi = RI.reinit(phi0, h, (T,) * 6, iters=n)
        near = np.abs(dist) < 0.12
        errs.append(np.abs(phi - dist)[near].max())
        # the initial field is far from a distance there
        assert np.abs(phi0 - dist)[near].max() > 3 * errs[-1]
    # first order: the frozen first layer carries phi_0's slope error, O(h)
    assert errs[1] < 0.6 * errs[0], errs


def check_invariants(RI):
    rng = np.random.default_rng(4)
    n = 20
    phi0, _, h = sphere(n, R=0.27)
    phi0 = phi0 * (1.0 + 0.3 * rng.random(phi0.shape))
    bc = (T, W, P, P, W, T)
    phi = RI.reinit(phi0, h, bc, iters=40)
    assert np.array_equal(phi >= 0.0, phi0 >= 0.0)
    fl = RI.first_layer(phi0, bc)
    assert fl.any() and np.array_equal(phi[fl], phi0[fl])
    band = 0.1
    pb = RI.reinit(phi0, h, bc, iters=40, band=band)
    out = np.abs(phi0) >= band
    assert out.any() and np.array_equal(pb[out], phi0[out])
    assert not np.array_equal(pb[~out & ~fl], phi0[~out & ~fl])
    s = RI.smoothed_sign(np.arange(-20, 21) * 0.05, 0.05)
    assert np.array_equal(s, -s[::-1]) and np.abs(s).max() < 1.0 and s[20] == 0.0


CHECKS = {f.__name__: f for f in (check_1d_steady_state, check_plane_fixed_point, check_sphere_converges,
                                  check_invariants)}


@pytest.mark.parametrize("name", sorted(CHECKS))
def test_pin(name):
    CHECKS[name](RI_MOD)


MUTANTS = [
    ("upwinding swapped", "g2 += np.where(S > 0.0, pos, neg)", "g2 += np.where(S > 0.0, neg, pos)",
     "check_1d_steady_state"),
    ("minus one dropped", "S * (grad_norm(phi, S, h, bc) - 1.0)", "S * grad_norm(phi, S, h, bc)",
     "check_plane_fixed_point"),
    ("first layer not frozen", "    S[first_layer(phi0, bc)] = 0.0\n", "", "check_1d_steady_state"),
    ("one-sided difference sign", "a = (c - P[lo]) / h[d]", "a = (P[lo] - c) / h[d]", "check_1d_steady_state"),
    ("pseudo-time step", "dtau = 0.5 * _hmin(", "dtau = 0.05 * _hmin(", "check_sphere_converges"),
]


@pytest.mark.parametrize("label,old,new,check", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistakes(label, old, new, check, tmp_path):
    src = open(RI_MOD.__file__).read()
    assert src.count(old) == 1, label
    path = tmp_path / "reinit_mutant.py"
    path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location("reinit_mutant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    with pytest.raises(AssertionError):
        CHECKS[check](mod)
