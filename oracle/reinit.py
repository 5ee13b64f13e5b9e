"""Level-set reinitialization (TEST INFRASTRUCTURE: only the tests, the smoke
check and the benchmark's CPU-baseline leg may use this module; it shares no
code with the GPU library).

What is computed (section "Level set method", eq. reinit, and section
"Level set method" of the numerical methods): the level set is driven
towards a signed distance by pseudo-time steps of

    d phi / d tau + S(phi_0) (|grad phi| - 1) = 0,
    S(phi_0) = phi_0 / sqrt(phi_0^2 + eps^2),  eps = smallest cell width,

with the upwind (Godunov) discretisation of |grad phi| used with this
equation by Sussman et al.: with one-sided differences a = D^- phi and
b = D^+ phi per axis,

    S > 0:  |grad phi|^2 = sum_d max(max(a_d, 0)^2, min(b_d, 0)^2)
    S < 0:  |grad phi|^2 = sum_d max(min(a_d, 0)^2, max(b_d, 0)^2)

and forward-Euler pseudo-time steps phi <- phi - dtau S (|grad phi| - 1),
dtau = 0.5 min_d h_d (below the monotonicity limit 1/sqrt(sum_d h_d^-2));
the minima run over the axes with more than one cell.

Readings (the paper gives the equation, not these choices): first-order
one-sided differences and forward Euler; a fixed number of pseudo-time
steps; of the paper's first-layer treatments, the one that fixes phi at
the first-layer cells (a cell with a face neighbour of the other sign,
phi >= 0 counting as the non-negative side, as for the material ids) --
they keep phi_0; narrow band: with band > 0 only cells with |phi_0| < band
are updated.  Frozen cells are expressed as S = 0.  Boundary images are
those of the finite-volume step: transmissive and wall boundaries repeat
the boundary cell for the one layer used here (zero-gradient and mirror
images coincide there), periodic boundaries wrap; axes with one cell are
inactive.
"""
from __future__ import annotations

import numpy as np

BC_TRANSMISSIVE, BC_WALL, BC_PERIODIC = 0, 1, 2


def _pad(phi, bc):
    """One image layer per side; phi is (nz, ny, nx), bc = (-x,+x,-y,+y,-z,+z)."""
    out = phi
    for axis_np, d in ((2, 0), (1, 1), (0, 2)):
        mode = "wrap" if bc[2 * d] == BC_PERIODIC else "edge"
        pw = [(0, 0)] * 3
        pw[axis_np] = (1, 1)
        out = np.pad(out, pw, mode=mode)
    return out


def smoothed_sign(phi0, eps):
    return phi0 / np.sqrt(phi0 * phi0 + eps * eps)


def first_layer(phi0, bc):
    """Cells with a face neighbour on the other side of the zero level set."""
    pos = _pad(phi0, bc) >= 0.0
    c = pos[1:-1, 1:-1, 1:-1]
    nz, ny, nx = phi0.shape
    fl = np.zeros(phi0.shape, dtype=bool)
    for sl, n in ((np.s_[1:-1, 1:-1, :-2], nx), (np.s_[1:-1, 1:-1, 2:], nx),
                  (np.s_[1:-1, :-2, 1:-1], ny), (np.s_[1:-1, 2:, 1:-1], ny),
                  (np.s_[:-2, 1:-1, 1:-1], nz), (np.s_[2:, 1:-1, 1:-1], nz)):
        if n > 1:
            fl |= pos[sl] != c
    return fl


def _hmin(shape, h):
    """Smallest cell width over the axes with more than one cell."""
    act = [h[d] for d in range(3) if shape[2 - d] > 1]
    return min(act) if act else min(h)


def speed(phi0, h, bc, band=0.0, eps=None):
    """S(phi_0) with the frozen cells (first layer, outside the band) at 0;
    eps defaults to the smallest cell width."""
    eps = _hmin(phi0.shape, h) if eps is None else eps
    S = smoothed_sign(phi0, eps)
    S[first_layer(phi0, bc)] = 0.0
    if band > 0.0:
        S[np.abs(phi0) >= band] = 0.0
    return S


def grad_norm(phi, S, h, bc):
    """Godunov |grad phi| with the upwinding chosen by the sign of S."""
    P = _pad(phi, bc)
    c = P[1:-1, 1:-1, 1:-1]
    g2 = np.zeros_like(phi)
    for d, (lo, hi) in enumerate(((np.s_[1:-1, 1:-1, :-2], np.s_[1:-1, 1:-1, 2:]),
                                  (np.s_[1:-1, :-2, 1:-1], np.s_[1:-1, 2:, 1:-1]),
                                  (np.s_[:-2, 1:-1, 1:-1], np.s_[2:, 1:-1, 1:-1]))):
        if phi.shape[2 - d] == 1:
            continue
        a = (c - P[lo]) / h[d]
        b = (P[hi] - c) / h[d]
        pos = np.maximum(np.maximum(a, 0.0) ** 2, np.minimum(b, 0.0) ** 2)
        neg = np.maximum(np.minimum(a, 0.0) ** 2, np.maximum(b, 0.0) ** 2)
        g2 += np.where(S > 0.0, pos, neg)
    return np.sqrt(g2)


def reinit(phi0, h, bc, iters, band=0.0, eps=None):
    """phi after `iters` pseudo-time steps (phi0 is (nz, ny, nx) float64)."""
    phi0 = np.asarray(phi0, dtype=np.float64)
    S = speed(phi0, h, bc, band, eps)
    dtau = 0.5 * _hmin(phi0.shape, h)
    phi = phi0.copy()
    for _ in range(iters):
        phi = phi - dtau * S * (grad_norm(phi, S, h, bc) - 1.0)
    return phi
