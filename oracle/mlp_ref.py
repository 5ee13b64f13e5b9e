"""FP64 reference of the learned star-pressure guess (TEST INFRASTRUCTURE).

The paper accelerates its exact two-material Riemann solver without new
approximations (section "Spatial discretization of governing equations",
last paragraph); here the acceleration is a learned initial guess for the
star-pressure Newton iteration, which then iterates to the same tolerance.
This module is the plain reference the GPU inference and training kernels
are checked against: a multilayer perceptron 8 -> 64 -> 64 -> 1 with tanh
hidden layers, mean-squared-error loss, and Adam.  It shares no code with
the GPU library.

Parameter vector (4801 values): W1 (64x8, row-major), b1 (64), W2 (64x64,
row-major), b2 (64), w3 (64), b3 (1).

Inputs of one Riemann problem (rho, u, p and (gamma, p_c) on both sides)
are mapped to eight dimensionless features, and the network predicts
y = ln((p* - p_lo)/P) with p_lo = -min(p_cL, p_cR) the lower end of the
admissible star pressures and P = sqrt((p_L - p_lo)(p_R - p_lo)), so that
the guess p_lo + P exp(y) is admissible for any output:

  rb = sqrt(rho_L rho_R), U = sqrt(P / rb), ub = (u_L + u_R)/2
  x = [ln(rho_L/rb), ln(rho_R/rb), (u_L - ub)/U, (u_R - ub)/U,
       ln((p_L - p_lo)/P), ln((p_R - p_lo)/P), ln(gamma_L/gamma_R),
       (p_cL - p_cR)/(p_cL + p_cR + P)]
"""
from __future__ import annotations

import numpy as np

NIN, NH = 8, 64
SIZES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("w3", (NH,)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def init(seed=0):
    """Glorot-uniform weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in SIZES:
        if len(shape) == 2:
            lim = np.sqrt(6.0 / (shape[0] + shape[1]))
            p[name] = rng.uniform(-lim, lim, shape)
        elif name == "w3":
            lim = np.sqrt(6.0 / (NH + 1))
            p[name] = rng.uniform(-lim, lim, shape)
        else:
            p[name] = np.zeros(shape)
    return pack(p)


def scales(inp, eos):
    """(p_lo, P) per problem; inp [n,6] = (rho_L,u_L,p_L,rho_R,u_R,p_R),
    eos [n,4] = (gamma_L, pc_L, gamma_R, pc_R)."""
    inp = np.atleast_2d(inp)
    eos = np.atleast_2d(eos)
    plo = -np.minimum(eos[:, 1], eos[:, 3])
    P = np.sqrt((inp[:, 2] - plo) * (inp[:, 5] - plo))
    return plo, P


def features(inp, eos):
    inp = np.atleast_2d(np.asarray(inp, dtype=np.float64))
    eos = np.atleast_2d(np.asarray(eos, dtype=np.float64))
    plo, P = scales(inp, eos)
    rL, uL, pL, rR, uR, pR = inp.T
    gL, pcL, gR, pcR = eos.T
    rb = np.sqrt(rL * rR)
    U = np.sqrt(P / rb)
    ub = 0.5 * (uL + uR)
    X = np.stack([np.log(rL / rb), np.log(rR / rb), (uL - ub) / U, (uR - ub) / U,
                  np.log((pL - plo) / P), np.log((pR - plo) / P), np.log(gL / gR),
                  (pcL - pcR) / (pcL + pcR + P)], axis=1)
    return X


def target(pstar, inp, eos):
    plo, P = scales(inp, eos)
    return np.log((np.asarray(pstar) - plo) / P)


def guess(y, inp, eos):
    plo, P = scales(inp, eos)
    return plo + P * np.exp(y)


def forward(theta, X, keep=False):
    p = unpack(theta)
    X = np.atleast_2d(X)
    Z1 = X @ p["W1"].T + p["b1"]
    H1 = np.tanh(Z1)
    Z2 = H1 @ p["W2"].T + p["b2"]
    H2 = np.tanh(Z2)
    y = H2 @ p["w3"] + p["b3"][0]
    if keep:
        return y, (X, H1, H2)
    return y


def loss(theta, X, t):
    y = forward(theta, X)
    return float(np.mean((y - t) ** 2))


def grad(theta, X, t):
    """Gradient of the mean squared error with respect to theta (chain rule
    through the two tanh layers)."""
    p = unpack(theta)
    y, (X, H1, H2) = forward(theta, X, keep=True)
    n = X.shape[0]
    dy = 2.0 * (y - t) / n
    g = {"w3": H2.T @ dy, "b3": np.array([dy.sum()])}
    dZ2 = np.outer(dy, p["w3"]) * (1.0 - H2 ** 2)
    g["W2"] = dZ2.T @ H1
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ p["W2"]) * (1.0 - H1 ** 2)
    g["W1"] = dZ1.T @ X
    g["b1"] = dZ1.sum(axis=0)
    return pack(g)


def adam_step(theta, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba); step counts from 1."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
