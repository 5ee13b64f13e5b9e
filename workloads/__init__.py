"""Seeded synthetic inputs shared by the CPU oracle tests and the GPU path.

This module only builds initial conditions and problem sets: grids, material
layouts, primitive fields and random Riemann-problem inputs.  It holds none of
the finite-volume method's arithmetic (no EOS inversion, fluxes, limiters,
Riemann solves or time stepping), so neither side of a parity comparison can
borrow numerics from the other through it.

Conventions
-----------
* Fields are float64 arrays of shape (6, nz, ny, nx) holding the primitive
  state (rho, u, v, w, p, phi) at cell centres; x is the fastest index, so the
  flat cell index is ``i + nx*(j + ny*k)``.
* Material 1 occupies ``phi < 0`` and material 0 occupies ``phi >= 0``.
* Random numbers come from SplitMix64 (Steele, Lea and Flood, 2014), turned
  into doubles in [0, 1) from the top 53 bits.  The draw order of every
  builder is fixed and documented in its docstring.

Physical set-up follows the paper's test families: the one-dimensional
two-material shock tube of the Riemann-problem verification section and the
shock-bubble problems of the bubble-collapse section, with the stiffened-gas
parameters of the material table the paper uses (air gamma=1.4, p_c=0; water
as stiffened gas).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "SplitMix64", "Problem", "WATER", "AIR",
    "shock_tube_1d", "shock_bubble", "bubble_cloud", "batched_shock_bubbles",
    "riemann_problem_set", "uniform_translation", "periodic_box",
    "post_shock_state", "EOS_MATERIALS", "general_eos_problem_set",
]

_MASK = (1 << 64) - 1

# (gamma, p_c) of the two stiffened gases used by every workload.
WATER = (6.12, 3.43e8)
AIR = (1.4, 0.0)

BC_TRANSMISSIVE, BC_WALL, BC_PERIODIC = 0, 1, 2


class SplitMix64:
    """SplitMix64 generator; ``uniform()`` returns doubles in [0, 1)."""

    def __init__(self, seed: int):
        self.state = int(seed) & _MASK

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def uniform(self, lo: float = 0.0, hi: float = 1.0) -> float:
        u = (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)
        return lo + (hi - lo) * u

    def log_uniform(self, lo: float, hi: float) -> float:
        return math.exp(self.uniform(math.log(lo), math.log(hi)))

    def choice(self, seq):
        return seq[int(self.uniform() * len(seq)) % len(seq)]

    def uniforms(self, n: int) -> np.ndarray:
        """n draws, vectorised (same sequence as n calls of ``uniform()``)."""
        k = np.arange(1, n + 1, dtype=np.uint64)
        with np.errstate(over="ignore"):
            z = np.uint64(self.state) + k * np.uint64(0x9E3779B97F4A7C15)
            z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
            z = z ^ (z >> np.uint64(31))
        self.state = (self.state + n * 0x9E3779B97F4A7C15) & _MASK
        return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


@dataclass
class Problem:
    """A grid, two stiffened-gas materials, boundary types, time-stepping
    parameters and the initial primitive field."""
    name: str
    n: tuple            # (nx, ny, nz)
    lo: tuple
    hi: tuple
    gamma: tuple        # (material 0, material 1)
    pc: tuple
    bc: tuple = (0, 0, 0, 0, 0, 0)   # -x,+x,-y,+y,-z,+z
    cfl: float = 0.4
    steps: int = 100
    dt_fixed: float = 0.0
    prim: np.ndarray = field(default=None, repr=False)   # (6, nz, ny, nx)
    meta: dict = field(default_factory=dict)
    # general EOS of materials 0 and 1 as (family, params) pairs (families
    # and parameter order of EOS_MATERIALS); None: the stiffened gases above
    eos: tuple = None

    @property
    def ncells(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    def dx(self):
        return tuple((self.hi[d] - self.lo[d]) / self.n[d] for d in range(3))


def _centres(n, lo, hi):
    """Cell-centre coordinate vectors along x, y, z."""
    out = []
    for d in range(3):
        h = (hi[d] - lo[d]) / n[d]
        out.append(lo[d] + (np.arange(n[d], dtype=np.float64) + 0.5) * h)
    return out


def post_shock_state(rho0: float, p0: float, p1: float, gamma: float, pc: float):
    """State behind a right-moving shock of pressure p1 running into a
    stiffened gas at rest (rho0, p0).  Returns (rho1, u1).

    Built from the three jump conditions only: the energy (Hugoniot)
    condition e1 - e0 = (p1 + p0)/2 * (1/rho0 - 1/rho1), with the
    stiffened-gas internal energy e = (p + gamma p_c)/((gamma - 1) rho), is
    solved for rho1 by bisection; mass and momentum then give
    u1 = sqrt((p1 - p0)(1/rho0 - 1/rho1)).
    """
    def e(rho, p):
        return (p + gamma * pc) / ((gamma - 1.0) * rho)

    def hug(rho1):
        return e(rho1, p1) - e(rho0, p0) - 0.5 * (p1 + p0) * (1.0 / rho0 - 1.0 / rho1)

    lo_r = rho0                       # hug(lo_r) > 0 for p1 > p0
    hi_r = rho0 * (gamma + 1.0) / (gamma - 1.0) * (1.0 - 1e-15)   # strong-shock limit
    for _ in range(200):
        mid = 0.5 * (lo_r + hi_r)
        if hug(mid) > 0.0:
            lo_r = mid
        else:
            hi_r = mid
    rho1 = 0.5 * (lo_r + hi_r)
    u1 = math.sqrt((p1 - p0) * (1.0 / rho0 - 1.0 / rho1))
    return rho1, u1


def shock_tube_1d(seed: int, nx: int = 1000, steps: int = 200, cfl: float = 0.5) -> Problem:
    """1D two-material shock tube on nx x 1 x 1 cells of width 1/nx.

    Water (stiffened gas, material 1, rho=1000) where phi = x - 0.5 < 0, air
    (material 0, rho=1) elsewhere; zero velocity; right pressure 1e5 Pa.
    Draw order: one draw, left pressure log-uniform in [1e6, 1e9] Pa.
    """
    rng = SplitMix64(seed)
    pL = rng.log_uniform(1e6, 1e9)
    h = 1.0 / nx
    n = (nx, 1, 1)
    lo, hi = (0.0, 0.0, 0.0), (1.0, h, h)
    x, _, _ = _centres(n, lo, hi)
    phi = x - 0.5
    left = phi < 0
    prim = np.zeros((6, 1, 1, nx))
    prim[0, 0, 0] = np.where(left, 1000.0, 1.0)
    prim[4, 0, 0] = np.where(left, pL, 1e5)
    prim[5, 0, 0] = phi
    return Problem("shock_tube_1d", n, lo, hi, gamma=(AIR[0], WATER[0]), pc=(AIR[1], WATER[1]),
                   cfl=cfl, steps=steps, prim=prim, meta={"seed": seed, "pL": pL})


def _fill_bubble_field(n, lo, hi, centres, radii, amb, slab_x, slab_state, chunk_planes=16):
    """Primitive field for water with air bubbles and a high-pressure slab.

    phi = min_k(|x - c_k| - r_k); air (rho=1, p=1e5) where phi < 0.
    ``slab_state`` = (rho, u, p) of the water for x < slab_x.
    """
    nx, ny, nz = n
    xs, ys, zs = _centres(n, lo, hi)
    prim = np.empty((6, nz, ny, nx))
    X = xs[None, None, :]
    for k0 in range(0, nz, chunk_planes):
        k1 = min(nz, k0 + chunk_planes)
        Z = zs[k0:k1, None, None]
        Y = ys[None, :, None]
        phi = np.full((k1 - k0, ny, nx), np.inf)
        for (cx, cy, cz), r in zip(centres, radii):
            d = np.sqrt((X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2) - r
            np.minimum(phi, d, out=phi)
        air = phi < 0
        slab = np.broadcast_to(X < slab_x, phi.shape) & ~air
        rho = np.where(air, amb["rho_air"], amb["rho_water"])
        p = np.full(phi.shape, amb["p"])
        u = np.zeros(phi.shape)
        rho = np.where(slab, slab_state[0], rho)
        u = np.where(slab, slab_state[1], u)
        p = np.where(slab, slab_state[2], p)
        prim[0, k0:k1] = rho
        prim[1, k0:k1] = u
        prim[2, k0:k1] = 0.0
        prim[3, k0:k1] = 0.0
        prim[4, k0:k1] = p
        prim[5, k0:k1] = phi
    return prim


_AMBIENT = {"rho_air": 1.0, "rho_water": 1000.0, "p": 1e5}


def shock_bubble(seed: int, n: int = 128, steps: int = 100, cfl: float = 0.4,
                 radius: float = 0.15, p_shock: float = 1e8, shock_x: float = 0.1,
                 nxyz=None, centre_x=None, bc=(0, 0, 0, 0, 0, 0)) -> Problem:
    """Air bubble in water hit by a planar shock, unit box, transmissive
    unless ``bc`` says otherwise.

    Bubble (material 1) of the given radius at (0.5,0.5,0.5) + U(-0.05,0.05)^3
    (x of the centre = ``centre_x`` when given, e.g. a bubble next to a rigid
    wall); water (material 0) at 1e5 Pa elsewhere; for x < shock_x the water
    takes the post-shock state of pressure p_shock moving in +x.
    Draw order: three draws, jitter of the centre along x, y, z (drawn also
    when centre_x replaces the first).
    """
    rng = SplitMix64(seed)
    c = tuple(0.5 + rng.uniform(-0.05, 0.05) for _ in range(3))
    if centre_x is not None:
        c = (float(centre_x), c[1], c[2])
    dims = tuple(nxyz) if nxyz is not None else (n, n, n)
    lo, hi = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)
    rho1, u1 = post_shock_state(1000.0, 1e5, p_shock, *WATER)
    prim = _fill_bubble_field(dims, lo, hi, [c], [radius], _AMBIENT, shock_x, (rho1, u1, p_shock))
    return Problem("shock_bubble", dims, lo, hi, gamma=(WATER[0], AIR[0]), pc=(WATER[1], AIR[1]),
                   bc=tuple(bc), cfl=cfl, steps=steps, prim=prim,
                   meta={"seed": seed, "centre": c, "radius": radius, "p_shock": p_shock,
                         "post_shock": (rho1, u1)})


def bubble_cloud(seed: int = 0, n: int = 384, nbubbles: int = 32, steps: int = 50,
                 cfl: float = 0.4, rmin: float = 0.02, rmax: float = 0.06,
                 slab_x: float = 0.05, p_slab: float = 5e7, max_tries: int = 100000) -> Problem:
    """Cloud of non-overlapping air bubbles in water with a high-pressure slab.

    Bubble k: radius r ~ U[rmin, rmax], then centre x ~ U[slab_x + r + 2h, 1 - r],
    y, z ~ U[r, 1 - r] (draw order r, x, y, z), rejected and redrawn while it
    comes closer than r_a + r_b + 2h to an accepted bubble.  The slab x < slab_x
    is water at rest with p = p_slab; ambient pressure 1e5 Pa.
    """
    rng = SplitMix64(seed)
    h = 1.0 / n
    centres, radii = [], []
    tries = 0
    while len(centres) < nbubbles:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("bubble_cloud: could not place all bubbles")
        r = rng.uniform(rmin, rmax)
        cx = rng.uniform(slab_x + r + 2 * h, 1.0 - r)
        cy = rng.uniform(r, 1.0 - r)
        cz = rng.uniform(r, 1.0 - r)
        ok = all(math.dist((cx, cy, cz), c2) >= r + r2 + 2 * h for c2, r2 in zip(centres, radii))
        if ok:
            centres.append((cx, cy, cz))
            radii.append(r)
    dims = (n, n, n)
    lo, hi = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)
    prim = _fill_bubble_field(dims, lo, hi, centres, radii, _AMBIENT, slab_x, (1000.0, 0.0, p_slab))
    return Problem("bubble_cloud", dims, lo, hi, gamma=(WATER[0], AIR[0]), pc=(WATER[1], AIR[1]),
                   cfl=cfl, steps=steps, prim=prim,
                   meta={"seed": seed, "centres": centres, "radii": radii})


def batched_shock_bubbles(seed: int = 0, runs: int = 64, steps: int = 100, cfl: float = 0.4,
                          edges=(32, 48, 64, 96, 128), build_fields: bool = True):
    """Independent shock-bubble runs of uneven grid sizes.

    Run k uses SplitMix64(seed*runs + k) and draws, in order: nx, ny, nz from
    ``edges``, radius ~ U[0.1, 0.25], shock pressure log-uniform in [1e7, 1e9],
    then the three centre jitters of ``shock_bubble``.
    """
    out = []
    for k in range(runs):
        rng = SplitMix64(seed * runs + k)
        dims = tuple(rng.choice(edges) for _ in range(3))
        r = rng.uniform(0.1, 0.25)
        ps = rng.log_uniform(1e7, 1e9)
        c = tuple(0.5 + rng.uniform(-0.05, 0.05) for _ in range(3))
        lo, hi = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)
        rho1, u1 = post_shock_state(1000.0, 1e5, ps, *WATER)
        prim = None
        if build_fields:
            prim = _fill_bubble_field(dims, lo, hi, [c], [r], _AMBIENT, 0.1, (rho1, u1, ps))
        out.append(Problem(f"batched_{k}", dims, lo, hi, gamma=(WATER[0], AIR[0]),
                           pc=(WATER[1], AIR[1]), cfl=cfl, steps=steps, prim=prim,
                           meta={"seed": seed * runs + k, "radius": r, "p_shock": ps,
                                 "centre": c}))
    return out


def uniform_translation(n: int = 200, axis: int = 0, velocity: float = 50.0,
                        pressure: float = 1e5, steps: int = 50, cfl: float = 0.5,
                        periodic: bool = True) -> Problem:
    """Water slab (material 1) and air (material 0) in uniform velocity and
    pressure along one axis: a two-material contact that must translate with
    u and p staying uniform.  Water occupies |s - 0.5| < 0.25 of the unit
    line s along ``axis``."""
    dims = [1, 1, 1]
    dims[axis] = n
    h = 1.0 / n
    hi = [h, h, h]
    hi[axis] = 1.0
    lo = (0.0, 0.0, 0.0)
    cs = _centres(dims, lo, hi)
    s = cs[axis]
    phi = np.abs(s - 0.5) - 0.25
    water = phi < 0
    prim = np.zeros((6, dims[2], dims[1], dims[0]))
    shape = [1, 1, 1]
    shape[2 - axis] = n
    prim[0] = np.where(water, 1000.0, 1.0).reshape(shape)
    prim[1 + axis] = velocity
    prim[4] = pressure
    prim[5] = phi.reshape(shape)
    bc = [BC_PERIODIC if periodic else BC_TRANSMISSIVE] * 6
    return Problem("uniform_translation", tuple(dims), lo, tuple(hi), gamma=(AIR[0], WATER[0]),
                   pc=(AIR[1], WATER[1]), bc=tuple(bc), cfl=cfl, steps=steps, prim=prim,
                   meta={"axis": axis, "velocity": velocity})


def periodic_box(seed: int, n=(16, 12, 10), steps: int = 20, cfl: float = 0.4,
                 material: int = 0, bc: int = BC_PERIODIC) -> Problem:
    """Single-material box with smooth random-phase perturbations.

    Draw order: 3 phases for each of rho, u, v, w, p (15 draws); phi > 0
    everywhere (material 0) unless ``material`` is 1, then phi < 0.
    """
    rng = SplitMix64(seed)
    lo, hi = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)
    xs, ys, zs = _centres(n, lo, hi)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    prim = np.empty((6, n[2], n[1], n[0]))
    base = [(1.0, 0.2), (30.0, 60.0), (-20.0, 60.0), (10.0, 60.0), (1e5, 3e4)]
    if material == 1:
        base = [(1000.0, 50.0), (5.0, 10.0), (-3.0, 10.0), (2.0, 10.0), (1e6, 3e5)]
    for v, (m, a) in enumerate(base):
        ph = [rng.uniform(0, 2 * math.pi) for _ in range(3)]
        prim[v] = m + a * (np.sin(2 * math.pi * X + ph[0]) * np.cos(2 * math.pi * Y + ph[1])
                           * np.sin(2 * math.pi * Z + ph[2]))
    prim[5] = 1.0 if material == 0 else -1.0
    return Problem("periodic_box", tuple(n), lo, hi, gamma=(AIR[0], WATER[0]), pc=(AIR[1], WATER[1]),
                   bc=(bc,) * 6, cfl=cfl, steps=steps, prim=prim, meta={"seed": seed})


def riemann_problem_set(seed: int, n: int, zero_du_fraction: float = 0.5):
    """Random two-material stiffened-gas Riemann problems (water/air pairs).

    Returns (inp, eos): inp[n, 6] = (rho_L, u_L, p_L, rho_R, u_R, p_R) and
    eos[n, 4] = (gamma_L, pc_L, gamma_R, pc_R).

    Per problem, nine draws in this order: EOS order (water on the left if
    U < 0.5); low pressure log-uniform in [1e4, 1e6] Pa; pressure ratio
    log-uniform in [1, 1e4]; high-pressure side (left if U < 0.5); water
    density log-uniform in [900, 1100]; water/air density ratio log-uniform
    in [1, 1e3]; velocity-jump switch (zero jump if U < zero_du_fraction);
    velocity-jump factor U(-0.2, 0.2); one spare draw.  The jump is
    du = factor * (a_L + a_R)/2 with a_K = sqrt(gamma_K (p_K + pc_K)/rho_K),
    the acoustic speed of side K, used here only to scale the input
    distribution; u_L = -du/2, u_R = +du/2.  Problems without an admissible
    star pressure (vacuum) are the caller's to discard.
    """
    rng = SplitMix64(seed)
    U = rng.uniforms(n * 9).reshape(n, 9)
    water_left = U[:, 0] < 0.5
    p_lo = np.exp(np.log(1e4) + U[:, 1] * (np.log(1e6) - np.log(1e4)))
    p_hi = p_lo * np.exp(U[:, 2] * np.log(1e4))
    p_hi_left = U[:, 3] < 0.5
    r_w = np.exp(np.log(900.0) + U[:, 4] * (np.log(1100.0) - np.log(900.0)))
    r_a = r_w / np.exp(U[:, 5] * np.log(1e3))
    du_on = U[:, 6] >= zero_du_fraction
    inp = np.empty((n, 6))
    eos = np.empty((n, 4))
    inp[:, 0] = np.where(water_left, r_w, r_a)
    inp[:, 3] = np.where(water_left, r_a, r_w)
    inp[:, 2] = np.where(p_hi_left, p_hi, p_lo)
    inp[:, 5] = np.where(p_hi_left, p_lo, p_hi)
    eos[:, 0] = np.where(water_left, WATER[0], AIR[0])
    eos[:, 1] = np.where(water_left, WATER[1], AIR[1])
    eos[:, 2] = np.where(water_left, AIR[0], WATER[0])
    eos[:, 3] = np.where(water_left, AIR[1], WATER[1])
    aL = np.sqrt(eos[:, 0] * (inp[:, 2] + eos[:, 1]) / inp[:, 0])
    aR = np.sqrt(eos[:, 2] * (inp[:, 5] + eos[:, 3]) / inp[:, 3])
    du = np.where(du_on, (-0.2 + 0.4 * U[:, 7]) * 0.5 * (aL + aR), 0.0)
    inp[:, 1] = -0.5 * du
    inp[:, 4] = 0.5 * du
    return inp, eos


# Materials of the general-EOS Riemann problems, as (family, parameters) in
# the layout of the library's material table (0 Noble-Abel stiffened gas:
# gamma, p_c, b, e_c; 1 Mie-Grueneisen: rho_0, c_0, Gamma_0, s, e_0, eta_min;
# 2 JWL: omega, A_1, A_2, R_1, R_2, rho_0; SI units), the kinds of materials
# of the paper's Riemann-problem and impact examples, with the sampling
# ranges of their states: density (lo, hi, log?), pressure (lo, hi, log?) and
# a nominal sound speed that only scales the velocity jumps.
EOS_MATERIALS = {
    "air": (0, [1.4, 0.0, 0.0, 0.0], (0.5, 50.0, True), (3e4, 3e7, True), 340.0),
    "gas_nasg": (0, [1.6, 0.0, 2.0e-4, 3.0e5], (0.5, 50.0, True), (3e4, 3e7, True), 400.0),
    "water_sg": (0, [6.12, 3.43e8, 0.0, 0.0], (950.0, 1100.0, False), (1e5, 1e9, True), 1500.0),
    "water_nasg": (0, [1.19, 7.028e8, 6.61e-4, -1.177788e6], (950.0, 1100.0, False), (1e5, 1e9, True), 1500.0),
    "glass": (1, [2204.0, 2220.0, 0.65, 1.61, 0.0, -0.5], (2193.0, 2336.0, False), (0.0, 5e9, False), 2220.0),
    "copper": (1, [8930.0, 3940.0, 2.0, 1.49, 0.0, -0.1], (8885.0, 9466.0, False), (0.0, 5e9, False), 3940.0),
    "tantalum": (1, [16650.0, 3414.0, 1.6, 1.2, 1.0e4, -0.05], (16567.0, 17649.0, False), (0.0, 5e9, False),
                 3414.0),
    "tnt": (2, [0.3, 3.712e11, 3.231e9, 4.15, 0.95, 1630.0], (300.0, 1700.0, False), (1e8, 2e10, True), 3000.0),
}

# Material pairs of the general-EOS problem sets: gas / solid, liquid / gas,
# solid / solid, detonation products / gas, liquid and solid.
EOS_PAIRS = [("air", "glass"), ("water_nasg", "gas_nasg"), ("copper", "tantalum"), ("tnt", "air"),
             ("tnt", "water_sg"), ("glass", "water_nasg"), ("copper", "tnt"), ("water_sg", "air")]


def general_eos_problem_set(seed: int, n: int, pairs=None):
    """Random two-material Riemann problems with general EOS.

    Returns (inp [6, n], mat [2, n] int32, materials, names): inp rows are
    (rho_L, u_L, p_L, rho_R, u_R, p_R), mat the left and right indices into
    materials = [(family, params)] (in the order of ``names``).

    Per problem, seven draws in this order: the pair (uniform over
    ``pairs``, default EOS_PAIRS); which member goes left (the first if
    U < 0.5); left density; left pressure; right density; right pressure
    (each uniform or log-uniform over the material's range); the velocity
    jump factor U(-1, 0.6), times the smaller nominal sound speed of the
    two: du = u_R - u_L > 0 separates the sides (rarefactions, and
    cavitation when too fast), du < 0 compresses them (shocks);
    u_L = -du/2, u_R = +du/2.
    """
    pairs = list(pairs or EOS_PAIRS)
    names = sorted({m for pr in pairs for m in pr})
    index = {m: i for i, m in enumerate(names)}
    materials = [(EOS_MATERIALS[m][0], list(EOS_MATERIALS[m][1])) for m in names]
    rng = SplitMix64(seed)
    U = rng.uniforms(n * 7).reshape(n, 7)

    def draw(u, rng_spec):
        lo, hi, log = rng_spec
        return np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo))) if log else lo + u * (hi - lo)

    inp = np.empty((6, n))
    mat = np.empty((2, n), dtype=np.int32)
    k = np.minimum((U[:, 0] * len(pairs)).astype(np.int64), len(pairs) - 1)
    for j, (a, b) in enumerate(pairs):
        sel = k == j
        first_left = U[sel, 1] < 0.5
        left = np.where(first_left, index[a], index[b])
        right = np.where(first_left, index[b], index[a])
        mat[0, sel], mat[1, sel] = left, right
        for side, (ur, up, row) in enumerate(((2, 3, 0), (4, 5, 3))):
            ids = left if side == 0 else right
            for m in (a, b):
                t = ids == index[m]
                spec = EOS_MATERIALS[m]
                where = np.flatnonzero(sel)[t]
                inp[row, where] = draw(U[where, ur], spec[2])
                inp[row + 2, where] = draw(U[where, up], spec[3])
        cmin = min(EOS_MATERIALS[a][4], EOS_MATERIALS[b][4])
        du = (-1.0 + 1.6 * U[sel, 6]) * cmin
        inp[1, sel] = -0.5 * du
        inp[4, sel] = 0.5 * du
    return inp, mat, materials, names


def _eos_of(name):
    fam, prm = EOS_MATERIALS[name][0], list(EOS_MATERIALS[name][1])
    return fam, prm + [0.0] * (7 - len(prm))


def eos_shock_tube_1d(left: str, right: str, left_state, right_state, nx: int = 200, steps: int = 60,
                      cfl: float = 0.5, x0: float = 0.5) -> Problem:
    """1D two-material Riemann problem with general EOS on nx x 1 x 1 cells
    of the unit line: material ``left`` (material 1, phi = x - x0 < 0) with
    primitive state (rho, u, p) left_state, material ``right`` (material 0)
    with right_state; transmissive ends."""
    h = 1.0 / nx
    n = (nx, 1, 1)
    lo, hi = (0.0, 0.0, 0.0), (1.0, h, h)
    x, _, _ = _centres(n, lo, hi)
    phi = x - x0
    L = phi < 0
    prim = np.zeros((6, 1, 1, nx))
    for v, k in ((0, 0), (1, 1), (4, 2)):
        prim[v, 0, 0] = np.where(L, left_state[k], right_state[k])
    prim[5, 0, 0] = phi
    return Problem("eos_shock_tube_1d", n, lo, hi, gamma=(1.4, 1.4), pc=(0.0, 0.0), cfl=cfl, steps=steps,
                   prim=prim, meta={"left": left, "right": right, "x0": x0},
                   eos=(_eos_of(right), _eos_of(left)))


def eos_charge(seed: int, n=(12, 11, 10), inner: str = "tnt", outer: str = "water_nasg",
               p_inner: float = 5e9, rho_inner: float = 1630.0, rho_outer: float = 1000.0,
               p_outer: float = 1e5, radius: float = 0.28, steps: int = 10, cfl: float = 0.4) -> Problem:
    """3D general-EOS problem: a sphere of material ``inner`` (material 1)
    at high pressure in material ``outer`` at rest (an underwater charge of
    detonation products when inner is JWL), on the unit box with
    transmissive boundaries.  Draw order: three centre offsets U(-0.05,
    0.05); then one relative density perturbation U(-0.02, 0.02) per cell
    of the outer material, in cell order (x fastest)."""
    rng = SplitMix64(seed)
    c = [0.5 + rng.uniform(-0.05, 0.05) for _ in range(3)]
    lo, hi = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)
    xs, ys, zs = _centres(n, lo, hi)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    phi = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) - radius
    jit = 1.0 + rng.uniforms(n[0] * n[1] * n[2]).reshape(n[2], n[1], n[0]) * 0.04 - 0.02
    inside = phi < 0
    prim = np.zeros((6, n[2], n[1], n[0]))
    prim[0] = np.where(inside, rho_inner, rho_outer * jit)
    prim[4] = np.where(inside, p_inner, p_outer)
    prim[5] = phi
    return Problem("eos_charge", tuple(n), lo, hi, gamma=(1.4, 1.4), pc=(0.0, 0.0), cfl=cfl, steps=steps,
                   prim=prim, meta={"seed": seed, "inner": inner, "outer": outer},
                   eos=(_eos_of(outer), _eos_of(inner)))
