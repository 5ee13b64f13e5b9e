"""CPU oracle of the two-material finite-volume step (TEST INFRASTRUCTURE).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It is the plain FP64 reference the GPU library is
checked against and shares no code with it.

Contents
--------
* ``m2c_oracle.c`` -- the scheme in plain C (built into ``liboracle.so``),
  wrapped here with ctypes: :class:`OracleSim` and point functions.
* ``exact_riemann.py`` -- an independent derivative-free (bisection) solver of
  the two-material stiffened-gas Riemann problem in high precision, plus the
  self-similar exact solution used to pin the scheme.
* ``mlp_ref.py`` -- FP64 features, forward, backward and Adam of the learned
  star-pressure guess.
* ``riemann_eos.py`` -- the two-material Riemann problem with a general EOS
  on each side (Noble-Abel stiffened gas, Mie-Grueneisen, JWL): bracketed
  roots and a DOP853 integration of the isentropes.
* ``reinit.py`` -- level-set reinitialization towards a signed distance
  (upwind Godunov |grad phi|, smoothed sign, fixed first layer, optional
  narrow band), in numpy.

Parity status: every part is pinned by the tests under
``tests/test_oracle_*.py``.  The zero-slope rule next to an interface and the
phase-update rule are readings of under-specified steps; the oracle's
implementation of each is pinned by a 30-digit hand-written forward-Euler
step and a single-flip case checked against the independent exact solver
(``tests/test_oracle_bruteforce.py``), but the choice of rule itself is a
reading, not something the paper fixes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "m2c_oracle.c")

OK, ERR_ARG, ERR_NONPHYSICAL, ERR_RIEMANN, ERR_NOMEM = 0, -1, -2, -3, -7


_SO_OMP = os.path.join(_HERE, "liboracle_omp.so")


def build(force: bool = True, extra_flags=(), openmp: bool = False):
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA); with
    ``openmp`` the all-core build (same source, -fopenmp), which gives
    bit-identical results."""
    so = _SO_OMP if openmp else _SO
    hdr = os.path.join(_HERE, "m2c_oracle.h")
    if (not force and os.path.exists(so)
            and os.path.getmtime(so) >= max(os.path.getmtime(_SRC), os.path.getmtime(hdr))):
        return so
    tmp = so + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
           *(["-fopenmp"] if openmp else []), *extra_flags, "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, so)
    return so


def build_variant(path: str, defines=()):
    """Build a separate copy of the oracle (e.g. with a planted mistake for a
    test that shows the pins catch it)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
           *[f"-D{d}" for d in defines], "-o", path, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return path


class EosC(C.Structure):
    _fields_ = [("family", C.c_int32), ("reserved", C.c_int32), ("prm", C.c_double * 7)]


# star state of one two-material Riemann problem: (ml, mr, in[6], out[4]) -> rc
RIEMANN_FN = C.CFUNCTYPE(C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double))


class Cfg(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("gamma", C.c_double * 2), ("pc", C.c_double * 2),
                ("bc", C.c_int32 * 6), ("alpha", C.c_double), ("rk_order", C.c_int32),
                ("cfl", C.c_double), ("dt_fixed", C.c_double), ("rtol", C.c_double),
                ("maxit", C.c_int32), ("limiter", C.c_int32), ("limiter_k", C.c_int32),
                ("flux", C.c_int32), ("ls_band", C.c_double), ("eos_general", C.c_int32),
                ("eos", EosC * 2), ("riemann", RIEMANN_FN)]


def general_eos_riemann(eos_pair):
    """The interface solver of a general-EOS run: the star state from
    ``riemann_eos`` (bracketed roots, adaptive isentropes) for the two
    materials (family, params) of eos_pair."""
    from . import riemann_eos as RE
    mats = [RE.make_eos(f, prm) for f, prm in eos_pair]

    def solve(ml, mr, inp, out):
        try:
            L = RE.Side(mats[ml], inp[0], inp[1], inp[2])
            R = RE.Side(mats[mr], inp[3], inp[4], inp[5])
            res = RE.star_state(L, R)
        except (ValueError, RuntimeError, ZeroDivisionError, OverflowError):
            return ERR_RIEMANN
        if not all(np.isfinite(res)):
            return ERR_RIEMANN
        for k in range(4):
            out[k] = res[k]
        return OK

    return RIEMANN_FN(solve)


LIM_MC, LIM_VA, LIM_VA_MOD = 0, 1, 2
FLUX_HLLC, FLUX_LLF = 0, 1


class Stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("t", C.c_double), ("dt_last", C.c_double),
                ("iface_faces_last", C.c_int64), ("newton_iters", C.c_int64),
                ("riemann_solves", C.c_int64), ("bisection_fallbacks", C.c_int64),
                ("flips", C.c_int64), ("orphans", C.c_int64), ("err_cell", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = np.ctypeslib.ndpointer
_D = _P(dtype=np.float64, flags="C_CONTIGUOUS")
_U8 = _P(dtype=np.uint8, flags="C_CONTIGUOUS")
_I32 = _P(dtype=np.int32, flags="C_CONTIGUOUS")


def load(path: str | None = None):
    path = path or _SO
    if path == _SO and not os.path.exists(_SO):
        build()
    lib = C.CDLL(path)
    lib.ora_create.restype = C.c_void_p
    lib.ora_create.argtypes = [C.POINTER(Cfg)]
    lib.ora_destroy.argtypes = [C.c_void_p]
    lib.ora_set_prim.argtypes = [C.c_void_p, _D]
    lib.ora_get_prim.argtypes = [C.c_void_p, _D, C.c_void_p]
    lib.ora_set_cons.argtypes = [C.c_void_p, _D]
    lib.ora_get_cons.argtypes = [C.c_void_p, _D]
    lib.ora_step.argtypes = [C.c_void_p, C.c_int32]
    lib.ora_step_dt.argtypes = [C.c_void_p, C.c_int32, C.c_double]
    lib.ora_dt.restype = C.c_double
    lib.ora_dt.argtypes = [C.c_void_p]
    lib.ora_get_stats.argtypes = [C.c_void_p, C.POINTER(Stats)]
    lib.ora_interface_faces.restype = C.c_int64
    lib.ora_interface_faces.argtypes = [C.c_void_p, C.c_void_p, C.c_int64]
    lib.ora_prim_to_cons.argtypes = [_D, C.c_double, C.c_double, _D]
    lib.ora_cons_to_prim.argtypes = [_D, C.c_double, C.c_double, _D]
    lib.ora_sound_speed.restype = C.c_double
    lib.ora_sound_speed.argtypes = [C.c_double] * 4
    lib.ora_mc_slope.restype = C.c_double
    lib.ora_mc_slope.argtypes = [C.c_double, C.c_double, C.c_double]
    lib.ora_hllc.argtypes = [_D, _D, C.c_double, C.c_double, _D]
    lib.ora_llf.argtypes = [_D, _D, C.c_double, C.c_double, _D]
    lib.ora_va_slope.restype = C.c_double
    lib.ora_va_slope.argtypes = [C.c_double, C.c_double, C.c_int32, C.c_int32]
    lib.ora_riemann.restype = C.c_int
    lib.ora_riemann.argtypes = [_D, _D, C.c_double, C.c_int32, _D, C.POINTER(C.c_int32)]
    lib.ora_riemann_many.restype = C.c_int64
    lib.ora_riemann_many.argtypes = [C.c_int64, _D, _D, C.c_double, C.c_int32, _D, C.c_void_p]
    lib.ora_ls_derivative.restype = C.c_double
    lib.ora_ls_derivative.argtypes = [_D, C.c_double, C.c_double]
    for name in ("ora_eos_p", "ora_eos_e", "ora_eos_c2"):
        getattr(lib, name).restype = C.c_double
        getattr(lib, name).argtypes = [C.POINTER(EosC), C.c_double, C.c_double]
    lib.ora_eos_floor.restype = C.c_double
    lib.ora_eos_floor.argtypes = [C.POINTER(EosC)]
    lib.ora_num_threads.restype = C.c_int32
    lib.ora_num_threads.argtypes = []
    return lib


_lib = None
_lib_omp = None


def lib():
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


def lib_openmp():
    """The all-core (OpenMP) build; threads from OMP_NUM_THREADS."""
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(_SO_OMP):
            build(openmp=True)
        _lib_omp = load(_SO_OMP)
    return _lib_omp


def make_cfg(problem, alpha=1.2, rk_order=2, rtol=1e-12, maxit=50, limiter=LIM_MC, limiter_k=2,
             flux=FLUX_HLLC, ls_band=0.0):
    """The oracle configuration of a problem; a problem with an ``eos``
    attribute (two (family, params) pairs) runs with those general EOS."""
    c = Cfg()
    c.nx, c.ny, c.nz = problem.n
    for d in range(3):
        c.lo[d] = problem.lo[d]
        c.hi[d] = problem.hi[d]
    for m in range(2):
        c.gamma[m] = problem.gamma[m]
        c.pc[m] = problem.pc[m]
    for f in range(6):
        c.bc[f] = problem.bc[f]
    c.alpha = alpha
    c.rk_order = rk_order
    c.cfl = problem.cfl
    c.dt_fixed = problem.dt_fixed
    c.rtol = rtol
    c.maxit = maxit
    c.limiter = limiter
    c.limiter_k = limiter_k
    c.flux = flux
    c.ls_band = ls_band
    eos = getattr(problem, "eos", None)
    if eos is not None:
        c.eos_general = 1
        for m in range(2):
            c.eos[m] = eos_struct(*eos[m])
        c.riemann = general_eos_riemann(eos)
    return c


def eos_struct(family, params):
    e = EosC()
    e.family = family
    for k, v in enumerate(params):
        e.prm[k] = v
    return e


class OracleSim:
    """The oracle on one grid."""

    def __init__(self, problem, lib_handle=None, **kw):
        self.lib = lib_handle or lib()
        self.problem = problem
        self.cfg = make_cfg(problem, **kw)
        self.h = self.lib.ora_create(C.byref(self.cfg))
        if not self.h:
            raise MemoryError("ora_create failed")
        self.N = problem.ncells
        if problem.prim is not None:
            rc = self.set_prim(problem.prim)
            if rc != OK:
                raise ValueError(f"ora_set_prim rc={rc}")

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.ora_destroy(self.h)
            self.h = None

    def set_prim(self, prim):
        return self.lib.ora_set_prim(self.h, np.ascontiguousarray(prim, dtype=np.float64).reshape(-1))

    def set_cons(self, w6):
        return self.lib.ora_set_cons(self.h, np.ascontiguousarray(w6, dtype=np.float64).reshape(-1))

    def prim(self):
        out = np.empty(6 * self.N)
        chi = np.empty(self.N, dtype=np.uint8)
        self.lib.ora_get_prim(self.h, out, chi.ctypes.data)
        nx, ny, nz = self.problem.n
        return out.reshape(6, nz, ny, nx), chi.reshape(nz, ny, nx)

    def cons(self):
        out = np.empty(6 * self.N)
        self.lib.ora_get_cons(self.h, out)
        nx, ny, nz = self.problem.n
        return out.reshape(6, nz, ny, nx)

    def step(self, n=1):
        return self.lib.ora_step(self.h, n)

    def step_dt(self, n, dt):
        return self.lib.ora_step_dt(self.h, n, dt)

    def dt(self):
        return self.lib.ora_dt(self.h)

    def stats(self):
        s = Stats()
        self.lib.ora_get_stats(self.h, C.byref(s))
        return s.as_dict()

    def interface_faces(self):
        n = self.lib.ora_interface_faces(self.h, None, 0)
        out = np.empty(max(n, 1), dtype=np.int32)
        self.lib.ora_interface_faces(self.h, out.ctypes.data, n)
        return out[:n]


# ---- point-function conveniences ------------------------------------------

def hllc(qL, qR, gamma, pc):
    F = np.empty(5)
    lib().ora_hllc(np.asarray(qL, dtype=np.float64), np.asarray(qR, dtype=np.float64),
                   gamma, pc, F)
    return F


def llf(qL, qR, gamma, pc):
    F = np.empty(5)
    lib().ora_llf(np.asarray(qL, dtype=np.float64), np.asarray(qR, dtype=np.float64), gamma, pc, F)
    return F


def va_slope(dm, dp, k=2, modified=False):
    return lib().ora_va_slope(dm, dp, k, 1 if modified else 0)


def riemann(inp, eos, rtol=1e-12, maxit=50):
    """Returns (rc, (p*, u*, rho*_L, rho*_R), iterations)."""
    out = np.empty(4)
    it = C.c_int32(0)
    rc = lib().ora_riemann(np.asarray(inp, dtype=np.float64), np.asarray(eos, dtype=np.float64),
                           rtol, maxit, out, C.byref(it))
    return rc, out, it.value


def riemann_many(inp, eos, rtol=1e-12, maxit=50):
    """Star states of many problems: inp [n,6], eos [n,4] -> (out [n,4],
    iters [n], number without an admissible root)."""
    inp = np.ascontiguousarray(inp, dtype=np.float64)
    eos = np.ascontiguousarray(eos, dtype=np.float64)
    n = inp.shape[0]
    out = np.empty((n, 4))
    it = np.empty(n, dtype=np.int32)
    bad = lib().ora_riemann_many(n, inp.reshape(-1), eos.reshape(-1), rtol, maxit, out.reshape(-1),
                                 it.ctypes.data)
    return out, it, int(bad)


def sound_speed(rho, p, gamma, pc):
    return lib().ora_sound_speed(rho, p, gamma, pc)


def mc_slope(dm, dp, alpha=1.2):
    return lib().ora_mc_slope(dm, dp, alpha)


def prim_to_cons(q, gamma, pc):
    w = np.empty(5)
    lib().ora_prim_to_cons(np.asarray(q, dtype=np.float64), gamma, pc, w)
    return w


def cons_to_prim(w, gamma, pc):
    q = np.empty(5)
    lib().ora_cons_to_prim(np.asarray(w, dtype=np.float64), gamma, pc, q)
    return q


def eos_point(family, params, rho, x, what):
    """General EOS point function of the C oracle: what = "p" (x = e),
    "e" or "c2" (x = p)."""
    e = eos_struct(family, params)
    return getattr(lib(), "ora_eos_" + what)(C.byref(e), rho, x)


def eos_floor(family, params):
    e = eos_struct(family, params)
    return lib().ora_eos_floor(C.byref(e))


def ls_derivative(f5, v, h):
    return lib().ora_ls_derivative(np.asarray(f5, dtype=np.float64), v, h)
