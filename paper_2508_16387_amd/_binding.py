"""ctypes declarations of the C ABI (``include/m2c.h``) and a small wrapper.

Argument marshalling only: no arithmetic of the method happens here.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# M2C_LIBRARY may name another build of the same library (tuning runs).
_LIB_PATH = os.environ.get("M2C_LIBRARY") or os.path.join(_HERE, "libm2c.so")

M2C_OK, M2C_ERR_ARG, M2C_ERR_NONPHYSICAL, M2C_ERR_RIEMANN = 0, -1, -2, -3
M2C_ERR_DEVICE, M2C_ERR_STATE, M2C_ERR_UNIMPLEMENTED, M2C_ERR_NOMEM = -4, -5, -6, -7
M2C_BC_TRANSMISSIVE, M2C_BC_WALL, M2C_BC_PERIODIC = 0, 1, 2
M2C_PREC_FP64, M2C_PREC_MIXED = 0, 1
M2C_GUESS_ACOUSTIC, M2C_GUESS_MLP = 0, 1
M2C_LIM_MC, M2C_LIM_VAN_ALBADA, M2C_LIM_VAN_ALBADA_MOD = 0, 1, 2
M2C_FLUX_HLLC, M2C_FLUX_LLF = 0, 1

# Every symbol the header declares (checked by the CPU test suite).
EXPORTS = [
    "m2c_config_default", "m2c_create", "m2c_destroy", "m2c_last_error", "m2c_strerror",
    "m2c_set_stream", "m2c_set_state", "m2c_set_state_device", "m2c_get_state",
    "m2c_get_state_device", "m2c_get_conserved", "m2c_set_conserved", "m2c_step", "m2c_step_dt",
    "m2c_get_stats", "m2c_reset_stats", "m2c_set_profiling", "m2c_interface_faces",
    "m2c_eval_hllc", "m2c_riemann_solve", "m2c_validate_config", "m2c_autotune", "m2c_get_tile",
    "m2c_batch_create", "m2c_batch_destroy", "m2c_batch_last_error", "m2c_batch_size",
    "m2c_batch_set_state", "m2c_batch_get_state", "m2c_batch_get_conserved", "m2c_batch_step",
    "m2c_batch_get_stats", "m2c_batch_set_tile", "m2c_batch_get_tile", "m2c_batch_autotune",
    "m2c_train_opts_default", "m2c_mlp_create", "m2c_mlp_destroy", "m2c_mlp_get_params", "m2c_mlp_features",
    "m2c_mlp_forward", "m2c_mlp_grad", "m2c_mlp_train", "m2c_riemann_solve_learned", "m2c_set_guess",
    "m2c_riemann_solve_learned_noalloc",
    "m2c_riemann_solve_eos", "m2c_eos_eval", "m2c_reinit", "m2c_reinit_workspace", "m2c_reinit_field",
    "m2c_mlp_features_eos", "m2c_riemann_solve_eos_learned",
]
_NO_STATUS = ("m2c_config_default", "m2c_destroy", "m2c_last_error", "m2c_strerror", "m2c_batch_destroy",
              "m2c_batch_last_error", "m2c_train_opts_default", "m2c_mlp_destroy")
NPARAM = 4801


class Eos(C.Structure):
    """One material of the general-EOS entry points: family and up to seven
    parameters (NASG: gamma, p_c, b, e_c; MG: rho_0, c_0, Gamma_0, s, e_0,
    eta_min; JWL: omega, A_1, A_2, R_1, R_2, rho_0)."""
    _fields_ = [("family", C.c_int32), ("reserved", C.c_int32), ("prm", C.c_double * 7)]


class Config(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("gamma", C.c_double * 2), ("pc", C.c_double * 2), ("bc", C.c_int32 * 6),
                ("limiter_alpha", C.c_double), ("rk_order", C.c_int32), ("cfl", C.c_double),
                ("dt_fixed", C.c_double), ("precision", C.c_int32), ("guess", C.c_int32),
                ("riemann_rtol", C.c_double), ("riemann_maxit", C.c_int32),
                ("tile_x", C.c_int32), ("tile_y", C.c_int32), ("tile_z", C.c_int32),
                ("limiter", C.c_int32), ("limiter_k", C.c_int32), ("flux", C.c_int32),
                ("ls_band", C.c_double), ("eos_general", C.c_int32), ("eos_reserved", C.c_int32),
                ("eos", Eos * 2), ("riemann_ds", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("t", C.c_double), ("dt_last", C.c_double),
                ("iface_faces_last", C.c_int64), ("riemann_solves", C.c_int64),
                ("newton_iters", C.c_int64), ("bisection_fallbacks", C.c_int64),
                ("flips", C.c_int64), ("orphans", C.c_int64), ("mlp_fallbacks", C.c_int64),
                ("err_code", C.c_int32), ("pad0", C.c_int32), ("err_cell", C.c_int64),
                ("ms_stage", C.c_double), ("ms_fiver", C.c_double), ("ms_other", C.c_double),
                ("stage_launches", C.c_int64), ("fiver_launches", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad0"}


class TrainOpts(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("epochs", C.c_int32), ("batch", C.c_int32),
                ("lr", C.c_float), ("lr_final", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float)]


M2C_EOS_NASG, M2C_EOS_MG, M2C_EOS_JWL = 0, 1, 2
M2C_EOS_MAX = 8


def eos_table(materials):
    """ctypes array of Eos from [(family, [params])]."""
    arr = (Eos * len(materials))()
    for i, (fam, prm) in enumerate(materials):
        arr[i].family = int(fam)
        for j, v in enumerate(prm):
            arr[i].prm[j] = float(v)
    return arr


class M2CError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"m2c error {code}: {msg}")
        self.code = code


_lib = None


def lib_path() -> str:
    return _LIB_PATH


def _declare(L):
    vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.m2c_config_default.argtypes = [C.POINTER(Config)]
    L.m2c_config_default.restype = None
    L.m2c_create.argtypes = [C.POINTER(Config), C.POINTER(vp)]
    L.m2c_destroy.argtypes = [vp]
    L.m2c_destroy.restype = None
    L.m2c_last_error.argtypes = [vp]
    L.m2c_last_error.restype = C.c_char_p
    L.m2c_strerror.argtypes = [C.c_int]
    L.m2c_strerror.restype = C.c_char_p
    L.m2c_set_stream.argtypes = [vp, vp]
    L.m2c_set_state.argtypes = [vp, vp]
    L.m2c_set_state_device.argtypes = [vp, vp]
    L.m2c_get_state.argtypes = [vp, vp, vp]
    L.m2c_get_state_device.argtypes = [vp, vp]
    L.m2c_get_conserved.argtypes = [vp, vp]
    L.m2c_set_conserved.argtypes = [vp, vp]
    L.m2c_step.argtypes = [vp, i32, C.POINTER(d)]
    L.m2c_step_dt.argtypes = [vp, i32, d, C.POINTER(d)]
    L.m2c_get_stats.argtypes = [vp, C.POINTER(Stats)]
    L.m2c_reset_stats.argtypes = [vp]
    L.m2c_set_profiling.argtypes = [vp, C.c_int]
    L.m2c_interface_faces.argtypes = [vp, vp, i64, C.POINTER(i64)]
    L.m2c_eval_hllc.argtypes = [i64, vp, vp, d, d, i32, vp, vp]
    L.m2c_riemann_solve.argtypes = [i64, vp, vp, i32, d, i32, vp, vp, vp]
    L.m2c_validate_config.argtypes = [C.POINTER(Config)]
    L.m2c_autotune.argtypes = [vp, i32, vp, C.POINTER(C.c_float)]
    L.m2c_get_tile.argtypes = [vp, vp]
    L.m2c_batch_create.argtypes = [i32, vp, C.POINTER(vp)]
    L.m2c_batch_destroy.argtypes = [vp]
    L.m2c_batch_destroy.restype = None
    L.m2c_batch_last_error.argtypes = [vp]
    L.m2c_batch_last_error.restype = C.c_char_p
    L.m2c_batch_size.argtypes = [vp]
    L.m2c_batch_set_state.argtypes = [vp, i32, vp]
    L.m2c_batch_get_state.argtypes = [vp, i32, vp, vp]
    L.m2c_batch_get_conserved.argtypes = [vp, i32, vp]
    L.m2c_batch_step.argtypes = [vp, i32]
    L.m2c_batch_get_stats.argtypes = [vp, i32, C.POINTER(Stats)]
    L.m2c_batch_set_tile.argtypes = [vp, i32, i32, i32]
    L.m2c_batch_get_tile.argtypes = [vp, vp]
    L.m2c_batch_autotune.argtypes = [vp, i32, vp, C.POINTER(C.c_float)]
    L.m2c_train_opts_default.argtypes = [C.POINTER(TrainOpts)]
    L.m2c_train_opts_default.restype = None
    L.m2c_mlp_create.argtypes = [vp, C.c_uint64, C.POINTER(vp)]
    L.m2c_mlp_destroy.argtypes = [vp]
    L.m2c_mlp_destroy.restype = None
    L.m2c_mlp_get_params.argtypes = [vp, vp]
    L.m2c_mlp_features.argtypes = [i64, vp, vp, vp, vp, vp, vp]
    L.m2c_mlp_forward.argtypes = [vp, i64, vp, vp, vp]
    L.m2c_mlp_grad.argtypes = [vp, i64, vp, vp, vp, C.POINTER(C.c_float), vp]
    L.m2c_mlp_train.argtypes = [vp, i64, vp, vp, C.POINTER(TrainOpts), vp, vp]
    L.m2c_riemann_solve_learned.argtypes = [vp, i64, vp, vp, d, i32, vp, vp, C.POINTER(i64), vp]
    L.m2c_set_guess.argtypes = [vp, vp]
    L.m2c_riemann_solve_learned_noalloc.argtypes = [vp, i64, vp, vp, d, i32, vp, vp, vp]
    L.m2c_riemann_solve_eos.argtypes = [i64, vp, vp, i32, vp, d, i32, d, vp, vp, vp]
    L.m2c_mlp_features_eos.argtypes = [i64, vp, vp, i32, vp, vp, vp, vp, vp]
    L.m2c_riemann_solve_eos_learned.argtypes = [vp, i64, vp, vp, i32, vp, d, i32, d, vp, vp, C.POINTER(i64), vp]
    L.m2c_eos_eval.argtypes = [i64, vp, vp, vp, i32, vp, vp, vp, vp]
    L.m2c_reinit.argtypes = [vp, i32, d]
    L.m2c_reinit_workspace.argtypes = [i32, i32, i32, C.POINTER(i64)]
    L.m2c_reinit_field.argtypes = [i32, i32, i32, vp, vp, vp, vp, i32, d, vp]
    for name in EXPORTS:
        if name not in _NO_STATUS:
            getattr(L, name).restype = C.c_int
    return L


def lib():
    """Load ``libm2c.so``; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                               "`python -m paper_2508_16387_amd.build` (there is no CPU fallback)")
        _lib = _declare(C.CDLL(_LIB_PATH))
    return _lib


def exported_symbols(path: str | None = None):
    """Names from EXPORTS that the shared object resolves (no GPU needed)."""
    L = C.CDLL(path or _LIB_PATH)
    return [n for n in EXPORTS if hasattr(L, n)]


def config_default() -> Config:
    c = Config()
    lib().m2c_config_default(C.byref(c))
    return c


def config_for(problem, precision=M2C_PREC_FP64, rtol=1e-12, maxit=50, alpha=1.2, tile=None,
               rk_order=2, limiter=M2C_LIM_MC, limiter_k=2, flux=M2C_FLUX_HLLC, ls_band=0.0) -> Config:
    """Configuration for a problem description with attributes n, lo, hi,
    gamma, pc, bc, cfl, dt_fixed and, for general equations of state, eos
    (as built by the ``workloads`` module)."""
    c = config_default()
    c.nx, c.ny, c.nz = (int(v) for v in problem.n)
    for d in range(3):
        c.lo[d], c.hi[d] = problem.lo[d], problem.hi[d]
    for m in range(2):
        c.gamma[m], c.pc[m] = problem.gamma[m], problem.pc[m]
    for f in range(6):
        c.bc[f] = int(problem.bc[f])
    c.limiter_alpha = alpha
    c.cfl = problem.cfl
    c.dt_fixed = problem.dt_fixed
    c.precision = precision
    c.riemann_rtol = rtol
    c.riemann_maxit = maxit
    c.rk_order = rk_order
    c.limiter = limiter
    c.limiter_k = limiter_k
    c.flux = flux
    c.ls_band = ls_band
    eos = getattr(problem, "eos", None)
    if eos is not None:
        # general EOS of materials 0 and 1: (family, [params]) pairs
        c.eos_general = 1
        for m in range(2):
            fam, prm = eos[m]
            c.eos[m].family = fam
            for k, v in enumerate(prm[:7]):
                c.eos[m].prm[k] = v
    if tile is not None:
        c.tile_x, c.tile_y, c.tile_z = tile
    return c


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()          # torch tensor


class Sim:
    """One simulation context on the current HIP device."""

    def __init__(self, cfg: Config, prim=None):
        self.L = lib()
        self.cfg = cfg
        self.n = (cfg.nx, cfg.ny, cfg.nz)
        self.N = cfg.nx * cfg.ny * cfg.nz
        h = C.c_void_p()
        rc = self.L.m2c_create(C.byref(cfg), C.byref(h))
        if rc != M2C_OK:
            raise M2CError(rc, "m2c_create failed: " + self.L.m2c_strerror(rc).decode())
        self.h = h
        if prim is not None:
            self.set_state(prim)

    def close(self):
        if getattr(self, "h", None):
            self.L.m2c_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def _check(self, rc):
        if rc != M2C_OK:
            raise M2CError(rc, self.L.m2c_last_error(self.h).decode())
        return rc

    def set_stream(self, stream):
        """stream: a torch.cuda.Stream, an int handle or None."""
        handle = None if stream is None else getattr(stream, "cuda_stream", stream)
        return self._check(self.L.m2c_set_stream(self.h, handle))

    def set_state(self, prim, check=True):
        a = np.ascontiguousarray(prim, dtype=np.float64).reshape(-1)
        assert a.size == 6 * self.N
        rc = self.L.m2c_set_state(self.h, a.ctypes.data)
        return self._check(rc) if check else rc

    def set_state_device(self, dprim):
        assert dprim.numel() == 6 * self.N and dprim.is_contiguous()
        return self._check(self.L.m2c_set_state_device(self.h, dprim.data_ptr()))

    def get_state(self):
        nx, ny, nz = self.n
        out = np.empty(6 * self.N)
        chi = np.empty(self.N, dtype=np.uint8)
        self._check(self.L.m2c_get_state(self.h, out.ctypes.data, chi.ctypes.data))
        return out.reshape(6, nz, ny, nx), chi.reshape(nz, ny, nx)

    def get_state_device(self, dprim):
        assert dprim.numel() == 6 * self.N and dprim.is_contiguous()
        return self._check(self.L.m2c_get_state_device(self.h, dprim.data_ptr()))

    def get_conserved(self):
        nx, ny, nz = self.n
        out = np.empty(6 * self.N)
        self._check(self.L.m2c_get_conserved(self.h, out.ctypes.data))
        return out.reshape(6, nz, ny, nx)

    def set_conserved(self, w6):
        a = np.ascontiguousarray(w6, dtype=np.float64).reshape(-1)
        assert a.size == 6 * self.N
        return self._check(self.L.m2c_set_conserved(self.h, a.ctypes.data))

    def step(self, n=1, check=True):
        t = C.c_double(0.0)
        rc = self.L.m2c_step(self.h, n, C.byref(t))
        if check:
            self._check(rc)
        return rc

    def reinit(self, iters, band=0.0, check=True):
        """Level-set reinitialization of the current state (between steps)."""
        rc = self.L.m2c_reinit(self.h, iters, band)
        if check:
            self._check(rc)
        return rc

    def step_dt(self, n, dt, check=True):
        t = C.c_double(0.0)
        rc = self.L.m2c_step_dt(self.h, n, dt, C.byref(t))
        if check:
            self._check(rc)
        return rc

    def stats(self):
        s = Stats()
        self._check(self.L.m2c_get_stats(self.h, C.byref(s)))
        return s.as_dict()

    def reset_stats(self):
        return self._check(self.L.m2c_reset_stats(self.h))

    def set_profiling(self, every=1):
        """Time one step in `every` with HIP events (True = every step,
        False or 0 = off)."""
        every = int(every) if not isinstance(every, bool) else (1 if every else 0)
        return self._check(self.L.m2c_set_profiling(self.h, every))

    def interface_faces(self):
        cnt = C.c_int64(0)
        self._check(self.L.m2c_interface_faces(self.h, None, 0, C.byref(cnt)))
        out = np.empty(max(cnt.value, 1), dtype=np.int32)
        self._check(self.L.m2c_interface_faces(self.h, out.ctypes.data, cnt.value, C.byref(cnt)))
        return out[:cnt.value]

    def last_error(self):
        return self.L.m2c_last_error(self.h).decode()

    def tile(self):
        t = (C.c_int32 * 3)()
        self._check(self.L.m2c_get_tile(self.h, t))
        return tuple(t)

    def set_guess(self, mlp):
        """Use the learned guess of an Mlp for later steps (None: acoustic)."""
        return self._check(self.L.m2c_set_guess(self.h, None if mlp is None else mlp.h))

    def autotune(self, steps=3):
        """Time every supported stage tile on this grid and keep the fastest;
        the state is restored.  Returns (tile, ms per step)."""
        t = (C.c_int32 * 3)()
        ms = C.c_float(0.0)
        self._check(self.L.m2c_autotune(self.h, steps, t, C.byref(ms)))
        return tuple(t), ms.value


class Batch:
    """Many independent runs advanced together (persistent kernels, hipGraph)."""

    def __init__(self, cfgs, prims=None):
        self.L = lib()
        n = len(cfgs)
        arr = (Config * n)(*cfgs)
        self.cfgs = list(cfgs)
        self.n = n
        h = C.c_void_p()
        rc = self.L.m2c_batch_create(n, arr, C.byref(h))
        if rc != M2C_OK:
            raise M2CError(rc, "m2c_batch_create failed: " + self.L.m2c_strerror(rc).decode())
        self.h = h
        if prims is not None:
            for k, p in enumerate(prims):
                self.set_state(k, p)

    def close(self):
        if getattr(self, "h", None):
            self.L.m2c_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def _check(self, rc):
        if rc != M2C_OK:
            raise M2CError(rc, self.L.m2c_batch_last_error(self.h).decode())
        return rc

    def _shape(self, k):
        c = self.cfgs[k]
        return c.nx, c.ny, c.nz

    def set_state(self, k, prim, check=True):
        nx, ny, nz = self._shape(k)
        a = np.ascontiguousarray(prim, dtype=np.float64).reshape(-1)
        assert a.size == 6 * nx * ny * nz
        rc = self.L.m2c_batch_set_state(self.h, k, a.ctypes.data)
        return self._check(rc) if check else rc

    def get_state(self, k):
        nx, ny, nz = self._shape(k)
        out = np.empty(6 * nx * ny * nz)
        chi = np.empty(nx * ny * nz, dtype=np.uint8)
        self._check(self.L.m2c_batch_get_state(self.h, k, out.ctypes.data, chi.ctypes.data))
        return out.reshape(6, nz, ny, nx), chi.reshape(nz, ny, nx)

    def get_conserved(self, k):
        nx, ny, nz = self._shape(k)
        out = np.empty(6 * nx * ny * nz)
        self._check(self.L.m2c_batch_get_conserved(self.h, k, out.ctypes.data))
        return out.reshape(6, nz, ny, nx)

    def step(self, n=1, check=True):
        rc = self.L.m2c_batch_step(self.h, n)
        if check:
            self._check(rc)
        return rc

    def stats(self, k):
        s = Stats()
        self._check(self.L.m2c_batch_get_stats(self.h, k, C.byref(s)))
        return s.as_dict()

    def set_tile(self, tx, ty, kz):
        return self._check(self.L.m2c_batch_set_tile(self.h, tx, ty, kz))

    def tile(self):
        t = (C.c_int32 * 3)()
        self._check(self.L.m2c_batch_get_tile(self.h, t))
        return tuple(t)

    def autotune(self, steps=3, cache=None, key=None):
        """Time every supported tile on the batch and keep the fastest (state
        restored).  With ``cache`` (a JSON file path) and ``key``, a tile
        found earlier for the same key is reused instead of timing again."""
        import json
        if cache and key and os.path.exists(cache):
            try:
                known = json.load(open(cache))
            except (OSError, ValueError):
                known = {}
            if key in known:
                self.set_tile(*known[key]["tile"])
                return tuple(known[key]["tile"]), known[key]["ms_per_step"]
        t = (C.c_int32 * 3)()
        ms = C.c_float(0.0)
        self._check(self.L.m2c_batch_autotune(self.h, steps, t, C.byref(ms)))
        if cache and key:
            try:
                known = json.load(open(cache)) if os.path.exists(cache) else {}
            except (OSError, ValueError):
                known = {}
            known[key] = {"tile": list(t), "ms_per_step": ms.value}
            with open(cache, "w") as f:
                json.dump(known, f, indent=1)
        return tuple(t), ms.value


def eval_hllc(qL, qR, gamma, pc, precision=M2C_PREC_FP64, F=None, stream=None):
    """HLLC at n faces; qL, qR: torch float64 cuda tensors [5, n] (face frame)."""
    import torch
    n = qL.shape[1]
    if F is None:
        F = torch.empty((5, n), dtype=torch.float64, device=qL.device)
    s = torch.cuda.current_stream(qL.device).cuda_stream if stream is None else stream
    rc = lib().m2c_eval_hllc(n, _ptr(qL), _ptr(qR), gamma, pc, precision, _ptr(F), s)
    if rc != M2C_OK:
        raise M2CError(rc, lib().m2c_strerror(rc).decode())
    return F


def riemann_solve(inp, eos, guess=M2C_GUESS_ACOUSTIC, rtol=1e-12, maxit=50, stream=None, check=True):
    """Two-material Riemann problems; inp [6, n], eos [4, n] float64 cuda
    tensors.  Returns (out [4, n], iters [n], rc)."""
    import torch
    n = inp.shape[1]
    out = torch.empty((4, n), dtype=torch.float64, device=inp.device)
    iters = torch.empty((n,), dtype=torch.int32, device=inp.device)
    s = torch.cuda.current_stream(inp.device).cuda_stream if stream is None else stream
    rc = lib().m2c_riemann_solve(n, _ptr(inp), _ptr(eos), guess, rtol, maxit, _ptr(out), _ptr(iters), s)
    if check and rc not in (M2C_OK, M2C_ERR_RIEMANN):
        raise M2CError(rc, lib().m2c_strerror(rc).decode())
    return out, iters, rc


def riemann_solve_eos(inp, mat, materials, rtol=1e-12, maxit=50, ds=0.0, stream=None, check=True):
    """General-EOS two-material Riemann problems: inp [6, n] float64 and mat
    [2, n] int32 cuda tensors, materials [(family, [params])].  Returns
    (out [4, n], iters [n], rc)."""
    import torch
    n = inp.shape[1]
    out = torch.empty((4, n), dtype=torch.float64, device=inp.device)
    iters = torch.empty((n,), dtype=torch.int32, device=inp.device)
    tab = eos_table(materials)
    rc = lib().m2c_riemann_solve_eos(n, _ptr(inp), _ptr(mat), len(materials), tab, rtol, maxit, ds, _ptr(out),
                                     _ptr(iters), _stream_of(inp, stream))
    if check and rc not in (M2C_OK, M2C_ERR_RIEMANN):
        raise M2CError(rc, lib().m2c_strerror(rc).decode())
    return out, iters, rc


def riemann_solve_eos_learned(mlp, inp, mat, materials, rtol=1e-12, maxit=50, ds=0.0, stream=None, check=True):
    """:func:`riemann_solve_eos` with the learned start of network ``mlp``
    (None: the acoustic start).  Returns (out [4, n], iters [n], rc,
    n_fallback)."""
    import torch
    n = inp.shape[1]
    out = torch.empty((4, n), dtype=torch.float64, device=inp.device)
    iters = torch.empty((n,), dtype=torch.int32, device=inp.device)
    nfb = C.c_int64(0)
    tab = eos_table(materials)
    rc = lib().m2c_riemann_solve_eos_learned(None if mlp is None else mlp.h, n, _ptr(inp), _ptr(mat), len(materials),
                                             tab, rtol, maxit, ds, _ptr(out), _ptr(iters), C.byref(nfb),
                                             _stream_of(inp, stream))
    if check and rc not in (M2C_OK, M2C_ERR_RIEMANN):
        raise M2CError(rc, lib().m2c_strerror(rc).decode())
    return out, iters, rc, nfb.value


def mlp_features_eos(inp, mat, materials, pstar=None, stream=None):
    """Features X [8, n] (and targets [n] when pstar is given) of the
    general-EOS learned start for problems inp [6, n] (float64) and mat
    [2, n] (int32) cuda tensors of materials [(family, [params])]."""
    import torch
    n = inp.shape[1]
    X = torch.empty((8, n), dtype=torch.float32, device=inp.device)
    t = torch.empty(n, dtype=torch.float32, device=inp.device) if pstar is not None else None
    rc = lib().m2c_mlp_features_eos(n, _ptr(inp), _ptr(mat), len(materials), eos_table(materials), _ptr(pstar),
                                    _ptr(X), _ptr(t), _stream_of(inp, stream))
    if rc != M2C_OK:
        raise M2CError(rc, "m2c_mlp_features_eos failed")
    return X, t


def eos_eval(rho, e, mat, materials, stream=None):
    """Pressure and sound speed of states (rho, e) (float64 cuda tensors)
    of materials mat (int32)."""
    import torch
    p, c = torch.empty_like(rho), torch.empty_like(rho)
    rc = lib().m2c_eos_eval(rho.numel(), _ptr(rho), _ptr(e), _ptr(mat), len(materials), eos_table(materials),
                            _ptr(p), _ptr(c), _stream_of(rho, stream))
    if rc != M2C_OK:
        raise M2CError(rc, lib().m2c_strerror(rc).decode())
    return p, c


def reinit_field(phi, h, bc, iters, band=0.0, stream=None):
    """Level-set reinitialization of a float64 cuda tensor phi shaped (nz,
    ny, nx), in place; h = cell widths (x, y, z), bc = six boundary codes."""
    import torch
    nz, ny, nx = phi.shape
    nbytes = C.c_int64()
    rc = lib().m2c_reinit_workspace(nx, ny, nz, C.byref(nbytes))
    if rc != M2C_OK:
        raise M2CError(rc, lib().m2c_strerror(rc).decode())
    work = torch.empty(int(nbytes.value), dtype=torch.uint8, device=phi.device)
    hh = (C.c_double * 3)(*h)
    bb = (C.c_int32 * 6)(*bc)
    rc = lib().m2c_reinit_field(nx, ny, nz, hh, bb, _ptr(phi), _ptr(work), iters, band, _stream_of(phi, stream))
    if rc != M2C_OK:
        raise M2CError(rc, lib().m2c_strerror(rc).decode())
    return phi


def _stream_of(t, stream):
    import torch
    return torch.cuda.current_stream(t.device).cuda_stream if stream is None else stream


class Mlp:
    """The learned star-pressure guess network (weights in device memory)."""

    def __init__(self, params=None, seed=0):
        self.L = lib()
        h = C.c_void_p()
        arr = None
        if params is not None:
            arr = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
            assert arr.size == NPARAM
        rc = self.L.m2c_mlp_create(None if arr is None else arr.ctypes.data, seed, C.byref(h))
        if rc != M2C_OK:
            raise M2CError(rc, "m2c_mlp_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.m2c_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def params(self):
        out = np.empty(NPARAM, dtype=np.float32)
        rc = self.L.m2c_mlp_get_params(self.h, out.ctypes.data)
        if rc != M2C_OK:
            raise M2CError(rc, "m2c_mlp_get_params failed")
        return out

    def forward(self, X, stream=None):
        import torch
        n = X.shape[1]
        y = torch.empty(n, dtype=torch.float32, device=X.device)
        rc = self.L.m2c_mlp_forward(self.h, n, _ptr(X), _ptr(y), _stream_of(X, stream))
        if rc != M2C_OK:
            raise M2CError(rc, "m2c_mlp_forward failed")
        return y

    def grad(self, X, t, stream=None):
        n = X.shape[1]
        g = np.empty(NPARAM, dtype=np.float32)
        loss = C.c_float(0.0)
        rc = self.L.m2c_mlp_grad(self.h, n, _ptr(X), _ptr(t), g.ctypes.data, C.byref(loss), _stream_of(X, stream))
        if rc != M2C_OK:
            raise M2CError(rc, "m2c_mlp_grad failed")
        return g, loss.value

    def train(self, X, t, epochs=20, batch=4096, lr=3e-3, lr_final=1e-4, stream=None):
        o = TrainOpts()
        self.L.m2c_train_opts_default(C.byref(o))
        o.epochs, o.batch, o.lr, o.lr_final = epochs, batch, lr, lr_final
        hist = np.zeros(epochs, dtype=np.float32)
        rc = self.L.m2c_mlp_train(self.h, X.shape[1], _ptr(X), _ptr(t), C.byref(o), hist.ctypes.data,
                                  _stream_of(X, stream))
        if rc != M2C_OK:
            raise M2CError(rc, "m2c_mlp_train failed")
        return hist


def mlp_features(inp, eos, pstar=None, stream=None):
    """Features X [8, n] (and targets [n] when pstar is given) of problems
    inp [6, n], eos [4, n] (float64 cuda tensors)."""
    import torch
    n = inp.shape[1]
    X = torch.empty((8, n), dtype=torch.float32, device=inp.device)
    t = torch.empty(n, dtype=torch.float32, device=inp.device) if pstar is not None else None
    rc = lib().m2c_mlp_features(n, _ptr(inp), _ptr(eos), _ptr(pstar), _ptr(X), _ptr(t), _stream_of(inp, stream))
    if rc != M2C_OK:
        raise M2CError(rc, "m2c_mlp_features failed")
    return X, t


def riemann_solve_learned(mlp, inp, eos, rtol=1e-12, maxit=50, stream=None):
    """Riemann problems with the learned guess (mlp None: acoustic).
    Returns (out [4, n], iters [n], rc, n_fallback)."""
    import torch
    n = inp.shape[1]
    out = torch.empty((4, n), dtype=torch.float64, device=inp.device)
    iters = torch.empty((n,), dtype=torch.int32, device=inp.device)
    nfb = C.c_int64(0)
    rc = lib().m2c_riemann_solve_learned(None if mlp is None else mlp.h, n, _ptr(inp), _ptr(eos), rtol, maxit,
                                         _ptr(out), _ptr(iters), C.byref(nfb), _stream_of(inp, stream))
    if rc not in (M2C_OK, M2C_ERR_RIEMANN):
        raise M2CError(rc, "m2c_riemann_solve_learned failed")
    return out, iters, rc, nfb.value


NOALLOC_MAX_PROBLEMS = 1 << 20


def riemann_solve_learned_async(mlp, inp, eos, out=None, iters=None, rtol=1e-12, maxit=50, stream=None):
    """The allocation-free, non-synchronising form of
    :func:`riemann_solve_learned` (mlp None: acoustic guess); the kernels are
    only enqueued.  Returns (out [4, n], iters [n]); iters 0 marks a problem
    without admissible star pressure.  At most NOALLOC_MAX_PROBLEMS problems."""
    import torch
    n = inp.shape[1]
    if out is None:
        out = torch.empty((4, n), dtype=torch.float64, device=inp.device)
    if iters is None:
        iters = torch.empty((n,), dtype=torch.int32, device=inp.device)
    rc = lib().m2c_riemann_solve_learned_noalloc(None if mlp is None else mlp.h, n, _ptr(inp), _ptr(eos), rtol,
                                                 maxit, _ptr(out), _ptr(iters), _stream_of(inp, stream))
    if rc != M2C_OK:
        raise M2CError(rc, "m2c_riemann_solve_learned_noalloc failed: " + lib().m2c_strerror(rc).decode())
    return out, iters
