"""Error measures for GPU-vs-oracle parity (shared by the tests and the
smoke check).

Per conserved variable k in (rho, rho u, rho v, rho w, rho E) and phi:

    e_k = max_i |x_i(GPU) - x_i(oracle)| / max(max_i |x_i(oracle)|, floor_k)

with floors 1 kg/m^3 (rho), 1e-3 max(rho c) (momenta), max|rho E| (energy)
and the smallest cell width (phi).  Cells whose material differs between the
two results are counted separately.
"""
from __future__ import annotations

import numpy as np

NAMES = ("rho", "rhou", "rhov", "rhow", "rhoE", "phi")

# FP64 forms: bound on e_k at the final step of every parity run.  Derived
# from the arithmetic: both sides evaluate the same formulas in IEEE FP64;
# they differ by fused multiply-add contraction, multiplication by
# reciprocals instead of division and libm vs device pow/sqrt (each <= 1 ulp
# per operation).  Relative perturbations of ~1e-16 per operation grow
# through ~1e2 operations per cell-stage and are amplified by the stiffened
# gas cancellation p = (gamma-1)(rho E - ke) - gamma p_c (~gamma p_c / p,
# ~2e4 for water at 1 bar) but enter the conserved variables only through
# fluxes, so 1e-9 leaves several decades of margin above the ~1e-13 expected
# while failing on any single wrong term.
TOL_FP64 = 1e-9


def conserved_errors(w_gpu, w_ora, prim_ora, gamma, pc, chi_ora, h_min, eos=None):
    """e_k for the six fields of two conservative states [6, ...]; eos:
    general EOS of materials 0 and 1 as (family, params) pairs (then the
    sound speeds of the momentum floor come from those)."""
    w_gpu = np.asarray(w_gpu).reshape(6, -1)
    w_ora = np.asarray(w_ora).reshape(6, -1)
    prim = np.asarray(prim_ora).reshape(6, -1)
    chi = np.asarray(chi_ora).reshape(-1)
    if eos is None:
        g = np.where(chi == 1, gamma[1], gamma[0])
        p_c = np.where(chi == 1, pc[1], pc[0])
        c = np.sqrt(g * (prim[4] + p_c) / prim[0])
    else:
        from oracle import riemann_eos as RE
        mats = [RE.make_eos(f, prm) for f, prm in eos]
        c = np.array([np.sqrt(max(mats[x].c2(r, mats[x].e(r, p)), 0.0))
                      for x, r, p in zip(chi, prim[0], prim[4])])
    rc_max = float(np.max(prim[0] * c))
    floors = [1.0, 1e-3 * rc_max, 1e-3 * rc_max, 1e-3 * rc_max, float(np.max(np.abs(w_ora[4]))), h_min]
    out = {}
    for k, name in enumerate(NAMES):
        scale = max(float(np.max(np.abs(w_ora[k]))), floors[k])
        out[name] = float(np.max(np.abs(w_gpu[k] - w_ora[k]))) / scale
    return out


def compare_runs(gpu_sim, ora_sim, problem):
    """Errors between the current states of a GPU context and the oracle."""
    w_g = gpu_sim.get_conserved()
    _, chi_g = gpu_sim.get_state()
    w_o = ora_sim.cons()
    prim_o, chi_o = ora_sim.prim()
    h_min = min(problem.dx())
    e = conserved_errors(w_g, w_o, prim_o, problem.gamma, problem.pc, chi_o, h_min, getattr(problem, "eos", None))
    e["id_mismatch"] = int(np.count_nonzero(chi_g.reshape(-1) != chi_o.reshape(-1)))
    return e
