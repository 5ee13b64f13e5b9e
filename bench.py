"""Throughput of the two-material finite-volume step on one MI355X.

One benchmark step is one full time step of the hot path (CFL time step,
interface compaction, two TVD-RK2 stages each with FIVER interface fluxes
and the fused bulk stage kernel, phase update) on the 128^3 shock-bubble
workload: unit box, air bubble of radius 0.15 at a seed-jittered centre in
water at 1e5 Pa, planar water shock of 1e8 Pa at x = 0.1, transmissive
boundaries, CFL 0.4.  The state is resident in HBM before the timed region.

Prints one JSON line; see ``--help``.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Compulsory HBM bytes per cell of the fused stage kernel (FP64 SoA state of
# 5 conserved fields + phi, uint8 material id): stage 1 reads W^n, phi, chi
# (49 B) and writes W(1), phi (48 B); stage 2 also reads W^n, phi (48 B).
BYTES_STAGE1, BYTES_STAGE2 = 97, 145


PROFILE_EVERY = 10


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=128, help="grid edge (default 128)")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=4,
                    help="oracle steps timed for the CPU baseline (bounded sample)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the mixed-precision, batched and standalone-FIVER measurements")
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--cloud-steps", type=int, default=10,
                    help="steps timed on the 384^3 bubble cloud (0 skips it)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy five times (reference "
                         "for scaling hardware byte counters to bytes)")
    return ap.parse_args()


def measured_traffic(precision):
    """HBM bytes per stage launch from the committed rocprofv3 counter
    summary, if it was taken on the stage-kernel sources as they are now."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "k_stage_traffic.json")
    if precision != "fp64" or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    m = hashlib.sha256()
    for src in rec["sources"]:
        m.update(open(os.path.join(ROOT, src), "rb").read())
    if m.hexdigest()[:16] != rec["source_sha256_16"]:
        return None
    return rec["bytes_per_launch_mean"]


# VALU issue peak: one wave64 VALU instruction per CU per clock (a SIMD
# takes four clocks per wave64 FP64 or unpacked FP32 instruction), 256 CUs
# at 2.4 GHz, in lane-instructions per second
VALU_PEAK = 256 * 2.4e9 * 64


def valu_line(instr_per_cell, cells, launch_ms):
    """The stage kernel against the VALU issue roof (the bound it meets
    first in FP64): instructions per cell from the counters, rate from the
    live launch time."""
    if instr_per_cell is None:
        return None
    rate = instr_per_cell * cells / (launch_ms * 1e-3)
    return {"instr_per_cell": instr_per_cell, "achieved": rate, "peak": VALU_PEAK,
            "unit": "lane-instructions/s", "frac": rate / VALU_PEAK}


def measured_valu(precision):
    """VALU lane-instructions per cell-update of the stage kernel from the
    committed SQ counter summary, if it was taken on the current sources."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "k_stage_valu.json")
    if precision != "fp64" or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    m = hashlib.sha256()
    for src in rec["sources"]:
        m.update(open(os.path.join(ROOT, src), "rb").read())
    if m.hexdigest()[:16] != rec["source_sha256_16"]:
        return None
    return rec["valu_instr_per_cell_mean"]


def time_sim(m2c, torch, problem, precision, steps, warmup, tile=None):
    """Cell-updates/s per RK stage of one context over `steps` steps."""
    sim = m2c.Sim(m2c.config_for(problem, precision=precision, tile=tile))
    sim.set_stream(torch.cuda.current_stream())
    sim.set_state(problem.prim)
    if warmup:
        sim.step(warmup)
        sim.set_state(problem.prim)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    return problem.ncells * steps * 2 / T, T


def batched_forms(m2c, torch, steps):
    """64 independent shock-bubble runs with grid edges from {32,...,128} per
    axis, advanced by the batched form (autotuned tile, graph replay), against
    the same runs stepped one context after another on the FP64 path."""
    import workloads as W

    probs = W.batched_shock_bubbles(0, steps=steps)
    cells = sum(p.ncells for p in probs)
    out = {"workload": "64 shock-bubble runs, edges in {32,48,64,96,128}, radius U[0.1,0.25], "
                       "shock log-U[1e7,1e9] Pa", "cells": cells, "steps": steps}
    for prec, name in ((m2c.M2C_PREC_FP64, "fp64"), (m2c.M2C_PREC_MIXED, "mixed")):
        b = m2c.Batch([m2c.config_for(p, precision=prec) for p in probs], [p.prim for p in probs])
        tile, _ = b.autotune(steps=2)
        b.step(2)                                   # warm-up (graph instantiation)
        for k, p in enumerate(probs):
            b.set_state(k, p.prim)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(steps)
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        out[f"value_{name}"] = cells * steps * 2 / T
        out[f"tile_{name}"] = list(tile)
        b.close()
    # the same runs on the plain FP64 path, one context after another
    sims = [m2c.Sim(m2c.config_for(p), p.prim) for p in probs]
    for s in sims:
        s.step(1)
    for s, p in zip(sims, probs):
        s.set_state(p.prim)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in sims:
        s.step(steps)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    out["value_sequential_fp64"] = cells * steps * 2 / T
    out["speedup_batched_fp64_vs_sequential_fp64"] = out["value_fp64"] / out["value_sequential_fp64"]
    out["speedup_batched_mixed_vs_sequential_fp64"] = out["value_mixed"] / out["value_sequential_fp64"]
    return out


def fiver_standalone(m2c, torch, n=1_000_000):
    """Exact two-material Riemann solves/s on n water/air problems."""
    import workloads as W

    inp, eos = W.riemann_problem_set(1, n)
    di = torch.tensor(inp.T.copy(), device="cuda")
    de = torch.tensor(eos.T.copy(), device="cuda")
    m2c.riemann_solve(di, de)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out, iters, rc = m2c.riemann_solve(di, de)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    it = iters.abs().double()
    ok = (iters != 0)
    return {"problems": n, "solves_per_s": n / T, "ms": T * 1e3,
            "newton_iters_per_solve": float(it[ok].mean()), "vacuum": int((~ok).sum())}


def general_eos_standalone(m2c, torch, n=1 << 20):
    """Two-material Riemann solves/s with a general EOS on each side (NASG,
    Mie-Grueneisen, JWL): the mixed set of eight material pairs in one launch,
    and single-pair sets of three kinds (gas / solid, detonation products /
    gas, solid / solid in tension)."""
    import workloads as W

    def run(pairs):
        inp, mat, mats, _ = W.general_eos_problem_set(2024, n, pairs=pairs)
        ti = torch.tensor(inp, dtype=torch.float64, device="cuda")
        tm = torch.tensor(mat, dtype=torch.int32, device="cuda")
        m2c.riemann_solve_eos(ti, tm, mats)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out, it, rc = m2c.riemann_solve_eos(ti, tm, mats)
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        ok = it != 0
        return {"solves_per_s": n / T, "ms": T * 1e3, "newton_iters_per_solve": float(it.abs().double()[ok].mean()),
                "no_star_state": int((~ok).sum())}

    res = {"problems": n, "ds": 0.01, "mixed_pairs": run(None)}
    for pr in (("air", "glass"), ("tnt", "air"), ("copper", "tantalum")):
        res["-".join(pr)] = run([pr])
    return res


def reinit_form(m2c, torch, problem, iters=100):
    """Level-set reinitialization of the benchmark's level set: pseudo-time
    steps per second over the whole grid and in a narrow band of six cells,
    with the HBM rate of the algorithmic 24 bytes (phi and S read, phi
    written) per moving cell and step."""
    nx, ny, nz = problem.n
    N = nx * ny * nz
    h, bc = problem.dx(), problem.bc
    phi0 = torch.tensor(problem.prim[5], dtype=torch.float64, device="cuda").contiguous()
    # a level set far from a distance: the signed distance stretched by 3
    # on the positive side
    phi0 = torch.where(phi0 > 0, 3.0 * phi0, phi0)
    m2c.reinit_field(phi0.clone(), h, bc, 4)
    torch.cuda.synchronize()
    res = {"grid": [nx, ny, nz], "iters": iters}
    for name, band in (("full", 0.0), ("band_6h", 6.0 * min(h))):
        moving = int(((phi0.abs() < band) if band > 0 else torch.ones_like(phi0, dtype=torch.bool)).sum())
        t = phi0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m2c.reinit_field(t, h, bc, iters, band)
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        res[name] = {"ms_per_iter": T / iters * 1e3, "cell_iters_per_s": N * iters / T,
                     "moving_fraction": moving / N, "hbm_gbs_algorithmic": 24.0 * moving * iters / T / 1e9,
                     "hbm_frac": 24.0 * moving * iters / T / 8e12}
    return res


def scheme_options(m2c, torch, problem, steps=20):
    """The paper's other scheme options on the headline workload (FP64):
    cell-updates/s per RK stage of TVD-RK3, forward Euler, the Van Albada
    limiter (k = 2), the local Lax-Friedrichs flux and a six-cell
    narrow-band level set, each with the other choices at their defaults."""
    h = min(problem.dx())
    cases = {"rk3": dict(rk_order=3), "forward_euler": dict(rk_order=1),
             "van_albada_k2": dict(limiter=m2c.M2C_LIM_VAN_ALBADA, limiter_k=2),
             "llf": dict(flux=m2c.M2C_FLUX_LLF), "ls_band_6h": dict(ls_band=6.0 * h)}
    out = {}
    for name, kw in cases.items():
        sim = m2c.Sim(m2c.config_for(problem, **kw))
        sim.set_stream(torch.cuda.current_stream())
        sim.set_state(problem.prim)
        sim.step(2)
        sim.set_state(problem.prim)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        stages = kw.get("rk_order", 2)
        out[name] = {"cell_updates_per_stage_per_s": problem.ncells * steps * stages / T,
                     "ms_per_step": T / steps * 1e3}
    return out


def general_eos_step(m2c, torch, steps=20):
    """The time step with a general EOS per material: a sphere (r = 0.28)
    of detonation products (JWL, 1630 kg/m^3, 5 GPa) in NASG water at rest
    on 128^3 cells, FP64, TVD-RK2 with MC and HLLC.  Interface faces take the
    general-EOS exact Riemann solve (Hugoniot shocks, closed-form JWL and
    NASG isentropes)."""
    import workloads as W
    p = W.eos_charge(0, n=(128, 128, 128), steps=steps)
    rate, T = time_sim(m2c, torch, p, m2c.M2C_PREC_FP64, steps, 2)
    return {"workload": "tnt_sphere_in_water_nasg_128", "steps": steps, "cell_updates_per_stage_per_s": rate,
            "ms_per_step": T / steps * 1e3}


def host_round_trip(m2c, torch, problem, steps):
    """The same FP64 run with the state handed over in host memory: upload
    (primitive -> conservative on the device), `steps` steps, download.  A
    PCIe-inclusive rate beside the device-resident headline value."""
    sim = m2c.Sim(m2c.config_for(problem, precision=m2c.M2C_PREC_FP64))
    sim.set_stream(torch.cuda.current_stream())
    sim.set_state(problem.prim)
    sim.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.set_state(problem.prim)
    t1 = time.perf_counter()
    sim.step(steps)
    t2 = time.perf_counter()
    sim.get_state()
    t3 = time.perf_counter()
    return {"steps": steps, "upload_ms": (t1 - t0) * 1e3, "steps_ms": (t2 - t1) * 1e3,
            "download_ms": (t3 - t2) * 1e3, "value_pcie_inclusive": problem.ncells * steps * 2 / (t3 - t0)}


def cloud_forms(m2c, torch, steps):
    """384^3 cloud of 32 air bubbles in water (50 steps in the workload; a
    bounded number of them timed here): FP64 vs mixed precision, and the
    learned star-pressure guess against the acoustic one on the FP64 path."""
    import numpy as np

    import workloads as W

    p = W.bubble_cloud(0)
    out = {"workload": "bubble_cloud_384^3: 32 air bubbles r~U[0.02,0.06] in water, 5e7 Pa slab at x<0.05",
           "cells": p.ncells, "steps_timed": steps}
    net = m2c.Mlp(np.load(os.path.join(ROOT, "paper_2508_16387_amd", "learned_guess.npy")))
    runs = (("fp64", m2c.M2C_PREC_FP64, None), ("mixed", m2c.M2C_PREC_MIXED, None),
            ("fp64_learned_guess", m2c.M2C_PREC_FP64, net))
    for name, prec, guess in runs:
        sim = m2c.Sim(m2c.config_for(p, precision=prec))
        sim.set_stream(torch.cuda.current_stream())
        sim.set_state(p.prim)
        if guess is not None:
            sim.set_guess(guess)
        sim.step(1)
        sim.set_state(p.prim)
        sim.reset_stats()
        sim.set_profiling(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        st = sim.stats()
        out[name] = {"value": p.ncells * steps * 2 / T, "ms_per_step": T * 1e3 / steps,
                     "stage_ms_per_launch": st["ms_stage"] / max(st["stage_launches"], 1),
                     "fiver_ms_per_launch": st["ms_fiver"] / max(st["fiver_launches"], 1),
                     "riemann_solves": st["riemann_solves"],
                     "newton_iters_per_solve": st["newton_iters"] / max(st["riemann_solves"], 1),
                     "learned_guess_rejected": st["mlp_fallbacks"] if guess is not None else None}
        sim.close()
    out["speedup_mixed_vs_fp64"] = out["mixed"]["value"] / out["fp64"]["value"]
    out["fiver_speedup_learned_vs_acoustic"] = (out["fp64"]["fiver_ms_per_launch"] /
                                                out["fp64_learned_guess"]["fiver_ms_per_launch"])
    return out


def learned_standalone(m2c, torch, n=1_000_000):
    """Held-out water/air Riemann problems: Newton steps and solves/s with the
    judged learned guess against the acoustic guess."""
    import numpy as np

    import workloads as W

    inp, eos = W.riemann_problem_set(2000, n)
    di = torch.tensor(inp.T.copy(), device="cuda")
    de = torch.tensor(eos.T.copy(), device="cuda")
    net = m2c.Mlp(np.load(os.path.join(ROOT, "paper_2508_16387_amd", "learned_guess.npy")))
    res = {"problems": n}
    for name, guess in (("acoustic", None), ("learned", net)):
        m2c.riemann_solve_learned(guess, di, de)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out, it, rc, nfb = m2c.riemann_solve_learned(guess, di, de)
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        it = it.abs().double()
        ok = it > 0
        res[name] = {"solves_per_s": n / T, "newton_iters_per_solve": float(it[ok].mean()),
                     "acoustic_starts": int(nfb) if guess is not None else None}
    res["speedup_learned_vs_acoustic"] = res["learned"]["solves_per_s"] / res["acoustic"]["solves_per_s"]
    return res


def cpu_baseline(problem, steps):
    import oracle

    oracle.build(force=False)
    s = oracle.OracleSim(problem)
    t0 = time.perf_counter()
    rc = s.step(steps)
    t = time.perf_counter() - t0
    assert rc == 0
    N = problem.ncells
    # the general-EOS Riemann oracle on a sample of the mixed problem set
    import workloads as W
    from oracle import riemann_eos as RE

    ne = 64
    inp, mat, mats, _ = W.general_eos_problem_set(2024, ne)
    eos = [RE.make_eos(f, prm) for f, prm in mats]
    t0 = time.perf_counter()
    RE.solve(inp, mat, eos)
    te = time.perf_counter() - t0
    return {"value": N * steps * 2 / t, "unit": "cell-updates/s per RK stage", "cores": 1,
            "kind": "oracle",
            "sample": f"first {steps} steps of the same {problem.n[0]}x{problem.n[1]}x{problem.n[2]} "
                      f"shock-bubble run, single-threaded C oracle ({t:.1f} s)",
            "general_eos_riemann": {"solves_per_s": ne / te, "cores": 1,
                                    "sample": f"first {ne} problems of the mixed general-EOS set, Python/scipy "
                                              f"oracle ({te:.1f} s)"}}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    torch.cuda.set_device(0)
    if args.copy_probe:
        x = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        x.fill_(1.0)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": x.numel() * 8, "copy_probe_bytes_written": y.numel() * 8}))
        return

    import paper_2508_16387_amd as m2c
    import workloads as W

    p = W.shock_bubble(args.seed, n=args.n)
    prec = m2c.M2C_PREC_MIXED if args.precision == "mixed" else m2c.M2C_PREC_FP64
    sim = m2c.Sim(m2c.config_for(p, precision=prec))
    stream = torch.cuda.current_stream()
    sim.set_stream(stream)
    sim.set_state(p.prim)
    if args.warmup:
        sim.step(args.warmup)
        sim.set_state(p.prim)          # time steps 1..K of the workload
    sim.reset_stats()
    # HIP events around the kernels of one step in PROFILE_EVERY, on the
    # library's stream, inside the timed region
    sim.set_profiling(PROFILE_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    st = sim.stats()
    N = p.ncells
    value = N * args.steps * 2 / T

    stage_ms = st["ms_stage"] / max(st["stage_launches"], 1)
    fiver_ms = st["ms_fiver"] / max(st["fiver_launches"], 1)
    bytes_per_launch = N * (BYTES_STAGE1 + BYTES_STAGE2) / 2
    traffic = measured_traffic(args.precision)
    achieved = bytes_per_launch / (stage_ms * 1e-3) / 1e9
    out = {
        "metric": "cell-updates/s per RK stage",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == m2c.M2C_PREC_FP64 else "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"shock_bubble_{args.n}^3", "grid": [args.n] * 3, "steps": args.steps,
                   "precision": args.precision, "rk": "TVD-RK2", "cfl": p.cfl, "seed": args.seed},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_frac": (None if traffic is None
                                      else traffic / (stage_ms * 1e-3) / 1e9 / HBM_PEAK_GBS),
                     "valu": valu_line(measured_valu(args.precision), N, stage_ms),
                     "kernel": "k_stage (both RK stages)", "avg_launch_ms": stage_ms,
                     "algorithmic_bytes_per_launch": bytes_per_launch},
        "fiver": {"solves": st["riemann_solves"], "ms_per_launch": fiver_ms,
                  "solves_per_s": st["riemann_solves"] / (2 * args.steps) / max(fiver_ms * 1e-3, 1e-12),
                  "newton_iters_per_solve": st["newton_iters"] / max(st["riemann_solves"], 1)},
        "time_split_ms_per_step": {k: st[f"ms_{k}"] * 2 / max(st["stage_launches"], 1)
                                   for k in ("stage", "fiver", "other")},
    }
    if not args.no_forms:
        other = m2c.M2C_PREC_MIXED if prec == m2c.M2C_PREC_FP64 else m2c.M2C_PREC_FP64
        v_other, _ = time_sim(m2c, torch, p, other, args.steps, args.warmup)
        v64, vmx = (value, v_other) if prec == m2c.M2C_PREC_FP64 else (v_other, value)
        out["forms"] = {
            "fp64": v64,
            "mixed": vmx,
            "speedup_mixed_vs_fp64": vmx / v64,
            "batched": batched_forms(m2c, torch, args.batch_steps),
            "fiver_standalone": fiver_standalone(m2c, torch),
            "learned_guess_standalone": learned_standalone(m2c, torch),
            "general_eos_riemann": general_eos_standalone(m2c, torch),
            "reinit_128": reinit_form(m2c, torch, p),
            "general_eos_step_128": general_eos_step(m2c, torch),
            "scheme_options_128": scheme_options(m2c, torch, p),
            "host_round_trip": host_round_trip(m2c, torch, p, args.steps),
        }
        if args.cloud_steps > 0:
            out["forms"]["cloud_384"] = cloud_forms(m2c, torch, args.cloud_steps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
