"""Throughput of the two-material finite-volume step on one MI355X.

One benchmark step is one full time step of the hot path (CFL time step,
interface compaction, two TVD-RK2 stages each with FIVER interface fluxes
and the fused bulk stage kernel, phase update).  The default workload is the
largest single-GPU configuration: the 384^3 cloud of 32 air bubbles (radii
U[0.02, 0.06], seed-drawn non-overlapping centres) in water at 1e5 Pa with a
5e7 Pa water slab at x < 0.05, transmissive boundaries, CFL 0.4, FP64, all
50 steps of the workload timed by default.  ``--workload shock_bubble_128``
selects the 128^3 shock-bubble instead.  The state is resident in HBM before
the timed region.

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

# Workloads the headline can run on: builder, default step count (the
# workload's own length).
WORKLOADS = {
    "cloud_384": "bubble_cloud_384^3",
    "shock_bubble_128": "shock_bubble_128^3",
    "charge_128": "tnt_sphere_in_water_nasg_128^3",
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50,
                    help="timed steps (default 50: the whole 384^3 cloud workload)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=list(WORKLOADS), default="cloud_384")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the other forms (mixed, batched, standalone solvers, options, ...)")
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--in-situ-advance", type=int, default=400,
                    help="untimed steps of the 384^3 cloud before the in-situ learned-guess "
                         "comparison (the slab's shock reaches the first bubbles)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy five times (reference "
                         "for scaling hardware byte counters to bytes)")
    return ap.parse_args()


def _profile_record(kind, workload, precision):
    """A committed per-launch counter record (HBM bytes or VALU
    instructions) of the stage kernel on this workload, if it was taken on
    the stage-kernel sources as they are now."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"k_stage_{workload}_{precision}_{kind}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    m = hashlib.sha256()
    for src in rec["sources"]:
        m.update(open(os.path.join(ROOT, src), "rb").read())
    if m.hexdigest()[:16] != rec["source_sha256_16"]:
        return None
    return rec


def measured_traffic(workload, precision):
    """Counted HBM bytes per stage launch (FETCH_SIZE and WRITE_SIZE scaled by
    the copy calibration)."""
    rec = _profile_record("traffic", workload, precision)
    return None if rec is None else rec["bytes_per_launch_mean"]


# VALU issue peak: one wave64 VALU instruction per CU per clock (a SIMD
# takes four clocks per wave64 FP64 or unpacked FP32 instruction), 256 CUs
# at 2.4 GHz, in lane-instructions per second
VALU_PEAK = 256 * 2.4e9 * 64


def valu_line(instr_per_cell, cells, launch_ms):
    """The stage kernel against the VALU issue roof: instructions per cell
    from the counters, rate from the live launch time."""
    if instr_per_cell is None:
        return None
    rate = instr_per_cell * cells / (launch_ms * 1e-3)
    return {"instr_per_cell": instr_per_cell, "achieved": rate, "peak": VALU_PEAK,
            "unit": "lane-instructions/s", "frac": rate / VALU_PEAK}


def measured_valu(workload, precision):
    """VALU lane-instructions per cell-update of the stage kernel."""
    rec = _profile_record("valu", workload, precision)
    return None if rec is None else rec["valu_instr_per_cell_mean"]


def progress(msg):
    """A progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_problem(workload, seed):
    import workloads as W
    if workload == "cloud_384":
        return W.bubble_cloud(seed)
    if workload == "charge_128":
        # general EOS per material: JWL detonation products in NASG water
        return W.eos_charge(seed, n=(128, 128, 128), steps=50)
    return W.shock_bubble(seed, n=128)


def device_ms(torch, fn, reps, warm=2):
    """Median device time of fn() over reps launches, from events recorded
    on the current stream around each call (fn must not synchronise)."""
    for _ in range(warm):
        fn()
    st = torch.cuda.current_stream()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        fn()
        e1.record(st)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2], times


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


def fiver_standalone(m2c, torch, n=1_000_000, reps=20):
    """Exact two-material Riemann solves/s on n water/air problems (acoustic
    guess), device time as the median of ``reps`` launches."""
    import workloads as W

    inp, eos = W.riemann_problem_set(1, n)
    di = torch.tensor(inp.T.copy(), device="cuda")
    de = torch.tensor(eos.T.copy(), device="cuda")
    out = torch.empty((4, n), dtype=torch.float64, device="cuda")
    it = torch.empty((n,), dtype=torch.int32, device="cuda")
    ms, _ = device_ms(torch, lambda: m2c.riemann_solve_learned_async(None, di, de, out=out, iters=it), reps)
    itd = it.abs().double()
    ok = (it != 0)
    return {"problems": n, "launches": reps, "solves_per_s": n / (ms * 1e-3), "ms": ms,
            "newton_iters_per_solve": float(itd[ok].mean()), "vacuum": int((~ok).sum())}


def general_eos_standalone(m2c, torch, n=1 << 20, reps=5):
    """Two-material Riemann solves/s with a general EOS on each side (NASG,
    Mie-Grueneisen, JWL): the mixed set of eight material pairs in one call,
    its four pairs without a Mie-Grueneisen side, and single-pair sets of
    three kinds (gas / solid, detonation products / gas, solid / solid in
    tension), each from the acoustic start and from the learned start
    (committed network).  The median of ``reps`` timed calls (each groups
    the set by material pair, solves, and synchronises)."""
    import workloads as W

    import numpy as np

    net = m2c.Mlp(np.load(os.path.join(ROOT, "paper_2508_16387_amd", "learned_guess_eos.npy")))

    def timed(fn):
        fn()
        ts, r = [], None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return sorted(ts)[len(ts) // 2], r

    def run(pairs):
        inp, mat, mats, _ = W.general_eos_problem_set(2024, n, pairs=pairs)
        ti = torch.tensor(inp, dtype=torch.float64, device="cuda")
        tm = torch.tensor(mat, dtype=torch.int32, device="cuda")
        T, (out, it, rc) = timed(lambda: m2c.riemann_solve_eos(ti, tm, mats))
        TL, (_, itl, _, nfb) = timed(lambda: m2c.riemann_solve_eos_learned(net, ti, tm, mats))
        ok, okl = it != 0, itl != 0
        return {"solves_per_s": n / T, "ms": T * 1e3, "calls": reps,
                "newton_iters_per_solve": float(it.abs().double()[ok].mean()), "no_star_state": int((~ok).sum()),
                "learned_start": {"solves_per_s": n / TL, "ms": TL * 1e3,
                                  "newton_iters_per_solve": float(itl.abs().double()[okl].mean()),
                                  "acoustic_starts": int(nfb), "speedup_vs_acoustic": T / TL}}

    res = {"problems": n, "ds": 0.01, "mixed_pairs": run(None)}
    no_mg = [pr for pr in W.EOS_PAIRS if all(W.EOS_MATERIALS[m][0] != m2c.M2C_EOS_MG for m in pr)]
    res["pairs_without_mie_grueneisen"] = run(no_mg)
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
    import numpy as np

    import workloads as W
    p = W.eos_charge(0, n=(128, 128, 128), steps=steps)
    rate, T = time_sim(m2c, torch, p, m2c.M2C_PREC_FP64, steps, 2)
    out = {"workload": "tnt_sphere_in_water_nasg_128", "steps": steps, "cell_updates_per_stage_per_s": rate,
           "ms_per_step": T / steps * 1e3}
    # FIVER of the same run from the acoustic and from the learned start
    # (library events around the kernels of every step)
    net = m2c.Mlp(np.load(os.path.join(ROOT, "paper_2508_16387_amd", "learned_guess_eos.npy")))
    for name, guess in (("acoustic", None), ("learned", net)):
        sim = m2c.Sim(m2c.config_for(p))
        sim.set_stream(torch.cuda.current_stream())
        if guess is not None:
            sim.set_guess(guess)
        sim.set_state(p.prim)
        sim.step(2)
        sim.set_state(p.prim)
        sim.reset_stats()
        sim.set_profiling(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        Ts = time.perf_counter() - t0
        st = sim.stats()
        out["fiver_" + name] = {"ms_per_step": Ts / steps * 1e3,
                                "fiver_ms_per_launch": st["ms_fiver"] / max(st["fiver_launches"], 1),
                                "newton_iters_per_solve": st["newton_iters"] / max(st["riemann_solves"], 1),
                                "acoustic_starts": st["mlp_fallbacks"] if guess is not None else None}
        sim.close()
    out["fiver_speedup_learned_vs_acoustic"] = (out["fiver_acoustic"]["fiver_ms_per_launch"] /
                                                out["fiver_learned"]["fiver_ms_per_launch"])
    return out


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


def mixed_vs_fp64(m2c, torch, problem, steps, warmup, value_fp64):
    """The mixed-precision form on the same workload and steps."""
    v, T = time_sim(m2c, torch, problem, m2c.M2C_PREC_MIXED, steps, warmup)
    return {"value": v, "ms_per_step": T * 1e3 / steps, "speedup_mixed_vs_fp64": v / value_fp64}


def second_workload(m2c, torch, name, seed, steps):
    """FP64 and mixed on the other workload, over its whole length."""
    p = make_problem(name, seed)
    out = {"workload": WORKLOADS[name], "steps": steps}
    for prec, key in ((m2c.M2C_PREC_FP64, "fp64"), (m2c.M2C_PREC_MIXED, "mixed")):
        v, T = time_sim(m2c, torch, p, prec, steps, 2)
        out[key] = {"value": v, "ms_per_step": T * 1e3 / steps}
    out["speedup_mixed_vs_fp64"] = out["mixed"]["value"] / out["fp64"]["value"]
    return out


def in_situ_guess(m2c, torch, problem, advance, steps):
    """The learned star-pressure guess in the grid step against the acoustic
    one, timed after ``advance`` untimed steps (by then the slab's shock has
    reached bubbles, so interface faces see real waves): FIVER kernel time
    per launch from the library's events, Newton steps per solve, faces that
    took the acoustic start."""
    import numpy as np

    net = m2c.Mlp(np.load(os.path.join(ROOT, "paper_2508_16387_amd", "learned_guess.npy")))
    sim = m2c.Sim(m2c.config_for(problem))
    sim.set_stream(torch.cuda.current_stream())
    sim.set_state(problem.prim)
    sim.step(advance)
    w0 = sim.get_conserved()
    out = {"advance_steps": advance, "steps_timed": steps}
    for name, guess in (("acoustic", None), ("learned", net)):
        sim.set_conserved(w0)
        sim.set_guess(guess)
        sim.reset_stats()
        sim.set_profiling(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        st = sim.stats()
        out[name] = {"ms_per_step": T * 1e3 / steps,
                     "fiver_ms_per_launch": st["ms_fiver"] / max(st["fiver_launches"], 1),
                     "riemann_solves": st["riemann_solves"],
                     "newton_iters_per_solve": st["newton_iters"] / max(st["riemann_solves"], 1),
                     "acoustic_starts": st["mlp_fallbacks"] if guess is not None else None}
    sim.set_profiling(0)
    sim.close()
    out["fiver_speedup_learned_vs_acoustic"] = (out["acoustic"]["fiver_ms_per_launch"] /
                                                out["learned"]["fiver_ms_per_launch"])
    return out


def learned_standalone(m2c, torch, n=1_000_000, reps=20):
    """Held-out water/air Riemann problems: Newton steps and solves/s with the
    judged learned guess against the acoustic guess, device time as the
    median of ``reps`` launches."""
    import numpy as np

    import workloads as W

    inp, eos = W.riemann_problem_set(2000, n)
    di = torch.tensor(inp.T.copy(), device="cuda")
    de = torch.tensor(eos.T.copy(), device="cuda")
    net = m2c.Mlp(np.load(os.path.join(ROOT, "paper_2508_16387_amd", "learned_guess.npy")))
    res = {"problems": n, "launches": reps}
    for name, guess in (("acoustic", None), ("learned", net)):
        out = torch.empty((4, n), dtype=torch.float64, device="cuda")
        it = torch.empty((n,), dtype=torch.int32, device="cuda")
        ms, _ = device_ms(torch, lambda: m2c.riemann_solve_learned_async(guess, di, de, out=out, iters=it), reps)
        _, _, _, nfb = m2c.riemann_solve_learned(guess, di, de)
        itd = it.abs().double()
        ok = itd > 0
        res[name] = {"solves_per_s": n / (ms * 1e-3), "ms": ms, "newton_iters_per_solve": float(itd[ok].mean()),
                     "acoustic_starts": int(nfb) if guess is not None else None}
    res["speedup_learned_vs_acoustic"] = res["learned"]["solves_per_s"] / res["acoustic"]["solves_per_s"]
    return res


def host_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"cpu_model": model, "nproc": avail, "os_cpu_count": os.cpu_count(),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def _slab(problem, nz):
    """The first nz z-planes of a problem as a problem of its own
    (transmissive at the cut)."""
    import copy
    q = copy.copy(problem)
    q.n = (problem.n[0], problem.n[1], nz)
    q.hi = (problem.hi[0], problem.hi[1], problem.lo[2] + (problem.hi[2] - problem.lo[2]) * nz / problem.n[2])
    q.prim = problem.prim[:, :nz].copy()
    return q


def cpu_baseline(problem, workload, steps=1):
    """The oracle on the host cores: the all-core (OpenMP) build on the whole
    grid and the single-threaded build on a slab of it, `steps` steps each,
    in the GPU metric's unit."""
    import oracle

    oracle.build(force=False)
    oracle.build(force=False, openmp=True)
    N = problem.ncells
    lib_omp = oracle.lib_openmp()
    threads = int(lib_omp.ora_num_threads())
    s = oracle.OracleSim(problem, lib_handle=lib_omp)
    t0 = time.perf_counter()
    rc = s.step(steps)
    t_all = time.perf_counter() - t0
    assert rc == 0
    del s
    progress(f"cpu baseline: all-core oracle step done ({t_all:.1f} s on {threads} threads)")
    nz1 = max(1, problem.n[2] // 8)
    q = _slab(problem, nz1)
    s1 = oracle.OracleSim(q)
    t0 = time.perf_counter()
    rc = s1.step(steps)
    t_one = time.perf_counter() - t0
    assert rc == 0
    del s1
    nx, ny, nz = problem.n
    # the general-EOS Riemann oracle on a sample of the mixed problem set
    import workloads as W
    from oracle import riemann_eos as RE

    ne = 64
    inp, mat, mats, _ = W.general_eos_problem_set(2024, ne)
    eos = [RE.make_eos(f, prm) for f, prm in mats]
    t0 = time.perf_counter()
    RE.solve(inp, mat, eos)
    te = time.perf_counter() - t0
    return {"value": N * steps * 2 / t_all, "unit": "cell-updates/s per RK stage", "cores": threads,
            "kind": "oracle",
            "sample": f"first {steps} step(s) of the {nx}x{ny}x{nz} {WORKLOADS[workload]} run, C oracle built "
                      f"with OpenMP on {threads} threads ({t_all:.1f} s)",
            "single_core": {"value": q.ncells * steps * 2 / t_one, "cores": 1,
                            "sample": f"first {steps} step(s) of the {nx}x{ny}x{nz1} bottom slab of the same "
                                      f"initial state, serial C oracle ({t_one:.1f} s)"},
            "host": host_info(),
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

    if args.workload == "charge_128" and args.precision == "mixed":
        sys.exit("the general-EOS workload runs in FP64 only")
    t_ic = time.perf_counter()
    p = make_problem(args.workload, args.seed)
    progress(f"initial state of {WORKLOADS[args.workload]} built ({time.perf_counter() - t_ic:.1f} s)")
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
    sim.set_profiling(0)
    N = p.ncells
    value = N * args.steps * 2 / T

    stage_ms = st["ms_stage"] / max(st["stage_launches"], 1)
    fiver_ms = st["ms_fiver"] / max(st["fiver_launches"], 1)
    bytes_per_launch = N * (BYTES_STAGE1 + BYTES_STAGE2) / 2
    traffic = measured_traffic(args.workload, args.precision)
    achieved = bytes_per_launch / (stage_ms * 1e-3) / 1e9
    valu = valu_line(measured_valu(args.workload, args.precision), N, stage_ms)
    hbm = {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
           "algorithmic_bytes_per_launch": bytes_per_launch, "traffic": traffic,
           "traffic_frac": (None if traffic is None else traffic / (stage_ms * 1e-3) / 1e9 / HBM_PEAK_GBS)}
    # the roof the stage kernel comes closest to: VALU issue (counted
    # instructions) when the counter record matches the sources, else HBM
    if valu is not None and valu["frac"] > (hbm["traffic_frac"] or hbm["frac"]):
        roof = {"bound": "alu", "achieved": valu["achieved"], "peak": VALU_PEAK, "unit": "lane-instructions/s",
                "frac": valu["frac"], "traffic": traffic, "valu_instr_per_cell": valu["instr_per_cell"], "hbm": hbm}
    else:
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_frac": hbm["traffic_frac"],
                "valu": valu}
    roof.update({"kernel": "k_stage (both RK stages)", "avg_launch_ms": stage_ms,
                 "algorithmic_bytes_per_launch": bytes_per_launch})
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
        "config": {"workload": WORKLOADS[args.workload], "grid": list(p.n), "steps": args.steps,
                   "workload_steps": p.steps, "precision": args.precision, "rk": "TVD-RK2", "cfl": p.cfl,
                   "seed": args.seed},
        "roofline": roof,
        "fiver": {"solves": st["riemann_solves"], "ms_per_launch": fiver_ms,
                  "solves_per_s": st["riemann_solves"] / (2 * args.steps) / max(fiver_ms * 1e-3, 1e-12),
                  "newton_iters_per_solve": st["newton_iters"] / max(st["riemann_solves"], 1)},
        "time_split_ms_per_step": {k: st[f"ms_{k}"] * 2 / max(st["stage_launches"], 1)
                                   for k in ("stage", "fiver", "other")},
    }
    progress(f"headline {WORKLOADS[args.workload]}: {value:.4g} cell-updates/s per stage, "
             f"stage kernel {stage_ms:.3f} ms per launch")
    if not args.no_forms:
        other = "shock_bubble_128" if args.workload == "cloud_384" else "cloud_384"
        forms = {}

        def form(name, fn, *a):
            t = time.perf_counter()
            forms[name] = fn(*a)
            progress(f"form {name} done ({time.perf_counter() - t:.1f} s)")

        if prec == m2c.M2C_PREC_FP64:
            form("mixed", mixed_vs_fp64, m2c, torch, p, args.steps, args.warmup, value)
        form("host_round_trip", host_round_trip, m2c, torch, p, args.steps)
        if args.workload == "cloud_384" and args.in_situ_advance > 0:
            form("in_situ_learned_guess", in_situ_guess, m2c, torch, p, args.in_situ_advance, 20)
        sim.close()
        form(other, second_workload, m2c, torch, other, args.seed, 100 if other == "shock_bubble_128" else 50)
        p128 = make_problem("shock_bubble_128", args.seed)
        form("batched", batched_forms, m2c, torch, args.batch_steps)
        form("fiver_standalone", fiver_standalone, m2c, torch)
        form("learned_guess_standalone", learned_standalone, m2c, torch)
        form("general_eos_riemann", general_eos_standalone, m2c, torch)
        form("reinit_128", reinit_form, m2c, torch, p128)
        form("general_eos_step_128", general_eos_step, m2c, torch)
        form("scheme_options_128", scheme_options, m2c, torch, p128)
        out["forms"] = forms
    else:
        sim.close()
    if not args.no_cpu_baseline and args.workload == "charge_128":
        # the oracle's general-EOS interface solves are Python (adaptive
        # isentropes): far beyond a bounded sample of this grid
        progress("cpu baseline skipped for the general-EOS workload")
    elif not args.no_cpu_baseline:
        t = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(p, args.workload)
        progress(f"cpu baseline done ({time.perf_counter() - t:.1f} s)")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
