"""Train the learned start of the general-EOS Riemann solver shipped with
the package.

Labels are the star pressures of the library's general-EOS solver at rtol
1e-12: roots of the outer equation F(p) = f_L(p) + f_R(p) + u_R - u_L = 0.
The learned start only decides where that iteration begins; the solver runs
to the same tolerance from either start, so no result depends on the
labels' source beyond the stopping tolerance (the tests compare the learned
solves with the acoustic ones and with the independent Python oracle).
Inputs: the seeded general-EOS problem set restricted to the material
pairs the solver consults the network for (a JWL side, no Mie-Grueneisen
side), random left/right order.
Training runs on the GPU with the library's BF16-MFMA kernels and Adam.

Run from the repository root on a machine with an MI355X:
    python tests/golden/train_learned_guess_eos.py [n_train] [epochs] [copy_dir]
Writes paper_2508_16387_amd/learned_guess_eos.npy (4801 float32
parameters) and learned_guess_eos.json (data set, schedule, loss history,
held-out Newton steps and times) beside it.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)


def _median_call(fn, reps=5):
    import torch
    ts, res = [], None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2], res


def main():
    import torch

    import paper_2508_16387_amd as m2c
    import workloads as W

    n = int(sys.argv[1]) if len(sys.argv) > 1 else 1_000_000
    epochs = int(sys.argv[2]) if len(sys.argv) > 2 else 200
    lr0, lr1 = 5e-3, 2e-5
    dev = "cuda"
    t0 = time.time()
    fam = {m: W.EOS_MATERIALS[m][0] for m in W.EOS_MATERIALS}
    no_mg = [pr for pr in W.EOS_PAIRS if all(fam[m] != m2c.M2C_EOS_MG for m in pr)]
    pairs = [pr for pr in no_mg if any(fam[m] == m2c.M2C_EOS_JWL for m in pr)]
    inp, mat, mats, names = W.general_eos_problem_set(3000, n, pairs=pairs)
    ti = torch.tensor(inp, dtype=torch.float64, device=dev)
    tm = torch.tensor(mat, dtype=torch.int32, device=dev)
    out, it, _ = m2c.riemann_solve_eos(ti, tm, mats, rtol=1e-12)
    X, t = m2c.mlp_features_eos(ti, tm, mats, pstar=out[0].contiguous())
    keep = (it != 0) & torch.isfinite(t)
    X, t = X[:, keep].contiguous(), t[keep].contiguous()
    print(f"labelled {int(keep.sum())} of {n} problems ({names}) in {time.time() - t0:.1f} s", flush=True)
    net = m2c.Mlp(seed=2)
    t1 = time.time()
    hist = net.train(X, t, epochs=epochs, batch=4096, lr=lr0, lr_final=lr1)
    torch.cuda.synchronize()
    ttrain = time.time() - t1
    print("loss per epoch", [round(float(h), 5) for h in hist[:: max(1, epochs // 20)]], float(hist[-1]),
          f"({ttrain:.1f} s)", flush=True)
    theta = net.params()
    # held-out: Newton steps and time of the learned and the acoustic start
    held = {}
    for label, hpairs, seed in (("mixed_pairs", None, 4000), ("without_mie_grueneisen", no_mg, 4001),
                                ("with_jwl_without_mie_grueneisen", pairs, 4005),
                                ("tnt-air", [("tnt", "air")], 4002), ("water_nasg-gas_nasg", [("water_nasg", "gas_nasg")], 4003),
                                ("copper-tantalum", [("copper", "tantalum")], 4004)):
        hin, hmat, hmats, _ = W.general_eos_problem_set(seed, 1 << 18, pairs=hpairs)
        hi = torch.tensor(hin, dtype=torch.float64, device=dev)
        hm = torch.tensor(hmat, dtype=torch.int32, device=dev)
        ta, (oa, ia, _, _) = _median_call(lambda: m2c.riemann_solve_eos_learned(None, hi, hm, hmats))
        tl, (ol, il, _, nfb) = _median_call(lambda: m2c.riemann_solve_eos_learned(net, hi, hm, hmats))
        ok = (ia != 0) & (il != 0)
        rel = ((ol[0] - oa[0]).abs() / oa[0].abs().clamp_min(1e5))[ok]
        held[label] = {"problems": int(hi.shape[1]), "seed": seed,
                       "newton_steps_acoustic": float(ia[ok].abs().double().mean()),
                       "newton_steps_learned": float(il[ok].abs().double().mean()),
                       "acoustic_starts": int(nfb), "ms_acoustic": ta * 1e3, "ms_learned": tl * 1e3,
                       "speedup": ta / tl, "max_rel_pstar_difference": float(rel.max())}
        print(label, held[label], flush=True)
    pkg = os.path.join(ROOT, "paper_2508_16387_amd")
    meta = {"problems": int(keep.sum()), "problem_set_seed": 3000, "pairs": ["-".join(pr) for pr in pairs],
            "epochs": epochs, "batch": 4096, "lr": [lr0, lr1], "loss_per_epoch": [float(h) for h in hist],
            "train_seconds": ttrain, "labels": "library general-EOS solver, rtol 1e-12", "held_out": held}
    dirs = [pkg] + ([sys.argv[3]] if len(sys.argv) > 3 else [])
    for d in dirs:
        os.makedirs(d, exist_ok=True)
        np.save(os.path.join(d, "learned_guess_eos.npy"), theta)
        with open(os.path.join(d, "learned_guess_eos.json"), "w") as f:
            json.dump(meta, f, indent=1)


if __name__ == "__main__":
    main()
