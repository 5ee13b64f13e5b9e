"""Train the learned star-pressure guess shipped with the package.

Labels come from the CPU oracle's exact two-material Riemann solver (Newton
to rtol 1e-14, every label a root of g(p) = 0 of the stiffened-gas wave
curves); inputs from the seeded water/air problem set (pressure ratios
log-uniform in [1, 1e4], density ratios log-uniform in [1, 1e3], half of the
problems with a velocity jump).  Training runs on the GPU with the
library's own BF16-MFMA forward/backward kernels and Adam.

Run from the repository root on a machine with an MI355X:
    python tests/golden/train_learned_guess.py [n_train] [epochs] [copy_dir]
Writes paper_2508_16387_amd/learned_guess.npy (4801 float32 parameters)
and learned_guess.json (data set, schedule, loss history) beside it.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)


def main():
    import torch

    import oracle
    import paper_2508_16387_amd as m2c
    import workloads as W

    n = int(sys.argv[1]) if len(sys.argv) > 1 else 1_000_000
    epochs = int(sys.argv[2]) if len(sys.argv) > 2 else 200
    lr0, lr1 = 5e-3, 2e-5
    t0 = time.time()
    inp, eos = W.riemann_problem_set(1000, n)
    out, _, bad = oracle.riemann_many(inp, eos, rtol=1e-14)
    ok = np.isfinite(out[:, 0])
    inp, eos, out = inp[ok], eos[ok], out[ok]
    print(f"labelled {ok.sum()} problems ({bad} without admissible star pressure) in {time.time() - t0:.1f} s",
          flush=True)
    dev = "cuda"
    X, t = m2c.mlp_features(torch.tensor(inp.T.copy(), device=dev), torch.tensor(eos.T.copy(), device=dev),
                            torch.tensor(out[:, 0].copy(), device=dev))
    net = m2c.Mlp(seed=1)
    t1 = time.time()
    hist = net.train(X, t, epochs=epochs, batch=4096, lr=lr0, lr_final=lr1)
    torch.cuda.synchronize()
    ttrain = time.time() - t1
    print("loss per epoch", [float(h) for h in hist], f"({ttrain:.1f} s)", flush=True)
    theta = net.params()
    # held-out evaluation: Newton steps from the judged learned guess vs the
    # acoustic guess, and agreement of the star pressure with the oracle
    hin, heos = W.riemann_problem_set(2000, 100_000)
    hout, _, _ = oracle.riemann_many(hin, heos, rtol=1e-14)
    ok2 = np.isfinite(hout[:, 0])
    hin, heos, hout = hin[ok2], heos[ok2], hout[ok2]
    di = torch.tensor(hin.T.copy(), device=dev)
    de = torch.tensor(heos.T.copy(), device=dev)
    o_l, i_l, _, nfb = m2c.riemann_solve_learned(net, di, de)
    o_a, i_a, _, _ = m2c.riemann_solve_learned(None, di, de)
    plo = -np.minimum(heos[:, 1], heos[:, 3])
    dev_l = float(np.max(np.abs(o_l.cpu().numpy()[0] - hout[:, 0]) / (hout[:, 0] - plo)))
    it_l = float(np.abs(i_l.cpu().numpy()).mean())
    it_a = float(np.abs(i_a.cpu().numpy()).mean())
    print(f"held-out: Newton steps learned {it_l:.3f} acoustic {it_a:.3f}, acoustic starts {nfb}, "
          f"max rel p* deviation {dev_l:.2e}", flush=True)
    pkg = os.path.join(ROOT, "paper_2508_16387_amd")
    np.save(os.path.join(pkg, "learned_guess.npy"), theta)
    meta = {"problems": int(ok.sum()), "problem_set_seed": 1000, "epochs": epochs, "batch": 4096,
            "lr": [lr0, lr1], "loss_per_epoch": [float(h) for h in hist], "train_seconds": ttrain,
            "labels": "CPU oracle Newton, rtol 1e-14",
            "held_out": {"problems": int(ok2.sum()), "seed": 2000, "newton_steps_learned": it_l,
                         "newton_steps_acoustic": it_a, "acoustic_starts": int(nfb),
                         "max_rel_pstar_deviation": dev_l}}
    with open(os.path.join(pkg, "learned_guess.json"), "w") as f:
        json.dump(meta, f, indent=1)
    # optional third argument: a directory that receives a copy of both files
    out_dir = sys.argv[3] if len(sys.argv) > 3 else None
    if out_dir:
        os.makedirs(out_dir, exist_ok=True)
        np.save(os.path.join(out_dir, "learned_guess.npy"), theta)
        with open(os.path.join(out_dir, "learned_guess.json"), "w") as f:
            json.dump(meta, f, indent=1)


if __name__ == "__main__":
    main()
