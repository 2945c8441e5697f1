"""Training data and training of the sample-count predictor (learned initial M and start
pruning), driven through the C ABI.

The paper leaves open how to choose the initial number of training states (Sec. 3,
Sec. 5) and relates the number needed to the parameter count per amplitude (Sec. 4).
Labels come from the method itself: for each problem, every start is run to its own
stop at fixed M = 2, 4, ..., 2^n (qfs_label_batch) until at least one start succeeds
and generalises (the Sec. 3 success relation). The label is (log2 of that M, the
fraction of starts that succeeded there); a problem with no success up to
min(2^n, 64) is labelled (NaN, 0). Features are the library's 64 template features.

Command line (runs on the GPU; writes the weight file loaded by qfs_mlp_load):
    python -m paper_2405_12866_amd.predictor --problems 6144 --out predictor.bin
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np

from . import inputs as I
from . import qfs as Q

DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "predictor.bin")


def label_params(**over):
    """Run settings of the labelling ladder (App. A defaults otherwise)."""
    d = dict(multistarts=16, dist_tol=1e-8, max_iter=400, batch_sweeps=0,
             precision=Q.QFS_PREC_MIXED)
    d.update(over)
    return d


def device_problems(problems, device="cuda"):
    import torch
    out = []
    for p in problems:
        out.append(dict(n=p["n"], pairs=p["pairs"], target_pairs=p["target_pairs"],
                        target_gates=torch.as_tensor(np.ascontiguousarray(p["target_gates"]),
                                                     dtype=torch.complex128).to(device)))
    return out


def training_problems(count, seed_base=0x5A17 + 5):
    """Three quarters drawn like the batched workload (n in 3..7, L in 2..20), one quarter
    larger (n in 8..10, L in 8..40); random distinct pairs, Haar target from the
    template."""
    small = I.batched_problems(count - count // 4, seed_base=seed_base)
    large = I.batched_problems(count // 4, seed_base=seed_base + 1, n_range=(8, 10), L_range=(8, 40))
    return small + large


def label(problems, params=None, seed=0x1AB, log=None, m_cap=64):
    """Labels [P][2] by the M ladder (M = 2, 4, ... up to min(2^n, m_cap)). ``problems``
    hold device target gates."""
    params = dict(params or label_params())
    S = params["multistarts"]
    P = len(problems)
    T = np.full((P, 2), np.nan, dtype=np.float32)
    T[:, 1] = 0.0
    todo = list(range(P))
    m = 2
    work = 0
    while todo:
        active = [i for i in todo if m <= min(1 << problems[i]["n"], m_cap)]
        if not active:
            break
        succ, infos = Q.qfs_label_batch([problems[i] for i in active],
                                        dict(params, m_init=m, seed=seed + m))
        work += sum(r["start_sweeps"] for r in infos)
        done = set()
        for j, i in enumerate(active):
            if succ[j] > 0:
                T[i, 0] = math.log2(m)
                T[i, 1] = succ[j] / S
                done.add(i)
        if log:
            log(f"label M={m}: {len(active)} problems, {len(done)} labelled")
        todo = [i for i in todo if i not in done and m < min(1 << problems[i]["n"], m_cap)]
        m *= 2
    return T, work


def features(problems):
    return np.stack([Q.qfs_features(p["n"], p["pairs"]) for p in problems]).astype(np.float32)


def train(X, T, epochs=300, batch=256, lr=2e-3, seed=7, init_seed=11):
    """Fresh weights trained on the device by the library's kernels; returns losses."""
    import torch
    Q.qfs_mlp_init(init_seed)
    xd = torch.as_tensor(X, dtype=torch.float32).contiguous().cuda()
    td = torch.as_tensor(T, dtype=torch.float32).contiguous().cuda()
    return Q.qfs_mlp_train(xd, td, epochs, min(batch, len(X)), lr, seed)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--problems", type=int, default=6144)
    ap.add_argument("--seed-base", type=int, default=0x5A17 + 5)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--save-data", default=None, help="optional .npz with X, T")
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    probs = training_problems(a.problems, seed_base=a.seed_base)
    dprobs = device_problems(probs)
    T, work = label(dprobs, log=log)
    X = features(probs)
    log(f"labelled {len(probs)} problems ({len(probs) * 16} runs, {work} start-sweeps) "
        f"in {time.perf_counter() - t0:.1f} s")
    if a.save_data:
        np.savez(a.save_data, X=X, T=T)
    losses = train(X, T, epochs=a.epochs)
    log(f"trained {a.epochs} epochs: loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    Q.qfs_mlp_save(a.out)
    log(f"wrote {a.out}")


if __name__ == "__main__":
    main()
