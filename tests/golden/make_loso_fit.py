"""Writes loso_fit_16x128.json: the FP64 oracle's 200-step Adam fit of the
variogram on the leave-one-slice-out loss of the 16 x 128^2 correlated-field
workload (exponential model from (nugget, sill, range) = (0.1, 1.0, 2.0),
Adam on log theta, lr 0.05, betas (0.9, 0.999), eps 1e-8).

Calls only oracle/ and the workload generator. Each loss and gradient is the
mean over the held-out slices, evaluated one held-out slice per process
(slices s-1, s, s+1 hold out s); every held-out slice has the same number of
voxels, so the mean of the per-slice means is the loss over all of them.

    python tests/golden/make_loso_fit.py      # about half an hour on 8 cores
"""
import json
import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

_S = {}


def _one(args):
    s, theta = args
    L, g = O.loso_loss_grad(_S["slices"][s - 1:s + 2], 2, ("exponential", *theta))
    return L, g


def main():
    w = W.workload("loso_16x128")
    slices, _ = W.make_inputs(w)
    _S["slices"] = slices
    held = list(range(1, w.nslices - 1))
    with mp.get_context("fork").Pool(min(len(held), os.cpu_count() or 1)) as pool:
        def loss_grad(theta):
            res = pool.map(_one, [(s, tuple(float(x) for x in theta)) for s in held])
            L = float(np.mean([r[0] for r in res]))
            g = np.mean([r[1] for r in res], axis=0)
            print(f"loss {L:.12e} theta {theta}", flush=True)
            return L, g
        traj = O.adam_fit(loss_grad, (0.1, 1.0, 2.0), steps=200, lr=0.05)
    out = {"workload": w.name, "model": "exponential", "theta0": [0.1, 1.0, 2.0], "steps": 200,
           "lr": 0.05, "betas": [0.9, 0.999], "eps": 1e-8,
           "loss": [t[0] for t in traj], "theta": [[float(x) for x in t[1]] for t in traj]}
    with open(os.path.join(HERE, "loso_fit_16x128.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
