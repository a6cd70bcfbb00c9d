"""Writes tests/golden/train_curve.json: the loss of the FP64 oracle network
trained by Adam (lr 1e-3, no TV term) on one fixed batch, at the steps the
GPU training test checks.  Calls only the oracle and the tests' seeded
generators.  Run: python tests/golden/make_train_curve.py"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

from oracle import net as onet  # noqa: E402
import test_net_parity as T  # noqa: E402

STEPS = (1, 20, 40, 60)


def main():
    B, H, W = 4, 32, 32
    P = T.random_net(13)
    rng = np.random.default_rng(14)
    planes = T.random_planes(rng, B, H, W)
    target = planes[:, :3].astype(np.float64)
    x = onet.features(planes)
    state, curve = {}, {}
    for s in range(1, max(STEPS) + 1):
        y, cache = onet.forward(P, x)
        L, g = onet.loss(y, target, lam_tv=0.0)
        if s in STEPS:
            curve[str(s)] = L
            print(s, L, flush=True)
        P = onet.adam(P, onet.backward(P, cache, g), state, lr=1e-3)
    rec = {"what": "FP64 oracle loss before Adam step k (k = 1 is the initial loss); batch 4x32x32 of "
                   "random_planes(seed 14), random_net(13), target = the RGB planes, lr 1e-3, lam_tv 0",
           "loss_before_step": curve}
    with open(os.path.join(HERE, "train_curve.json"), "w") as fh:
        json.dump(rec, fh, indent=1)


if __name__ == "__main__":
    main()
