"""Write hea_batch_n16_param_shift.json: the oracle's loss and full
parameter-shift gradient (all 128 parameters) for 8 seeded circuits of the
batched-gradient workload (256 ansatz circuits at n=16, 4 layers, each with
its own angles and ZZ+X Hamiltonian; workloads.hea_batch_n16, seed 7).

Calls only the oracle and the seeded input generators (no GPU code).  Run
from the repository root:

    python tests/golden/make_hea_batch_n16_grads.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def sample(ncirc=256, count=8, seed=1616):
    rng = np.random.default_rng(seed)
    return sorted(rng.choice(ncirc, size=count, replace=False).tolist())


def main():
    pairs = W.hea_batch_n16()
    t0 = time.time()
    out = {"problem": "batched ansatz circuits at n=16, 4 layers, 128 parameters each (workloads.hea_batch_n16, "
                      "seed 7)",
           "method": "oracle loss and parameter-shift rule over all 128 parameters",
           "script": "tests/golden/make_hea_batch_n16_grads.py", "circuits": []}
    for ci in sample(len(pairs)):
        c, h = pairs[ci]
        loss = oracle.loss(c, c.params, h)
        g = oracle.grad_param_shift(c, c.params, h)
        out["circuits"].append({"index": ci, "loss": loss, "grad": g.tolist()})
        print("circuit %3d loss %+.12f |g|max %.3e (%.0f s)" % (ci, loss, np.abs(g).max(), time.time() - t0),
              flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hea_batch_n16_param_shift.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
