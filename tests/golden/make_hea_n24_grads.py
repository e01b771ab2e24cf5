"""Write hea_n24_param_shift.json: the oracle's loss and parameter-shift
gradient of the n=24 ansatz problem (16 layers of RY and RZ on every qubit
plus a CNOT chain, 768 parameters, H = sum a_i Z_i Z_{i+1} + b_i X_i; seed 5)
for 32 seeded parameters spread over the first, two middle and the last
layers, RY and RZ alike.

Calls only the oracle and the seeded input generators (no GPU code).  About
65 forward passes of 1136 gates over 2^24 amplitudes: some 20 minutes on 8
cores.  Run from the repository root:

    python tests/golden/make_hea_n24_grads.py
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

LAYERS = (0, 5, 10, 15)
PER_KIND = 4  # RY and RZ parameters per layer


def sample(n=24, seed=2424):
    """Parameter p of layer l on qubit q is 2n l + 2q (RY) or 2n l + 2q + 1 (RZ)."""
    rng = np.random.default_rng(seed)
    idx = []
    for layer in LAYERS:
        for kind in (0, 1):
            for q in sorted(rng.choice(n, size=PER_KIND, replace=False).tolist()):
                idx.append(2 * n * layer + 2 * q + kind)
    return idx


def main():
    c, terms = W.hea_problem_n24()
    idx = sample(c.n)
    t0 = time.time()
    loss = oracle.loss(c, c.params, terms)
    print("loss %.15f (%.0f s)" % (loss, time.time() - t0), flush=True)
    grads = []
    for k, j in enumerate(idx):
        g = float(oracle.grad_param_shift(c, c.params, terms, which=[j])[0])
        grads.append(g)
        print("%2d/%d param %3d grad %+.15f (%.0f s)" % (k + 1, len(idx), j, g, time.time() - t0), flush=True)
    out = {"problem": "n=24 ansatz, 16 layers, 768 parameters, ZZ+X Hamiltonian (workloads.hea_problem_n24, seed 5)",
           "method": "oracle loss and parameter-shift rule (plain loop over all 2^24 indices per gate)",
           "script": "tests/golden/make_hea_n24_grads.py",
           "loss": loss, "params": idx, "grad": grads}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hea_n24_param_shift.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
