"""GPU parity of long diagonal sweeps through the phase tables: the host
groups a sweep's phases by their tile-local condition (phase patterns, each
member with a predicate on the tile's outer index bits), splits sweeps with
more patterns than the LDS holds, and refreshes the phases of parameterised
gates before each run.  Checked against the oracle with two angle sets per
plan, through single-circuit plans and planned batches."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}


def _say(*a):
    print(*a, flush=True)


def _diag_sweeps(n, seed, ngates, layers=2, pfrac=0.4):
    """H on every qubit, then `layers` blocks of `ngates` diagonal gates (P
    and RZ, 0-3 controls with random values, targets anywhere, a fraction
    parameterised) separated by H on three qubits: long sweeps whose phases
    read every mix of tile-local and outer bits, with many distinct
    tile-local conditions."""
    rng = np.random.default_rng(seed)
    gates, p = [W.Gate("H", q) for q in range(n)], 0
    for layer in range(layers):
        for _ in range(ngates):
            t = int(rng.integers(0, n))
            others = [q for q in range(n) if q != t]
            k = int(rng.integers(0, 4))
            ctrls = tuple(int(q) for q in rng.choice(others, size=k, replace=False)) if k else ()
            vals = tuple(int(v) for v in rng.integers(0, 2, size=k)) if k else ()
            kind = "P" if rng.random() < 0.5 else "RZ"
            if rng.random() < pfrac:
                gates.append(W.Gate(kind, t, ctrls, vals, param=p))
                p += 1
            else:
                gates.append(W.Gate(kind, t, ctrls, vals, float(rng.uniform(0, 2 * np.pi))))
        for q in rng.choice(n, size=3, replace=False):
            gates.append(W.Gate("H", int(q)))
    return W.Circuit(n, gates, rng.uniform(0, 2 * np.pi, size=p), meta={"seed": seed})


def _err(got, ref):
    return float(np.max(np.abs(got.astype(np.complex128) - ref)))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,ngates", [(14, 120), (16, 1500)])
def test_long_sweeps_with_parameters(gpu, dtype, n, ngates):
    """Sweeps of 120 gates (a few hundred patterns) and of 1500 gates (more
    patterns than one sweep may hold, so the host splits it), parameterised
    phases refreshed between two runs with different angles."""
    import torch
    c = _diag_sweeps(n, 100 + n, ngates)
    psi0 = W.random_state(n, n)
    plan = gpu.Circuit(n, c, dtype=0 if dtype == "c128" else 1, nparams=c.nparams, flags=gpu.SV_FUSE)
    try:
        info = plan.info()
        assert info["passes"] < len(c.gates) // 10, info
        for rep in range(2):
            angles = c.params + 0.71 * rep
            ref = oracle.run_circuit(c, angles, psi0)
            d = torch.from_numpy(psi0).cuda()
            if dtype == "c64":
                d = d.to(torch.complex64)
            plan.run(d, torch.from_numpy(angles).cuda())
            e = _err(d.cpu().numpy(), ref)
            _say("n", n, "gates", len(c.gates), dtype, "rep", rep, "err", e)
            assert e <= TOL[dtype], (rep, e)
    finally:
        plan.close()


@pytest.mark.parametrize("tile", [7, 9])
def test_sweep_tables_small_tiles(gpu, tile):
    """The smallest table widths (one and three tile-local bits above the
    six of u), where B and D tables have fewer entries than lanes."""
    import torch
    gpu.sv_tune_set("tile_log2_c128", tile)
    n = 13
    c = _diag_sweeps(n, 7 + tile, 200)
    psi0 = W.random_state(n, 5)
    ref = oracle.run_circuit(c, c.params, psi0)
    d = torch.from_numpy(psi0).cuda()
    plan = gpu.Circuit(n, c, nparams=c.nparams, flags=gpu.SV_FUSE)
    try:
        plan.run(d, torch.from_numpy(c.params).cuda())
    finally:
        plan.close()
    assert _err(d.cpu().numpy(), ref) <= 1e-12


def test_batched_long_sweeps(gpu):
    """Planned batch of circuits with long parameterised sweeps (widths 13 to
    16, so every circuit runs fused passes from global memory), two runs with
    different angles, each circuit against the oracle."""
    import torch
    circs = [_diag_sweeps(n, 300 + i, 150 + 40 * i) for i, n in enumerate((13, 14, 15, 16, 14, 13))]
    ns = [c.n for c in circs]
    offs = np.concatenate([[0], np.cumsum([1 << n for n in ns])])
    buf = torch.zeros(int(offs[-1]), dtype=torch.complex128, device="cuda")
    views = [buf[int(offs[i]):int(offs[i + 1])] for i in range(len(circs))]
    b = gpu.Batch(views, circs)
    try:
        for rep in range(2):
            angles = [c.params - 0.53 * rep for c in circs]
            buf.zero_()
            for v in views:
                v[0] = 1
            b.run(torch.from_numpy(np.concatenate(angles)).cuda())
            for c, a, v in zip(circs, angles, views):
                e = _err(v.cpu().numpy(), oracle.run_circuit(c, a))
                assert e <= 1e-12, (rep, c.n, e)
    finally:
        b.close()
