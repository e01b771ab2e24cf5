"""GPU parity of the batched entry points against the oracle: mixed-width
batches (LDS-resident and global-memory circuits), the 4096-circuit batch at full size on
a seeded sample of circuits, batched adjoint gradients, and planned batches
(sv_batch_*) run repeatedly."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _packed_states(ns, dtype):
    """One device buffer holding every state (|0..0> each) and views into it."""
    import torch
    td = torch.complex128 if dtype == "c128" else torch.complex64
    sizes = [1 << n for n in ns]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    buf = torch.zeros(int(offs[-1]), dtype=td, device="cuda")
    idx = torch.from_numpy(offs[:-1].astype(np.int64)).cuda()
    buf[idx] = 1
    views = [buf[int(offs[i]):int(offs[i + 1])] for i in range(len(ns))]
    return buf, views


def _err(got, ref):
    return float(np.max(np.abs(got.astype(np.complex128) - ref)) / np.max(np.abs(ref)))


def _mixed(seed, ncirc=40):
    rng = np.random.default_rng(seed)
    circs = []
    for i in range(ncirc):
        n = int(rng.integers(2, 17))
        c = W.random_gates_n12(seed=seed * 1000 + i, n=n, ngates=int(rng.integers(20, 120)))
        # turn some rotations into parameterised gates
        gates, p = [], 0
        for g in c.gates:
            if g.kind in ("RY", "RZ") and rng.random() < 0.5:
                gates.append(W.Gate(g.kind, g.target, g.controls, g.values, param=p)); p += 1
            else:
                gates.append(g)
        circs.append(W.Circuit(n, gates, rng.uniform(0, 2 * np.pi, size=p)))
    return circs


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("tile", [12, 7])
def test_batched_mixed_widths(gpu, dtype, tile):
    import torch
    gpu.sv_tune_set("tile_log2_c128", tile)
    gpu.sv_tune_set("tile_log2_c64", tile + 1)
    try:
        circs = _mixed(3)
        buf, views = _packed_states([c.n for c in circs], dtype)
        params = torch.from_numpy(np.concatenate([c.params for c in circs])).cuda()
        gpu.sv_apply_circuits_batched(views, circs, params)
        worst = 0.0
        for c, v in zip(circs, views):
            ref = oracle.run_circuit(c, c.params)
            e = _err(v.cpu().numpy(), ref)
            worst = max(worst, e)
            assert e <= (1e-12 if dtype == "c128" else 1e-5), (c.n, e)
        _say("batched", dtype, "tile", tile, "worst", worst)
    finally:
        gpu.sv_tune_set("tile_log2_c128", 12)
        gpu.sv_tune_set("tile_log2_c64", 13)


def test_batched_errors_name_circuit(gpu):
    import torch
    circs = [W.random_gates_n12(n=5, ngates=10), W.Circuit(5, [W.Gate("X", 7)])]
    buf, views = _packed_states([5, 5], "c128")
    before = buf.clone()
    with pytest.raises(gpu.SvError) as e:
        gpu.sv_apply_circuits_batched(views, circs)
    assert "circuit 1" in str(e.value)
    torch.cuda.synchronize()
    assert torch.equal(buf, before)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_uneven_batch_full_sampled(gpu, dtype):
    """4096 circuits, n uniform in 10..20, 100-400 gates each
    (12.5 GB of complex128 states); 24 seeded circuits and one of every width
    checked against the oracle, every state's norm checked on the device."""
    import torch
    circs = W.uneven_batch()
    _say("uneven batch", dtype, "states", sum(1 << c.n for c in circs) * (16 if dtype == "c128" else 8) / 2 ** 30, "GiB")
    buf, views = _packed_states([c.n for c in circs], dtype)
    torch.cuda.synchronize()
    gpu.sv_apply_circuits_batched(views, circs)
    torch.cuda.synchronize()
    rng = np.random.default_rng(17)
    sample = sorted(rng.choice(len(circs), size=24, replace=False).tolist())
    big = [next(i for i, c in enumerate(circs) if c.n == nq) for nq in range(10, 21)]  # every width once
    tol = 1e-12 if dtype == "c128" else 1e-5
    for i in sample + big:
        ref = oracle.run_circuit(circs[i])
        e = _err(views[i].cpu().numpy(), ref)
        _say("uneven batch circuit", i, "n", circs[i].n, "err", e)
        assert e <= tol
    norms = torch.stack([v.abs().pow(2).sum() for v in views]).double()
    assert float((norms - 1).abs().max()) <= (1e-12 if dtype == "c128" else 1e-4)


def test_batched_adjoint_small(gpu):
    import torch
    circs, hams = [], []
    for i in range(10):
        n = 3 + i % 7
        c = W.hea(n, 2, seed=200 + i)
        circs.append(c)
        hams.append(W.zz_x_hamiltonian(n, 300 + i))
    buf, views = _packed_states([c.n for c in circs], "c128")
    params = torch.from_numpy(np.concatenate([c.params for c in circs])).cuda()
    gpu.sv_apply_circuits_batched(views, circs, params)
    lbuf = torch.empty_like(buf)
    lviews = []
    off = 0
    for c in circs:
        lviews.append(lbuf[off:off + (1 << c.n)]); off += 1 << c.n
    grad, loss = gpu.sv_adjoint_grad_batched(views, lviews, circs, params, hams)
    g = grad.cpu().numpy()
    L = loss.cpu().numpy()
    off = 0
    for i, (c, h) in enumerate(zip(circs, hams)):
        ref = oracle.grad_param_shift(c, c.params, h)
        got = g[off:off + c.nparams]
        off += c.nparams
        assert np.max(np.abs(got - ref)) <= 1e-8 * max(1, np.max(np.abs(ref))), i
        assert abs(L[i] - oracle.loss(c, c.params, h)) <= 1e-12 * 20
        back = views[i].cpu().numpy()
        assert abs(back[0] - 1) <= 1e-12 and np.max(np.abs(back[1:])) <= 1e-12


def test_hea_batch_n16_full_size(gpu):
    """256 ansatz circuits at n=16, 4 layers (128 parameters each): batched
    forward and batched adjoint; 8 seeded circuits checked on all 128
    gradients and the loss against the oracle's parameter shift stored by
    tests/golden/make_hea_batch_n16_grads.py; every circuit's psi back at
    |0...0> after the reverse sweep."""
    import torch
    pairs = W.hea_batch_n16()
    circs = [c for c, _ in pairs]
    hams = [h for _, h in pairs]
    buf, views = _packed_states([c.n for c in circs], "c128")
    lbuf = torch.empty_like(buf)
    lviews = [lbuf[i << 16:(i + 1) << 16] for i in range(len(circs))]
    params = torch.from_numpy(np.concatenate([c.params for c in circs])).cuda()
    gpu.sv_apply_circuits_batched(views, circs, params)
    grad, loss = gpu.sv_adjoint_grad_batched(views, lviews, circs, params, hams)
    g = grad.cpu().numpy()
    L = loss.cpu().numpy()
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "hea_batch_n16_param_shift.json")) as fh:
        gold = json.load(fh)
    assert len(gold["circuits"]) == 8
    for rec in gold["circuits"]:
        ci = rec["index"]
        ref = np.array(rec["grad"])
        got = g[ci * 128:(ci + 1) * 128]
        e = np.max(np.abs(got - ref)) / max(1.0, np.max(np.abs(ref)))
        _say("hea batch circuit", ci, "grad err", e)
        assert e <= 1e-8
        assert abs(L[ci] - rec["loss"]) <= 1e-10
    back = buf.view(len(circs), 1 << 16)
    e0 = torch.zeros_like(back)
    e0[:, 0] = 1
    assert float((back - e0).abs().max()) <= 1e-12


def test_batch_object_reuse(gpu):
    """A planned batch (sv_batch_create) run twice with different angles on
    re-initialised states, each run against the oracle; a forward-only batch
    refuses gradients."""
    import torch
    circs = _mixed(5, ncirc=24)
    buf, views = _packed_states([c.n for c in circs], "c128")
    init = buf.clone()
    b = gpu.Batch(views, circs)
    try:
        for rep in range(2):
            angles = [c.params + 0.37 * rep for c in circs]
            params = torch.from_numpy(np.concatenate(angles)).cuda()
            buf.copy_(init)
            b.run(params)
            for c, a, v in zip(circs, angles, views):
                e = _err(v.cpu().numpy(), oracle.run_circuit(c, a))
                assert e <= 1e-12, (rep, c.n, e)
    finally:
        b.close()
    with pytest.raises(gpu.SvError):
        gpu.Batch(views, circs).adjoint(params)  # created without lambda states


def test_batch_object_adjoint(gpu):
    import torch
    circs, hams = [], []
    for i in range(8):
        n = 4 + i % 5
        circs.append(W.hea(n, 2, seed=400 + i))
        hams.append(W.zz_x_hamiltonian(n, 500 + i))
    buf, views = _packed_states([c.n for c in circs], "c128")
    init = buf.clone()
    lbuf = torch.empty_like(buf)
    lviews, off = [], 0
    for c in circs:
        lviews.append(lbuf[off:off + (1 << c.n)]); off += 1 << c.n
    params = torch.from_numpy(np.concatenate([c.params for c in circs])).cuda()
    b = gpu.Batch(views, circs, lam_states=lviews, hamiltonians=hams)
    try:
        for rep in range(2):
            buf.copy_(init)
            b.run(params)
            grad, loss = b.adjoint(params)
            g = grad.cpu().numpy()
            off = 0
            for i, (c, h) in enumerate(zip(circs, hams)):
                ref = oracle.grad_param_shift(c, c.params, h)
                got = g[off:off + c.nparams]
                off += c.nparams
                assert np.max(np.abs(got - ref)) <= 1e-8 * max(1, np.max(np.abs(ref))), (rep, i)
                assert abs(loss[i].item() - oracle.loss(c, c.params, h)) <= 1e-10
    finally:
        b.close()


def test_batched_qubit_set_tiles(gpu):
    """Circuits of 13-15 qubits whose gates target every qubit: the fused
    plan's tiles span the low qubits plus planner-chosen high ones."""
    import torch
    circs = []
    for i in range(6):
        n = 13 + i % 3
        circs.append(W.random_gates_n12(seed=900 + i, n=n, ngates=150))
    for dtype, tol in (("c128", 1e-12), ("c64", 1e-5)):
        buf, views = _packed_states([c.n for c in circs], dtype)
        gpu.sv_apply_circuits_batched(views, circs)
        for c, v in zip(circs, views):
            e = _err(v.cpu().numpy(), oracle.run_circuit(c))
            assert e <= tol, (dtype, c.n, e)


def test_batch_with_empty_circuits(gpu):
    """Circuits without gates (LDS-resident and global-memory sizes) leave
    their states untouched while the others in the same batch run."""
    import torch
    circs = [W.Circuit(9, []), W.random_gates_n12(seed=31, n=9, ngates=50), W.Circuit(14, []),
             W.random_gates_n12(seed=32, n=14, ngates=120)]
    psis = [W.random_state(c.n, 40 + i) for i, c in enumerate(circs)]
    views = [torch.from_numpy(p).cuda() for p in psis]
    gpu.sv_apply_circuits_batched(views, circs)
    for c, p, v in zip(circs, psis, views):
        ref = oracle.run_circuit(c, None, p) if c.gates else p
        assert _err(v.cpu().numpy(), ref) <= 1e-12, (c.n, len(c.gates))


def test_batch_mixed_operations_forward_and_gradients(gpu):
    """A batch of circuits mixing controlled gates, diagonal-heavy blocks and
    parameterised rotations (n = 8..15): forward states and, through a
    planned batch, gradients against the oracle."""
    import torch
    from tests.test_circuit_gpu import _mixed_circuit
    circs, hams = [], []
    for i in range(8):
        n = 8 + i
        circs.append(_mixed_circuit(n, 70 + i))
        hams.append(W.zz_x_hamiltonian(n, 80 + i))
    buf, views = _packed_states([c.n for c in circs], "c128")
    init = buf.clone()
    lbuf = torch.empty_like(buf)
    lviews, off = [], 0
    for c in circs:
        lviews.append(lbuf[off:off + (1 << c.n)]); off += 1 << c.n
    params = torch.from_numpy(np.concatenate([c.params for c in circs])).cuda()
    b = gpu.Batch(views, circs, lam_states=lviews, hamiltonians=hams)
    try:
        b.run(params)
        for c, v in zip(circs, views):
            assert _err(v.cpu().numpy(), oracle.run_circuit(c, c.params)) <= 1e-12, c.n
        grad, loss = b.adjoint(params)
        g = grad.cpu().numpy()
        off = 0
        rng = np.random.default_rng(5)
        for i, (c, h) in enumerate(zip(circs, hams)):
            which = sorted(rng.choice(c.nparams, size=4, replace=False).tolist())
            ref = oracle.grad_param_shift(c, c.params, h, which=which)
            got = g[off + np.array(which)]
            off += c.nparams
            assert np.max(np.abs(got - ref)) <= 1e-8 * max(1, np.max(np.abs(ref))), (i, got, ref)
            assert abs(loss[i].item() - oracle.loss(c, c.params, h)) <= 1e-10
    finally:
        b.close()
