"""GPU parity of batched circuits split over several workgroups.  A forward
circuit whose cost is well above the batch's mean per workgroup is cut into
chunks of whole tiles (fused passes) or whole pair-loop steps (single gates)
that the workgroups joining it take in program order.  Each tile and pair is
computed exactly as by one workgroup, so the split must not change a single
bit of any state; the states are also checked against the oracle."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}


def _say(*a):
    print(*a, flush=True)


def _circuits(seed, ns, ngates=160, pfrac=0.4):
    """Random circuits (H, rotations, controlled gates) with a share of
    parameterised rotations; n = 13..18 run from global memory, smaller ones
    stay in LDS."""
    rng = np.random.default_rng(seed)
    circs = []
    for i, n in enumerate(ns):
        c = W.random_gates_n12(seed=seed * 100 + i, n=n, ngates=ngates)
        gates, p = [], 0
        for g in c.gates:
            if g.kind in ("RY", "RZ", "RX") and rng.random() < pfrac:
                gates.append(W.Gate(g.kind, g.target, g.controls, g.values, param=p))
                p += 1
            else:
                gates.append(g)
        circs.append(W.Circuit(n, gates, rng.uniform(0, 2 * np.pi, size=p)))
    return circs


def _buffer(ns, dtype):
    import torch
    td = torch.complex128 if dtype == "c128" else torch.complex64
    offs = np.concatenate([[0], np.cumsum([1 << n for n in ns])])
    buf = torch.zeros(int(offs[-1]), dtype=td, device="cuda")
    views = [buf[int(offs[i]):int(offs[i + 1])] for i in range(len(ns))]
    return buf, views, offs


def _reset(buf, offs):
    import torch
    buf.zero_()
    buf[torch.from_numpy(offs[:-1].astype(np.int64)).cuda()] = 1


def _run(gpu, circs, dtype, split, angle_sets):
    """Plan the batch with the given split limit, run it once per angle set
    (re-initialising the states), and return the batch's work items and the
    final buffers of every run."""
    import torch
    gpu.sv_tune_set("batch_split", split)
    buf, views, offs = _buffer([c.n for c in circs], dtype)
    b = gpu.Batch(views, circs)
    try:
        items = b.items()
        outs = []
        for angles in angle_sets:
            _reset(buf, offs)
            b.run(torch.from_numpy(np.concatenate(angles)).cuda())
            torch.cuda.synchronize()
            outs.append(buf.clone())
        assert b.wait_timeouts() == 0
    finally:
        b.close()
    return items, outs, offs


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("single", [False, True], ids=["fused", "single_gates"])
def test_split_is_bit_identical(gpu, dtype, single):
    """Two runs with different angles: the batch planned with every circuit
    on one workgroup and planned with splits up to 8 workgroups give equal
    bits; a sample of circuits is checked against the oracle.  single: no
    fused runs (fuse_min_gates above any run), so every pass of the split
    circuits is a chunked pair loop over global memory."""
    if single:
        gpu.sv_tune_set("fuse_min_gates", 1 << 20)
    ns = [16, 13, 17, 9, 14, 15, 11, 16]
    circs = _circuits(5 + int(single), ns, ngates=60 if single else 160)
    angle_sets = [[c.params for c in circs], [c.params + 0.37 for c in circs]]
    items1, out1, offs = _run(gpu, circs, dtype, 1, angle_sets)
    items8, out8, _ = _run(gpu, circs, dtype, 8, angle_sets)
    assert sorted(items1) == list(range(len(circs)))
    split = sorted({c for c in items8 if items8.count(c) > 1})
    _say(dtype, "single" if single else "fused", "items", len(items8), "split circuits", split)
    assert split, "no circuit was split"
    assert all(ns[c] >= (13 if dtype == "c128" else 14) for c in split)  # LDS-resident ones never are
    for rep in range(2):
        eq = bool((out1[rep] == out8[rep]).all())
        assert eq, ("split changed bits", rep)
    for i in (0, 2, 5):
        ref = oracle.run_circuit(circs[i], angle_sets[1][i])
        got = out8[1][int(offs[i]):int(offs[i + 1])].cpu().numpy().astype(np.complex128)
        e = float(np.max(np.abs(got - ref)))
        _say("circuit", i, "n", ns[i], "err", e)
        assert e <= TOL[dtype]


def test_lone_wide_circuit_many_workgroups(gpu):
    """A batch of one n=18 circuit: the whole split limit joins it (64
    workgroups, more than most passes have chunks), against the oracle."""
    import torch
    circs = _circuits(41, [18], ngates=200)
    items, outs, offs = _run(gpu, circs, "c128", 64, [[circs[0].params]])
    assert items == [0] * 64
    ref = oracle.run_circuit(circs[0], circs[0].params)
    e = float(np.max(np.abs(outs[0].cpu().numpy() - ref)))
    _say("lone n=18 err", e)
    assert e <= 1e-12


def test_item_stamps(gpu):
    """Per-item clock stamps of a split batch: every item has a start and an
    end no earlier than it, and a split circuit's items overlap in time."""
    import torch
    gpu.sv_tune_set("batch_split", 8)
    circs = _circuits(77, [17, 16, 12, 15], ngates=200)
    buf, views, offs = _buffer([c.n for c in circs], "c128")
    _reset(buf, offs)
    b = gpu.Batch(views, circs)
    try:
        items = b.items()
        stamps = torch.zeros(2 * max(len(items), len(circs)), dtype=torch.int64, device="cuda")
        b.set_timing(stamps)
        b.run(torch.from_numpy(np.concatenate([c.params for c in circs])).cuda())
        torch.cuda.synchronize()
        b.set_timing(None)
        assert b.wait_timeouts() == 0
    finally:
        b.close()
    st = stamps.cpu().numpy()[:2 * len(items)]
    t0, t1 = st[0::2], st[1::2]
    assert (t0 > 0).all() and (t1 >= t0).all()
    c0 = items[0]
    mine = [k for k, c in enumerate(items) if c == c0]
    assert len(mine) > 1
    # the first circuit's workgroups all start before any of them finishes
    assert max(t0[mine]) < min(t1[mine])
    ref = oracle.run_circuit(circs[0], circs[0].params)
    got = views[0].cpu().numpy()
    assert float(np.max(np.abs(got - ref))) <= 1e-12
