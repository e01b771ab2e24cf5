"""Host-only checks of the circuit planner: the gate order it executes is
equivalent to the circuit's own order (checked with the oracle), runs are
made only of gates whose target lies below the tile width, and validation
names the offending gate."""
import numpy as np
import pytest

import oracle
import workloads as W


@pytest.fixture(scope="module")
def sv():
    import paper_2411_18354_amd as sv
    return sv


def _rand_circuit(n, ngates, seed, kinds=("X", "Y", "Z", "H", "RX", "RY", "RZ", "P")):
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(ngates):
        k = kinds[int(rng.integers(0, len(kinds)))]
        t = int(rng.integers(0, n))
        others = [q for q in range(n) if q != t]
        c = int(rng.integers(0, 4))
        ctrls = tuple(int(q) for q in rng.choice(others, size=c, replace=False)) if c else ()
        vals = tuple(int(v) for v in rng.integers(0, 2, size=c))
        gates.append(W.Gate(k, t, ctrls, vals, float(rng.uniform(0, 2 * np.pi))))
    return W.Circuit(n, gates)


def _apply_in_order(c, order, psi0):
    psi = psi0.copy()
    for i in order:
        g = c.gates[i]
        oracle.apply_gate(psi, c.n, g.target, g.controls, g.values, oracle.gate_matrix(g.kind, g.theta, g.matrix))
    return psi


@pytest.mark.parametrize("depth", [0, 1, 2])
@pytest.mark.parametrize("seed", range(6))
def test_planned_order_equivalent(sv, seed, depth):
    """The planner's gate order (deferrals past commuting gates, each run's
    tile qubits chosen without lookahead, one step or two) applied by the
    oracle equals the circuit's own order."""
    n = 10
    sv.sv_tune_set("tile_log2_c128", 6)
    sv.sv_tune_set("plan_lookahead", depth)
    try:
        c = _rand_circuit(n, 300, seed)
        order, pass_of, npasses = sv.sv_circuit_plan(n, c, flags=sv.SV_FUSE)
        assert sorted(order) == list(range(len(c.gates)))
        rng = np.random.default_rng(100 + seed)
        psi0 = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
        psi0 /= np.linalg.norm(psi0)
        ref = _apply_in_order(c, range(len(c.gates)), psi0)
        got = _apply_in_order(c, order, psi0)
        assert np.max(np.abs(got - ref)) < 1e-12
        # fused passes hold only gates with target < m and keep their relative order
        passes = {}
        for k, (g, p) in enumerate(zip(order, pass_of)):
            passes.setdefault(p, []).append(g)
        fused = [v for v in passes.values() if len(v) > 1]
        assert fused, "expected some fused runs"
        for v in fused:
            assert len({c.gates[g].target for g in v if c.gates[g].kind not in ("Z", "RZ", "P")}) <= 6
        assert npasses == len(passes) < len(c.gates)
    finally:
        sv.sv_tune_set("tile_log2_c128", 12)


def test_reordering_happens_and_respects_dependencies(sv):
    """A high-target gate between two low runs is moved after the second run
    only when it commutes with it (contiguous 6-qubit tiles)."""
    sv.sv_tune_set("tile_log2_c128", 6)
    sv.sv_tune_set("tile_low_bits_c128", 6)
    try:
        n = 8
        g = [W.Gate("H", 0), W.Gate("X", 7, (1,)), W.Gate("H", 2), W.Gate("H", 1)]
        order, pass_of, _ = sv.sv_circuit_plan(n, g, flags=sv.SV_FUSE)
        # H(2) commutes with CX(1->7) and joins the first run; H(1) does not
        assert order[:2] == [0, 2] and pass_of[0] == pass_of[1]
        assert order.index(1) < order.index(3)
        # diagonal gates commute with controls on their target
        g = [W.Gate("H", 0), W.Gate("X", 7, (1,)), W.Gate("RZ", 1, theta=0.3), W.Gate("Z", 0)]
        order, pass_of, _ = sv.sv_circuit_plan(n, g, flags=sv.SV_FUSE)
        assert pass_of[0] == pass_of[1] == pass_of[2]
    finally:
        sv.sv_tune_set("tile_log2_c128", 12)


def test_qubit_set_tiles_fuse_high_targets(sv):
    """Tiles over chosen qubit sets: the n=29 QFT staircase and a layer of
    gates on every qubit collapse into a few passes, and diagonal gates join
    runs whatever their target."""
    n = 29
    _, _, npasses = sv.sv_circuit_plan(n, W.qft(n), flags=sv.SV_FUSE)
    assert npasses <= 6, npasses
    g = [W.Gate("H", q) for q in range(n)] + [W.Gate("RZ", q, theta=0.1) for q in range(n)]
    order, pass_of, npasses = sv.sv_circuit_plan(n, g, flags=sv.SV_FUSE)
    assert npasses <= 5, npasses
    psi0 = np.random.default_rng(0).standard_normal(1 << 12) + 0j
    # equivalence of the planned order on a smaller register with the same structure
    m = 12
    c = W.Circuit(m, [W.Gate("H", q) for q in range(m)] + [W.Gate("P", q, (q - 1,) if q else (), (), 0.3)
                                                         for q in range(m)])
    sv.sv_tune_set("tile_log2_c128", 8)
    sv.sv_tune_set("tile_low_bits_c128", 4)
    try:
        order, pass_of, npasses = sv.sv_circuit_plan(m, c, flags=sv.SV_FUSE)
        assert npasses < len(c.gates)
        ref = _apply_in_order(c, range(len(c.gates)), psi0)
        got = _apply_in_order(c, order, psi0)
        assert np.max(np.abs(got - ref)) < 1e-12
    finally:
        sv.sv_tune_set("tile_log2_c128", 12)
        sv.sv_tune_set("tile_low_bits_c128", 6)


def test_unfused_and_masked_keep_order(sv):
    c = _rand_circuit(9, 50, 3)
    for flags in (0, sv.SV_MASKED, sv.SV_MASKED | sv.SV_FUSE):
        order, pass_of, npasses = sv.sv_circuit_plan(9, c, flags=flags)
        assert order == list(range(50)) and npasses == 50


def test_workload_plan_stats(sv):
    for c, npar, max_passes in ((W.random_gates_n12(), 0, 1), (W.layered_circuit_n32(), 0, 1000), (W.hea_problem_n24()[0], 768, 650)):
        _, _, npasses = sv.sv_circuit_plan(c.n, c, nparams=npar, flags=sv.SV_FUSE)
        assert npasses <= max_passes, (c.meta, npasses)


def test_circuit_validation_names_gate(sv):
    bad = [W.Gate("H", 0), W.Gate("X", 3, (3,))]
    with pytest.raises(sv.SvError) as e:
        sv.sv_circuit_plan(4, bad)
    assert "gate 1" in str(e.value)
    with pytest.raises(sv.SvError) as e:
        sv.sv_circuit_plan(4, [W.Gate("H", 0, param=0)], nparams=1)
    assert "takes no parameter" in str(e.value)
    with pytest.raises(sv.SvError) as e:
        sv.sv_circuit_plan(4, [W.Gate("RY", 0, param=3)], nparams=2)
    assert "nparams" in str(e.value)
    with pytest.raises(sv.SvError):
        sv.sv_circuit_plan(4, [W.Gate("RY", 4)])
    # the C entry point rejects an unknown kind and unknown flags
    arr = sv.circuit_gates([W.Gate("H", 0)])
    arr[0].kind = 99
    with pytest.raises(sv.SvError):
        sv.sv_circuit_plan(4, arr)
    with pytest.raises(sv.SvError):
        sv.sv_circuit_plan(4, [W.Gate("H", 0)], flags=64)


def test_library_gate_matrices_match_definitions(sv):
    for k in ("X", "Y", "Z", "H", "RX", "RY", "RZ", "P", "~RX", "~RY", "~RZ", "~P", "~H"):
        for th in (0.0, 0.7, 2.5):
            a = np.array(sv.sv_gate_matrix(k, th))
            m = oracle.gate_matrix(k, th)
            assert np.max(np.abs(a - np.stack([m.real, m.imag], -1).reshape(8))) < 1e-15, (k, th)
    U = W.haar_unitary_2x2(5)
    assert np.allclose(sv.sv_gate_matrix("U", 0.0, U), U)


def test_circuit_json_round_trip(tmp_path):
    """The serialised circuit format reproduces every gate exactly (angles,
    parameters, explicit matrices, negative controls)."""
    circs = [W.qft(6), W.hea(5, 2, seed=3), W.random_gates_n12(seed=4, n=7, ngates=40),
             W.Circuit(4, [W.Gate("U", 1, (0, 3), (1, 0), matrix=tuple(W.haar_unitary_2x2(5))),
                           W.Gate("RY", 2, (), (), param=0)], np.array([0.123456789012345678]))]
    path = str(tmp_path / "c.jsonl")
    W.save_circuits(path, circs)
    back = W.load_circuits(path)
    assert len(back) == len(circs)
    for a, b in zip(circs, back):
        assert a.n == b.n and a.gates == b.gates
        assert (a.params is None) == (b.params is None)
        if a.params is not None:
            assert np.array_equal(a.params, b.params)
        psi_a = oracle.run_circuit(a, a.params)
        psi_b = oracle.run_circuit(b, b.params)
        assert np.array_equal(psi_a, psi_b)


def test_remap_plan_host():
    """SV_REMAP (host dry run): a circuit whose controls sit on the lowest
    qubits gets the two qubit-exchange passes; one without such controls
    does not; the execution order is that of the plan without remapping."""
    import paper_2411_18354_amd as sv
    c = W.low_control_circuit(n=20, ngates=30, seed=2)
    o0, p0, n0 = sv.sv_circuit_plan(20, c, flags=0)
    o1, p1, n1 = sv.sv_circuit_plan(20, c, flags=sv.SV_REMAP)
    assert n1 == n0 + 2 and o0 == o1
    plain = W.random_gates_n12(seed=3, n=20, ngates=30)
    plain.gates = [g for g in plain.gates if not any(q < 3 for q in g.controls)]
    _, _, a = sv.sv_circuit_plan(20, plain, flags=0)
    _, _, b = sv.sv_circuit_plan(20, plain, flags=sv.SV_REMAP)
    assert a == b


def test_diagonal_gates_grouped_inside_runs(sv):
    """Inside a fused run, diagonal gates move later past the non-diagonal
    gates they commute with: an ansatz layer RY(q) RZ(q) for every qubit
    becomes all RY then all RZ (one diagonal block), and the order stays
    equivalent to the circuit's (oracle).  A diagonal gate never passes a
    pair gate on its own qubit."""
    n = 8
    c = W.hea(n, 2, seed=3)
    order, pass_of, _ = sv.sv_circuit_plan(n, c, nparams=c.nparams, flags=sv.SV_FUSE)
    kinds = [c.gates[i].kind for i in order]
    assert len(set(pass_of)) == 1  # n=8 fits one tile: one run
    # per layer: every RY, then every RZ (one diagonal block), then the CNOT chain
    assert kinds == (["RY"] * n + ["RZ"] * n + ["X"] * (n - 1)) * 2, kinds
    for i, gi in enumerate(order):
        g = c.gates[gi]
        if g.kind == "RZ":  # its own qubit's RY (the gate before it in the circuit) still comes first
            assert order.index(gi - 1) < i
    psi0 = W.random_state(n, 4)
    ref = oracle.run_circuit(c, c.params, psi0)
    psi = psi0.copy()
    for gi in order:
        g = c.gates[gi]
        oracle.apply_gate(psi, n, g.target, g.controls, g.values, oracle.gate_matrix(g.kind, c.params[g.param]))
    assert np.max(np.abs(psi - ref)) < 1e-12
