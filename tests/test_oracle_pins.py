"""Pins for the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each check is a worked example
printed in the paper, a closed form, an identity, a brute-force enumeration
computed a different way, or a dense Kronecker-product construction.
"""
import itertools
import json
import math
import os

import numpy as np
from scipy.linalg import expm
import pytest

import oracle
import workloads as W
from tests import dense_ref as D

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_state(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return v / np.linalg.norm(v)


def _rand_unitary(seed):
    return oracle.gate_matrix("U", matrix=W.haar_unitary_2x2(seed))


# ---------------------------------------------------------------- index sets

def _ith_cleared(i, t):
    """Insert a 0 at bit t of i (the pair-index helper the paper borrows)."""
    return ((i >> t) << (t + 1)) | (i & ((1 << t) - 1))


def _skip_map(i_r, t, controls):
    """The paper's iterative skip-interval map (Sec. III-B), ascending
    controls, each adjusted relative to the target, then ithCleared."""
    i = i_r
    for c in sorted(controls):
        c_adj = c - 1 if c > t else c
        s = 1 << c_adj
        i = i + (i // s + 1) * s
    return i


def test_worked_example_golden():
    g = json.load(open(os.path.join(GOLDEN, "worked_example_n3_t1.json")))
    n, t = g["n"], g["target"]
    for case in g["cases"]:
        ctrls = case["controls"]
        adj = [c - 1 if c > t else c for c in ctrls]
        assert adj == case["adjusted_controls"]
        assert [1 << a for a in adj] == case["skip_intervals"]
        got = [_skip_map(i, t, ctrls) for i in case["reduced_set"]]
        assert got == case["global_iterations"]
        # the oracle's brute-force pair list, mapped back to iteration indices
        pl = oracle.pair_list(n, t, ctrls)
        it = [((int(k) >> (t + 1)) << t) | (int(k) & ((1 << t) - 1)) for k in pl]
        assert it == case["global_iterations"]


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7])
def test_pair_list_matches_skip_map_exhaustive(n):
    """Every target and every control subset (values 1): brute force equals
    the paper's iterative map followed by ithCleared, order included."""
    for t in range(n):
        others = [q for q in range(n) if q != t]
        for c in range(len(others) + 1):
            for ctrls in itertools.combinations(others, c):
                bf = oracle.pair_list(n, t, ctrls)
                sm = [_ith_cleared(_skip_map(i, t, ctrls), t) for i in range(1 << (n - 1 - c))]
                assert bf.tolist() == sm, (n, t, ctrls)


def test_pair_list_descending_controls_fails():
    """The map needs ascending controls (Sec. III-B); applying it in
    descending order gives a different set for some two-control case."""
    n, t, ctrls = 4, 0, (1, 2)
    i = 0
    for c in sorted(ctrls, reverse=True):
        c_adj = c - 1 if c > t else c
        s = 1 << c_adj
        i = i + (i // s + 1) * s
    assert _ith_cleared(i, t) != int(oracle.pair_list(n, t, ctrls)[0])


@pytest.mark.parametrize("n", [3, 5, 7])
def test_pair_list_any_control_values(n):
    """Values 0/1: the list equals all k with bit t clear and control bits equal
    to the values, enumerated by itertools over the free bits."""
    rng = np.random.default_rng(n)
    for _ in range(30):
        t = int(rng.integers(0, n))
        others = [q for q in range(n) if q != t]
        c = int(rng.integers(0, len(others) + 1))
        ctrls = tuple(sorted(rng.choice(others, size=c, replace=False).tolist())) if c else ()
        vals = tuple(int(v) for v in rng.integers(0, 2, size=c))
        free = [q for q in range(n) if q != t and q not in ctrls]
        fixed = sum(v << q for q, v in zip(ctrls, vals))
        expect = sorted(fixed + sum(b << q for b, q in zip(bits, free))
                        for bits in itertools.product((0, 1), repeat=len(free)))
        assert oracle.pair_list(n, t, ctrls, vals).tolist() == expect


# ---------------------------------------------------------------- gate update

@pytest.mark.parametrize("t", [0, 1, 4])
def test_x_swaps_bit_exact(t):
    n = 5
    psi = _rand_state(n, 1)
    out = oracle.apply_gate(psi.copy(), n, t, (), (), oracle.gate_matrix("X"))
    idx = np.arange(1 << n) ^ (1 << t)
    assert np.array_equal(out, psi[idx])


def test_h_all_qubits_uniform():
    n = 8
    psi = oracle.zero_state(n)
    for q in range(n):
        oracle.apply_gate(psi, n, q, (), (), oracle.gate_matrix("H"))
    assert np.max(np.abs(psi - 2.0 ** (-n / 2))) < 1e-15


def test_h_basis_states():
    n = 1
    for b, sgn in ((0, 1), (1, -1)):
        psi = np.zeros(2, dtype=np.complex128); psi[b] = 1
        oracle.apply_gate(psi, n, 0, (), (), oracle.gate_matrix("H"))
        assert np.allclose(psi, np.array([1, sgn]) / math.sqrt(2), atol=1e-16)


def test_norm_preserved():
    n = 10
    psi = _rand_state(n, 2)
    rng = np.random.default_rng(3)
    for i in range(50):
        t = int(rng.integers(0, n))
        others = [q for q in range(n) if q != t]
        c = int(rng.integers(0, 4))
        ctrls = tuple(rng.choice(others, size=c, replace=False).tolist())
        oracle.apply_gate(psi, n, t, ctrls, (), _rand_unitary(100 + i))
    assert abs(oracle.norm2(psi, n) - 1.0) < 1e-13


def test_ghz():
    n = 9
    psi = oracle.run_circuit(W.ghz(n))
    ref = np.zeros(1 << n, dtype=np.complex128)
    ref[0] = ref[-1] = 1 / math.sqrt(2)
    assert np.max(np.abs(psi - ref)) < 1e-15


def _bitrev(x, n):
    return int(format(x, "0%db" % n)[::-1], 2)


@pytest.mark.parametrize("n", [3, 4, 5, 7])
def test_qft_closed_form(n):
    """The staircase as drawn (no swaps) equals the Fourier matrix with
    e^{+2 pi i x y / N} / sqrt(N) after bit-reversing the input index."""
    N = 1 << n
    psi0 = _rand_state(n, 10 + n)
    out = oracle.run_circuit(W.qft(n), psi0=psi0)
    rev = np.array([_bitrev(x, n) for x in range(N)])
    ref = np.fft.ifft(psi0[rev]) * math.sqrt(N)
    assert np.max(np.abs(out - ref)) < 1e-13


@pytest.mark.parametrize("n", [2, 4, 6])
def test_stream_decrements(n):
    """The streaming circuit maps |x> to |x - 1 mod 2^n> (Sec. IV-C figure)."""
    psi0 = _rand_state(n, 20 + n)
    out = oracle.run_circuit(W.stream(n), psi0=psi0)
    # amplitude of |x> moves to |x-1>
    assert np.array_equal(out, np.roll(psi0, -1))


def test_negative_control_identity():
    """X on the control, controlled G, X on the control equals G controlled
    on value 0 (Sec. I, two-qubit circuit figure)."""
    n = 4
    G = _rand_unitary(7)
    for t, c in ((0, 1), (1, 0), (3, 1), (0, 3)):
        psi = _rand_state(n, 30 + t)
        a = psi.copy()
        oracle.apply_gate(a, n, c, (), (), oracle.gate_matrix("X"))
        oracle.apply_gate(a, n, t, (c,), (), G)
        oracle.apply_gate(a, n, c, (), (), oracle.gate_matrix("X"))
        b = oracle.apply_gate(psi.copy(), n, t, (c,), (0,), G)
        assert np.max(np.abs(a - b)) < 1e-15


@pytest.mark.parametrize("n", [1, 2, 4, 7])
def test_dense_kron_random_gates(n):
    rng = np.random.default_rng(40 + n)
    for i in range(25):
        t = int(rng.integers(0, n))
        others = [q for q in range(n) if q != t]
        c = int(rng.integers(0, min(3, n - 1) + 1))
        ctrls = tuple(rng.choice(others, size=c, replace=False).tolist()) if c else ()
        vals = tuple(int(v) for v in rng.integers(0, 2, size=c))
        G = _rand_unitary(500 + i)
        psi = _rand_state(n, 600 + i)
        got = oracle.apply_gate(psi.copy(), n, t, ctrls, vals, G)
        ref = D.controlled_unitary(n, t, ctrls, vals, G) @ psi
        assert np.max(np.abs(got - ref)) < 1e-14


def test_dense_kron_random_gates_small():
    """A random controlled-gate circuit at n=8 against the product of dense gates."""
    c = W.random_gates_n12(seed=11, n=8, ngates=60)
    got = oracle.run_circuit(c)
    psi = np.zeros(1 << c.n, dtype=np.complex128); psi[0] = 1
    for g in c.gates:
        G = oracle.gate_matrix(g.kind, g.theta, g.matrix)
        psi = D.controlled_unitary(c.n, g.target, g.controls, g.values, G) @ psi
    assert np.max(np.abs(got - psi)) < 1e-13


def test_gate_matrices_closed_forms():
    th = 0.7
    for kind, P in (("RX", D.PX), ("RY", D.PY), ("RZ", D.PZ)):
        ref = math.cos(th / 2) * np.eye(2) - 1j * math.sin(th / 2) * P
        assert np.allclose(oracle.gate_matrix(kind, th), ref, atol=1e-15)
    for m in range(1, 6):
        Rm = oracle.gate_matrix("P", 2 * math.pi / (1 << m))
        assert np.allclose(Rm, np.diag([1, np.exp(2j * math.pi / (1 << m))]), atol=1e-15)
    for kind in ("X", "Y", "Z", "H"):
        U = oracle.gate_matrix(kind)
        assert np.allclose(U @ U.conj().T, np.eye(2), atol=1e-15)
    U = _rand_unitary(3)
    assert np.allclose(oracle.gate_matrix("~U", matrix=W.haar_unitary_2x2(3)), U.conj().T)


def test_gate_amplitudes_match_full_gate():
    n = 9
    psi = _rand_state(n, 50)
    G = _rand_unitary(51)
    for t, ctrls, vals in ((0, (), ()), (4, (1, 7), (1, 0)), (8, (0, 2, 5), ())):
        full = oracle.apply_gate(psi.copy(), n, t, ctrls, vals, G)
        idx = np.arange(1 << n)
        amp = oracle.gate_amplitudes(psi, n, t, ctrls, vals, G, idx)
        assert np.array_equal(amp, full)


# ---------------------------------------------------------------- expectation

def test_pauli_expectation_dense_all_strings():
    n = 3
    psi = _rand_state(n, 60)
    for x in range(1 << n):
        for z in range(1 << n):
            ref = np.vdot(psi, D.pauli_matrix(n, x, z) @ psi)
            got = oracle.expect_pauli(psi, n, x, z)
            assert abs(got - ref) < 1e-14
            assert abs(got.imag) < 1e-14


def test_expectation_product_states():
    n = 6
    zero = oracle.zero_state(n)
    plus = zero.copy()
    for q in range(n):
        oracle.apply_gate(plus, n, q, (), (), oracle.gate_matrix("H"))
    for i in range(n - 1):
        assert abs(oracle.expect_pauli(zero, n, 0, 3 << i).real - 1.0) < 1e-15
    for i in range(n):
        assert abs(oracle.expect_pauli(plus, n, 1 << i, 0).real - 1.0) < 1e-14
        assert abs(oracle.expect_pauli(zero, n, 1 << i, 0).real) < 1e-15


def test_hamiltonian_apply_dense():
    n = 5
    terms = W.zz_x_hamiltonian(n, 3) + [W.PauliTerm(0.3, 0b00101, 0b00111)]
    psi = _rand_state(n, 61)
    ref = D.hamiltonian_matrix(n, terms) @ psi
    assert np.max(np.abs(oracle.apply_hamiltonian(psi, n, terms) - ref)) < 1e-14
    assert abs(oracle.expect(psi, n, terms) - np.vdot(psi, ref).real) < 1e-14


# ---------------------------------------------------------------- gradients

def test_gradient_one_qubit_analytic():
    """<Z> after RY(theta)|0> is cos(theta): gradient -sin(theta)."""
    c = W.Circuit(1, [W.Gate("RY", 0, param=0)], np.array([0.9]))
    terms = [W.PauliTerm(1.0, 0, 1)]
    assert abs(oracle.loss(c, c.params, terms) - math.cos(0.9)) < 1e-15
    g = oracle.grad_param_shift(c, c.params, terms)
    assert abs(g[0] + math.sin(0.9)) < 1e-14


def _generator(kind):
    """A with dG/dtheta = A G(theta) for the angle kinds: -i P/2 for
    RX/RY/RZ = exp(-i theta P/2), i |1><1| for P = diag(1, e^{i theta}); an
    adjoint-flagged kind G(-theta) has -A."""
    adj = kind.startswith("~")
    A = {"RX": -0.5j * D.PX, "RY": -0.5j * D.PY, "RZ": -0.5j * D.PZ, "P": 1j * D.P1}[kind.lstrip("~")]
    return -A if adj else A


def _dense_grad(c, params, terms):
    """Exact gradient from dense matrices: d/dtheta of a (controlled) gate
    is P_sat (x) dG/dtheta, summed over every gate using the parameter."""
    n = c.n
    H = D.hamiltonian_matrix(n, terms)
    mats = []
    for g in c.gates:
        th = params[g.param] if g.param >= 0 else g.theta
        mats.append(D.controlled_unitary(n, g.target, g.controls, g.values,
                                         oracle.gate_matrix(g.kind, th, g.matrix)))
    grad = np.zeros(len(params))
    psi0 = np.zeros(1 << n, dtype=np.complex128); psi0[0] = 1
    for gi, g in enumerate(c.gates):
        if g.param < 0:
            continue
        th = params[g.param]
        dR = _generator(g.kind) @ oracle.gate_matrix(g.kind, th)
        vals = g.values if len(g.values) else [1] * len(g.controls)
        proj = {q: (D.P1 if v else D.P0) for q, v in zip(g.controls, vals)}
        dM = D.kron_ops({**proj, g.target: dR}, n)
        psi = psi0.copy(); dpsi = None
        for k, M in enumerate(mats):
            if k == gi:
                dpsi = dM @ psi
                psi = M @ psi
            else:
                psi = M @ psi
                if dpsi is not None:
                    dpsi = M @ dpsi
        grad[g.param] += 2.0 * np.vdot(psi, H @ dpsi).real
    return grad


def test_param_shift_vs_dense_with_controlled_rotations():
    n = 4
    rng = np.random.default_rng(70)
    gates, p = [], 0
    for layer in range(2):
        for q in range(n):
            gates.append(W.Gate("RY", q, param=p)); p += 1
        gates.append(W.Gate("RZ", 2, (0,), param=p)); p += 1
        gates.append(W.Gate("RY", 1, (3, 0), (1, 0), param=p)); p += 1
        gates.append(W.Gate("RX", 3, param=p)); p += 1
        for q in range(n - 1):
            gates.append(W.Gate("X", q + 1, (q,)))
    params = rng.uniform(0, 2 * math.pi, size=p)
    c = W.Circuit(n, gates, params)
    terms = W.zz_x_hamiltonian(n, 9)
    ref = _dense_grad(c, params, terms)
    ps = oracle.grad_param_shift(c, params, terms)
    fd = oracle.grad_finite_diff(c, params, terms)
    assert np.max(np.abs(ps - ref)) < 1e-12
    assert np.max(np.abs(fd - ref)) < 1e-8


ANGLE_KINDS = ("RX", "RY", "RZ", "P", "~RX", "~RY", "~RZ", "~P")


def _all_kinds_circuit(seed):
    """Every angle kind, uncontrolled and with one and two controls of mixed
    values, parameters shared between kinds, fixed gates in between."""
    n = 4
    rng = np.random.default_rng(seed)
    gates = []
    for i, kind in enumerate(ANGLE_KINDS * 3):
        t = int(rng.integers(0, n))
        others = [q for q in range(n) if q != t]
        nc = (i // len(ANGLE_KINDS)) % 3
        ctrls = tuple(int(q) for q in rng.choice(others, size=nc, replace=False))
        vals = tuple(int(v) for v in rng.integers(0, 2, size=nc))
        gates.append(W.Gate(kind, t, ctrls, vals, param=int(rng.integers(0, 6))))
        gates.append(W.Gate("H", int(rng.integers(0, n))))
    return W.Circuit(n, gates, rng.uniform(0, 2 * math.pi, size=6))


def test_param_shift_every_kind_vs_dense():
    """The shift rule for controlled RX (C^kZ conjugation), controlled P
    (two generator eigenvalues), and adjoint-flagged kinds, against dense
    derivatives, and central differences against the same."""
    for seed in (71, 72):
        c = _all_kinds_circuit(seed)
        terms = W.zz_x_hamiltonian(c.n, seed)
        ref = _dense_grad(c, c.params, terms)
        ps = oracle.grad_param_shift(c, c.params, terms)
        fd = oracle.grad_finite_diff(c, c.params, terms)
        assert np.max(np.abs(ps - ref)) < 1e-12, np.max(np.abs(ps - ref))
        assert np.max(np.abs(fd - ref)) < 1e-8


def test_param_shift_planted_mistakes_fail(monkeypatch):
    """The dense pin catches plausible mistakes in the shift rule: a
    conjugating Pauli that commutes with the rotation (X for RX, Y for RY,
    Z for RZ) and a dropped sign for adjoint-flagged controlled rotations."""
    c = _all_kinds_circuit(71)
    terms = W.zz_x_hamiltonian(c.n, 71)
    ref = _dense_grad(c, c.params, terms)
    for flip in ({"RX": "X", "RY": "X", "RZ": "X"}, {"RX": "Z", "RY": "Y", "RZ": "X"},
                 {"RX": "Z", "RY": "X", "RZ": "Z"}):
        monkeypatch.setattr(oracle, "_SHIFT_FLIP", flip)
        assert np.max(np.abs(oracle.grad_param_shift(c, c.params, terms) - ref)) > 1e-3
    monkeypatch.undo()
    # drop the adjoint sign: shift ~R as if it were R(+theta) controlled
    gates = [W.Gate(g.kind.lstrip("~"), g.target, g.controls, g.values, g.theta, g.param)
             if g.kind.startswith("~") and g.controls and g.kind != "~P" else g for g in c.gates]
    wrong = oracle.grad_param_shift(W.Circuit(c.n, gates, c.params), c.params, terms)
    assert np.max(np.abs(wrong - ref)) > 1e-3


def _pauli_pin_failures(gm):
    """Checks that fix Y and Z from X and H (pinned by the paper's closed
    forms) and the Pauli algebra; returns the names of the failing ones."""
    X, Y, Z, H = gm("X"), gm("Y"), gm("Z"), gm("H")
    I = np.eye(2)
    bad = []
    checks = {
        "Z = H X H": np.allclose(Z, H @ X @ H, atol=1e-15),
        "Y = i X Z": np.allclose(Y, 1j * X @ Z, atol=1e-15),
        "XY = iZ": np.allclose(X @ Y, 1j * Z, atol=1e-15),
        "YZ = iX": np.allclose(Y @ Z, 1j * X, atol=1e-15),
        "ZX = iY": np.allclose(Z @ X, 1j * Y, atol=1e-15),
        "squares": all(np.allclose(P @ P, I, atol=1e-15) for P in (X, Y, Z)),
        "Z|0> = |0>": np.allclose(Z @ [1, 0], [1, 0], atol=1e-15),
        "Y|0> = i|1>": np.allclose(Y @ [1, 0], [0, 1j], atol=1e-15),
    }
    for th in (0.3, 2.1):
        checks["RX = exp(-i th X/2) %g" % th] = np.allclose(gm("RX", th), expm(-0.5j * th * X), atol=1e-14)
        checks["RY = exp(-i th Y/2) %g" % th] = np.allclose(gm("RY", th), expm(-0.5j * th * Y), atol=1e-14)
        checks["RZ = exp(-i th Z/2) %g" % th] = np.allclose(gm("RZ", th), expm(-0.5j * th * Z), atol=1e-14)
        checks["P = e^{i th/2} RZ %g" % th] = np.allclose(gm("P", th), np.exp(0.5j * th) * gm("RZ", th), atol=1e-14)
    checks["RY(pi/2)|0> = H|0>"] = np.allclose(gm("RY", math.pi / 2) @ [1, 0], H @ [1, 0], atol=1e-15)
    return [k for k, ok in checks.items() if not ok]


def test_pauli_and_rotation_matrices_pinned():
    """Y and Z (named but not printed in the paper) from the paper's X and H
    via Z = HXH and Y = iXZ, the Pauli algebra, and the rotations as matrix
    exponentials of them (scipy expm).  Planted sign mistakes fail."""
    assert _pauli_pin_failures(oracle.gate_matrix) == []

    def mutate(which, f):
        def gm(kind, theta=0.0, matrix=None):
            U = oracle.gate_matrix(kind, theta, matrix)
            return f(U) if kind == which else U
        return gm
    for which, f in (("Y", lambda U: -U), ("Z", lambda U: -U), ("Y", lambda U: U.T),
                     ("RY", lambda U: U.T), ("RZ", lambda U: U.conj()), ("RX", lambda U: U.conj()),
                     ("P", lambda U: U.conj())):
        assert _pauli_pin_failures(mutate(which, f)), which


def test_param_shift_shared_parameter():
    """One parameter used by two gates: contributions add (product rule)."""
    n = 2
    gates = [W.Gate("RY", 0, param=0), W.Gate("RZ", 1, (0,), param=0), W.Gate("RY", 1, param=0)]
    c = W.Circuit(n, gates, np.array([0.4]))
    terms = [W.PauliTerm(0.7, 0, 3), W.PauliTerm(-0.2, 1, 0), W.PauliTerm(0.5, 2, 0)]
    ref = _dense_grad(c, c.params, terms)
    assert abs(oracle.grad_param_shift(c, c.params, terms)[0] - ref[0]) < 1e-12


# ---------------------------------------------------------------- generators

def test_generators_deterministic_and_shaped():
    a, b = W.random_gates_n12(), W.random_gates_n12()
    assert a.gates == b.gates and len(a.gates) == 200 and a.n == 12
    kinds = {g.kind for g in a.gates}
    assert kinds <= {"X", "H", "RY", "RZ"}
    assert all(len(g.controls) <= 3 and g.target not in g.controls for g in a.gates)
    cases = W.gate_sweep_cases()
    assert len(cases) == 27
    for t, ctrls in cases:
        assert t not in ctrls and len(set(ctrls)) == len(ctrls)
    c3, H = W.hea_problem_n24()
    assert c3.nparams == 768 and len(c3.gates) == 16 * (48 + 23) and len(H) == 23 + 24
    c2 = W.layered_circuit_n32()
    assert len(c2.gates) == 20 * (32 + 31 + 8)
    U = oracle.gate_matrix("U", matrix=W.haar_unitary_2x2(2))
    assert np.allclose(U @ U.conj().T, np.eye(2), atol=1e-15)


def test_block_low_matches_kron_and_gate_sequence():
    """A k-qubit matrix on the lowest qubits equals kron(I, M) (dense), and the
    matrix composed from a gate sequence on those qubits (by dense products)
    acts like the sequence applied gate by gate."""
    rng = np.random.default_rng(91)
    for n, k in ((5, 2), (7, 4), (8, 5)):
        z = rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))
        M, _ = np.linalg.qr(z)
        psi = _rand_state(n, 92 + n)
        got = oracle.apply_block_low(psi.copy(), n, k, M)
        ref = np.kron(np.eye(1 << (n - k)), M) @ psi
        assert np.max(np.abs(got - ref)) < 1e-14
        gates = W.random_gates_n12(seed=n, n=k, ngates=30).gates
        Mg = np.eye(1 << k, dtype=np.complex128)
        for g in gates:
            Mg = D.controlled_unitary(k, g.target, g.controls, g.values, oracle.gate_matrix(g.kind, g.theta)) @ Mg
        a = oracle.apply_block_low(psi.copy(), n, k, Mg)
        b = psi.copy()
        for g in gates:
            oracle.apply_gate(b, n, g.target, g.controls, g.values, oracle.gate_matrix(g.kind, g.theta))
        assert np.max(np.abs(a - b)) < 1e-13


def test_swap_qubits_matches_axis_transpose_and_three_cnots():
    """Exchanging qubits a and b equals swapping those two axes of the state
    seen as an n-axis tensor (numpy, no index loops), and equals three CNOTs
    (a->b, b->a, a->b) applied through the oracle's gate loop."""
    n = 6
    for a, b in ((0, 1), (0, 5), (2, 4), (5, 3)):
        psi = W.random_state(n, 10 + a * 7 + b)
        got = oracle.swap_qubits(psi.copy(), n, [(a, b)])
        # axis q of the C-order tensor is qubit n-1-q
        t = psi.reshape((2,) * n)
        ref = np.swapaxes(t, n - 1 - a, n - 1 - b).reshape(-1)
        assert np.array_equal(got, ref), (a, b)
        X = oracle.gate_matrix("X")
        cn = psi.copy()
        for c, t_ in ((a, b), (b, a), (a, b)):
            oracle.apply_gate(cn, n, t_, (c,), (), X)
        assert np.array_equal(cn, ref), (a, b)
    # several disjoint pairs in one call compose
    psi = W.random_state(n, 3)
    got = oracle.swap_qubits(psi.copy(), n, [(0, 4), (1, 5)])
    t = psi.reshape((2,) * n)
    ref = np.swapaxes(np.swapaxes(t, n - 1, n - 5), n - 2, n - 6).reshape(-1)
    assert np.array_equal(got, ref)


# ---------------------------------------------------------------- fixed-point states
#
# Block-scaled 16-bit states: value = code * 2^scale, one scale per 64
# amplitudes.  The pins below use only integers, closed forms and bounds that
# any correct encoding must meet; none restates the scale formula.

def _q16_random_buf(n, seed):
    return oracle.q16_encode(_rand_state(n, seed), n)


def test_q16_basis_and_hadamard_closed_forms():
    n = 8
    buf = oracle.q16_encode(oracle.zero_state(n), n)
    codes, scales = oracle.q16_views(buf, n)
    # 1.0 must be a code in [2^14, 2^15) times a power of two: 2^14 * 2^-14
    assert tuple(codes[0]) == (16384, 0) and scales[0] == -14
    assert not codes[1:].any()
    # zero blocks take the smallest scale
    assert (scales[1:] == -126).all()
    # H on |0>: both amplitudes 1/sqrt(2) = 23170.47... * 2^-15
    oracle.q16_apply_gate(buf, n, 0, [], [], np.array([[1, 1], [1, -1]]) / math.sqrt(2))
    assert tuple(codes[0]) == (23170, 0) and tuple(codes[1]) == (23170, 0)
    assert scales[0] == -15 and not codes[2:].any()
    # a single block below 64 amplitudes (n < 6) has one scale
    b3 = oracle.q16_encode(oracle.zero_state(3), 3)
    assert b3.size == 4 * 8 + 1 and oracle.q16_views(b3, 3)[1][0] == -14


def test_q16_exactly_representable_blocks_round_trip():
    rng = np.random.default_rng(40)
    n = 9
    N, B = 1 << n, 64
    codes = rng.integers(-32767, 32768, size=(N, 2)).astype(np.int64)
    scales = rng.integers(-60, 0, size=N // B)
    for b in range(N // B):  # put the block's largest magnitude in [2^14, 2^15)
        blk = codes[b * B:(b + 1) * B]
        big = int(rng.integers(16384, 32768))
        blk[int(rng.integers(0, B)), int(rng.integers(0, 2))] = big * (1 if rng.random() < 0.5 else -1)
        np.clip(blk, -big, big, out=blk)
    vals = codes.astype(np.float64) * np.ldexp(1.0, np.repeat(scales, B))[:, None]
    psi = vals[:, 0] + 1j * vals[:, 1]
    buf = oracle.q16_encode(psi, n)
    c2, s2 = oracle.q16_views(buf, n)
    assert np.array_equal(c2, codes) and np.array_equal(s2, scales)
    assert np.array_equal(oracle.q16_decode(buf, n), psi)
    # encoding a decoded state reproduces it (random state)
    b2 = _q16_random_buf(n, 41)
    assert np.array_equal(oracle.q16_encode(oracle.q16_decode(b2, n), n), b2)


def test_q16_encode_error_and_normalisation():
    rng = np.random.default_rng(42)
    n = 10
    B = 64
    psi = _rand_state(n, 43) * np.repeat(10.0 ** rng.uniform(-12, 0, size=(1 << n) // B), B)
    psi[5 * B:6 * B] = 0  # a zero block
    f = (psi.real.astype(np.float32).astype(np.float64) + 1j * psi.imag.astype(np.float32).astype(np.float64))
    buf = oracle.q16_encode(psi, n)
    codes, scales = oracle.q16_views(buf, n)
    dec = oracle.q16_decode(buf, n)
    for b in range(len(scales)):
        blk = slice(b * B, (b + 1) * B)
        m = max(np.abs(f[blk].real).max(), np.abs(f[blk].imag).max())
        if m == 0:
            assert not codes[blk].any()
            continue
        # largest code magnitude in [2^14, 2^15): 15 significant bits used
        assert 16384 <= np.abs(codes[blk]).max() <= 32767
        # rounding error at most half a step, and a step is at most m 2^-14
        step = math.ldexp(1.0, int(scales[b]))
        assert step <= m * 2.0 ** -14
        err = max(np.abs(dec[blk].real - f[blk].real).max(), np.abs(dec[blk].imag - f[blk].imag).max())
        assert err <= step / 2
    # saturation: 1 - 2^-24 scales to 32767.99..., which rounds to 32768 and saturates
    assert oracle.q16_code(np.float32(1 - 2.0 ** -24), oracle.q16_scale(np.float32(1 - 2.0 ** -24))) == 32767
    # a block far below 2^-111 keeps the smallest scale, exactly
    tiny = np.zeros(64, dtype=np.complex128)
    tiny[3] = 2.0 ** -120
    bt = oracle.q16_encode(tiny, 6)
    ct, st = oracle.q16_views(bt, 6)
    assert st[0] == -126 and ct[3, 0] == 64 and oracle.q16_decode(bt, 6)[3] == 2.0 ** -120


def test_q16_permutation_and_sign_gates_are_exact():
    n = 9
    X = np.array([[0, 1], [1, 0]])
    Z = np.diag([1, -1])
    buf0 = _q16_random_buf(n, 44)
    c0, s0 = oracle.q16_views(buf0, n)
    # X on a high target swaps whole blocks, codes and scales
    buf = buf0.copy()
    oracle.q16_apply_gate(buf, n, 7, [], [], X)
    c, s = oracle.q16_views(buf, n)
    perm = np.arange(1 << n) ^ (1 << 7)
    assert np.array_equal(c, c0[perm]) and np.array_equal(s, s0[np.arange(len(s0)) ^ 2])
    # X on a low target permutes codes inside each block, scales unchanged
    buf = buf0.copy()
    oracle.q16_apply_gate(buf, n, 3, [], [], X)
    c, s = oracle.q16_views(buf, n)
    assert np.array_equal(c, c0[np.arange(1 << n) ^ 8]) and np.array_equal(s, s0)
    # controlled on qubit 8: only blocks whose index has bit 2 set move
    buf = buf0.copy()
    oracle.q16_apply_gate(buf, n, 7, [8], [1], X)
    k = np.arange(1 << n)
    perm = np.where(k & 256, k ^ 128, k)
    c, s = oracle.q16_views(buf, n)
    assert np.array_equal(c, c0[perm])
    bi = np.arange(len(s0))
    assert np.array_equal(s, s0[np.where(bi & 4, bi ^ 2, bi)])
    # Z negates the codes whose target bit is 1
    buf = buf0.copy()
    oracle.q16_apply_gate(buf, n, 2, [], [], Z)
    c, s = oracle.q16_views(buf, n)
    sign = np.where(k & 4, -1, 1)[:, None]
    assert np.array_equal(c, c0 * sign) and np.array_equal(s, s0)


@pytest.mark.parametrize("case", [(0, (), ()), (4, (1,), (0,)), (7, (2, 8), (1, 1)), (9, (0, 6), (1, 0)),
                                  (2, (), ()), (5, (9,), (1,))])
def test_q16_gate_within_quantisation_of_double(case):
    n = 10
    t, ctrls, vals = case
    B = 64
    U = _rand_unitary(45 + t)
    buf = _q16_random_buf(n, 46 + t)
    x = oracle.q16_decode(buf, n)
    exact = oracle.apply_gate(x.copy(), n, t, ctrls, vals, U)
    # the float matrix the arithmetic uses, applied exactly
    U32 = U.real.astype(np.float32).astype(np.float64) + 1j * U.imag.astype(np.float32).astype(np.float64)
    exact32 = oracle.apply_gate(x.copy(), n, t, ctrls, vals, U32)
    out_buf = oracle.q16_apply_gate(buf.copy(), n, t, ctrls, vals, U)
    out = oracle.q16_decode(out_buf, n)
    cm, cv = oracle.masks(ctrls, vals)
    k = np.arange(1 << n)
    moved = ((k & cm) == cv)  # amplitudes of updated pairs
    touched_blocks = np.unique(k[moved] // B)
    for b in range(len(x) // B):
        blk = slice(b * B, (b + 1) * B)
        if b not in touched_blocks:
            assert np.array_equal(out[blk], x[blk])  # untouched blocks keep their bytes
            continue
        m = max(np.abs(exact32[blk].real).max(), np.abs(exact32[blk].imag).max())
        # half a quantisation step (<= m 2^-15) plus float rounding of the products
        tol = m * 2.0 ** -15 * (1 + 1e-5) + 8 * 2.0 ** -24 * np.abs(x).max() * 2
        err = max(np.abs(out[blk].real - exact32[blk].real).max(), np.abs(out[blk].imag - exact32[blk].imag).max())
        assert err <= tol, (b, err, tol)
    # and the float matrix differs from the double one by float rounding only
    assert np.abs(exact32 - exact).max() <= 4 * 2.0 ** -24 * np.abs(x).max() * 2


def test_q16_qft_within_rigorous_bound():
    n = 10
    circ = W.qft(n)
    psi0 = _rand_state(n, 47)
    buf = oracle.q16_run_circuit(circ, buf0=oracle.q16_encode(psi0, n))
    # closed form of the QFT as drawn (no swaps, + sign): ifft of the
    # bit-reversed input times sqrt(N)
    N = 1 << n
    rev = np.array([int(format(i, "0%db" % n)[::-1], 2) for i in range(N)])
    want = np.fft.ifft(psi0[rev]) * math.sqrt(N)
    err = np.linalg.norm(oracle.q16_decode(buf, n) - want)
    # each gate adds at most sqrt(2 * 64) * 2^-15 (half steps over the
    # re-encoded blocks, norm 1) plus float rounding; unitaries keep errors'
    # norms, and the initial encoding adds one more such term
    G = len(circ.gates)
    assert err <= (G + 1) * (math.sqrt(128) * 2.0 ** -15 + 1e-6)
    assert err < 5e-3  # far inside the bound in practice


# ---------------------------------------------------------------- 32-bit fixed point
#
# The same block rule with 32-bit codes in double: pinned like the 16-bit
# codes, by closed forms, exactly representable blocks and bounds.

def test_q32_basis_and_hadamard_closed_forms():
    n = 8
    buf = oracle.q32_encode(oracle.zero_state(n), n)
    codes, scales = oracle.q32_views(buf, n)
    assert tuple(codes[0]) == (1 << 30, 0) and scales[0] == -30
    assert not codes[1:].any() and (scales[1:] == -128).all()
    oracle.q32_apply_gate(buf, n, 0, [], [], np.array([[1, 1], [1, -1]]) / math.sqrt(2))
    # 2^31 / sqrt(2) = 1518500249.988...
    assert tuple(codes[0]) == (1518500250, 0) and tuple(codes[1]) == (1518500250, 0) and scales[0] == -31
    assert oracle.q32_nbytes(3) == 8 * 8 + 1


def test_q32_exactly_representable_blocks_and_error_bound():
    rng = np.random.default_rng(50)
    n = 9
    N, B = 1 << n, 64
    codes = rng.integers(-(2 ** 31) + 1, 2 ** 31, size=(N, 2)).astype(np.int64)
    scales = rng.integers(-90, -40, size=N // B)
    for b in range(N // B):
        blk = codes[b * B:(b + 1) * B]
        big = int(rng.integers(2 ** 30, 2 ** 31))
        blk[int(rng.integers(0, B)), 0] = big
        np.clip(blk, -big, big, out=blk)
    vals = codes.astype(np.float64) * np.ldexp(1.0, np.repeat(scales, B))[:, None]
    psi = vals[:, 0] + 1j * vals[:, 1]
    buf = oracle.q32_encode(psi, n)
    c2, s2 = oracle.q32_views(buf, n)
    assert np.array_equal(c2, codes) and np.array_equal(s2, scales)
    assert np.array_equal(oracle.q32_decode(buf, n), psi)
    # random state: half-step error, 31 significant bits, decode-encode identity
    psi = _rand_state(n, 51) * np.repeat(10.0 ** rng.uniform(-20, 0, size=N // B), B)
    buf = oracle.q32_encode(psi, n)
    codes, scales = oracle.q32_views(buf, n)
    dec = oracle.q32_decode(buf, n)
    for b in range(N // B):
        blk = slice(b * B, (b + 1) * B)
        m = max(np.abs(psi[blk].real).max(), np.abs(psi[blk].imag).max())
        assert 2 ** 30 <= np.abs(codes[blk]).max() <= 2 ** 31 - 1
        step = math.ldexp(1.0, int(scales[b]))
        assert step <= m * 2.0 ** -30
        assert np.abs(dec[blk] - psi[blk]).max() <= step / 2 * math.sqrt(2)
    assert np.array_equal(oracle.q32_encode(dec, n), buf)
    # saturation and the smallest scale
    v = 1 - 2.0 ** -53
    assert oracle.q32_code(v, oracle.q32_scale(v)) == 2 ** 31 - 1
    tiny = np.zeros(64, dtype=np.complex128)
    tiny[5] = 2.0 ** -120
    bt = oracle.q32_encode(tiny, 6)
    ct, st = oracle.q32_views(bt, 6)
    assert st[0] == -128 and ct[5, 0] == 256 and oracle.q32_decode(bt, 6)[5] == 2.0 ** -120


def test_q32_permutation_gates_exact_and_gate_within_quantisation():
    n = 9
    X = np.array([[0, 1], [1, 0]])
    buf0 = oracle.q32_encode(_rand_state(n, 52), n)
    c0, s0 = oracle.q32_views(buf0, n)
    k = np.arange(1 << n)
    buf = oracle.q32_apply_gate(buf0.copy(), n, 7, [8], [1], X)
    c, s = oracle.q32_views(buf, n)
    assert np.array_equal(c, c0[np.where(k & 256, k ^ 128, k)])
    bi = np.arange(len(s0))
    assert np.array_equal(s, s0[np.where(bi & 4, bi ^ 2, bi)])
    buf = oracle.q32_apply_gate(buf0.copy(), n, 3, [], [], X)
    assert np.array_equal(oracle.q32_views(buf, n)[0], c0[k ^ 8])
    # one Haar gate: within half a step (<= m 2^-31) plus double rounding
    B = 64
    for t, ctrls, vals in ((0, (), ()), (7, (2, 8), (1, 0)), (4, (6,), (1,))):
        U = _rand_unitary(53 + t)
        x = oracle.q32_decode(buf0, n)
        exact = oracle.apply_gate(x.copy(), n, t, ctrls, vals, U)
        out = oracle.q32_decode(oracle.q32_apply_gate(buf0.copy(), n, t, ctrls, vals, U), n)
        cm, cv = oracle.masks(ctrls, vals)
        touched = set(k[(k & cm) == cv] // B)
        for b in range(len(x) // B):
            blk = slice(b * B, (b + 1) * B)
            if b not in touched:
                assert np.array_equal(out[blk], x[blk])
                continue
            m = max(np.abs(exact[blk].real).max(), np.abs(exact[blk].imag).max())
            err = max(np.abs(out[blk].real - exact[blk].real).max(), np.abs(out[blk].imag - exact[blk].imag).max())
            assert err <= m * 2.0 ** -31 * (1 + 1e-9) + 1e-15 * np.abs(x).max(), (t, b, err)


def test_q32_qft_within_rigorous_bound():
    n = 10
    circ = W.qft(n)
    psi0 = _rand_state(n, 54)
    buf = oracle.q32_run_circuit(circ, buf0=oracle.q32_encode(psi0, n))
    N = 1 << n
    rev = np.array([int(format(i, "0%db" % n)[::-1], 2) for i in range(N)])
    want = np.fft.ifft(psi0[rev]) * math.sqrt(N)
    err = np.linalg.norm(oracle.q32_decode(buf, n) - want)
    G = len(circ.gates)
    assert err <= (G + 1) * (math.sqrt(128) * 2.0 ** -31 + 1e-13)
    assert err < 1e-7


def test_thread_count_does_not_change_results():
    """The oracle's parallel loops write disjoint outputs, so one thread and
    all threads give the same bits (the CPU baseline is timed both ways)."""
    n = 14
    psi = W.random_state(n, 3)
    c = W.random_gates_n12(seed=4, n=n, ngates=40)
    threads = oracle.num_threads()
    try:
        oracle.set_num_threads(1)
        one = oracle.run_circuit(c, psi0=psi)
        assert oracle.num_threads() == 1
    finally:
        oracle.set_num_threads(threads)
    every = oracle.run_circuit(c, psi0=psi)
    assert np.array_equal(one, every)
