"""GPU parity of the block-scaled 16-bit fixed-point states (SV_CQ16).

The library and the oracle follow the same definition: decode to float, the
pair update in float with a fixed fused multiply-add order, re-encode every
block an updated pair touches.  Codes and scales are integers, so parity is
bit-exact: the state bytes must be identical.  The error against the
double-precision oracle is checked against the rigorous norm bound of the
format and reported.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads as W

sv = pytest.importorskip("paper_2411_18354_amd")

pytestmark = pytest.mark.gpu


def _dev(buf):
    return torch.from_numpy(np.ascontiguousarray(buf)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _encode_gpu(psi, n):
    src = torch.from_numpy(psi).cuda()
    q = sv.fixed_state(n)
    sv.sv_convert(q, src)
    return q


def _diff_report(got, want, n):
    gc, gs = oracle.q16_views(got, n)
    wc, ws = oracle.q16_views(want, n)
    bad_c = np.nonzero((gc != wc).any(axis=1))[0]
    bad_s = np.nonzero(gs != ws)[0]
    return "codes differ at %d amplitudes (first %s), scales at %d blocks (first %s)" % (
        len(bad_c), bad_c[:5].tolist(), len(bad_s), bad_s[:5].tolist())


def _assert_same(got, want, n, what=""):
    assert got.shape == want.shape
    if not np.array_equal(got, want):
        pytest.fail("%s: %s" % (what, _diff_report(got, want, n)))


@pytest.mark.parametrize("n", [1, 3, 5, 6, 7, 12, 16])
def test_convert_encode_decode_bit_exact(n):
    psi = W.random_state(n, 100 + n)
    psi[: min(64, 1 << n) // 2] *= 1e-9  # blocks of very different magnitude
    want = oracle.q16_encode(psi, n)
    q = _encode_gpu(psi, n)
    _assert_same(_host(q), want, n, "encode from complex128")
    out = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    sv.sv_convert(out, q)
    assert np.array_equal(_host(out), oracle.q16_decode(want, n))
    # complex64 in and out: the float values are the ones encoded
    p64 = torch.from_numpy(psi.astype(np.complex64)).cuda()
    q2 = sv.fixed_state(n)
    sv.sv_convert(q2, p64)
    _assert_same(_host(q2), oracle.q16_encode(psi.astype(np.complex64).astype(np.complex128), n), n,
                 "encode from complex64")
    o64 = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    sv.sv_convert(o64, q2)
    assert np.array_equal(_host(o64).astype(np.complex128), oracle.q16_decode(_host(q2), n))
    # complex128 <-> complex64 round to nearest / widen exactly
    c64 = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    sv.sv_convert(c64, torch.from_numpy(psi).cuda())
    assert np.array_equal(_host(c64), psi.astype(np.complex64))


@pytest.mark.parametrize("n,b", [(1, 1), (3, 5), (6, 63), (7, 64), (12, 4095), (12, 1234)])
def test_init_basis_bit_exact(n, b):
    q = sv.fixed_state(n)
    q.fill_(0xA5)  # garbage the init must overwrite
    sv.sv_init(q, b)
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[b] = 1.0
    _assert_same(_host(q), oracle.q16_encode(psi, n), n, "basis %d" % b)


def _gate_cases(n, rng, count):
    """(target, controls, values) cases: no controls, in-block controls only,
    block-index controls only, mixed, negative values; targets low and high."""
    cases = []
    targets = sorted({t for t in (0, 1, 2, 5, 6, 7, n - 1, int(rng.integers(0, n))) if t < n})
    for t in targets:
        others = [q for q in range(n) if q != t]
        low = [q for q in others if q < 6]
        high = [q for q in others if q >= 6]
        opts = [()]
        if low:
            opts.append(tuple(rng.choice(low, size=min(2, len(low)), replace=False)))
        if high:
            opts.append(tuple(rng.choice(high, size=min(2, len(high)), replace=False)))
        if low and high:
            opts.append((int(rng.choice(low)), int(rng.choice(high))))
        for ctrls in opts:
            ctrls = tuple(int(c) for c in ctrls)
            vals = tuple(int(v) for v in rng.integers(0, 2, size=len(ctrls)))
            cases.append((t, ctrls, vals))
    rng.shuffle(cases)
    return cases[:count]


@pytest.mark.parametrize("n", [1, 2, 4, 5, 6, 7, 9, 13])
@pytest.mark.parametrize("mode", ["auto", "masked"])
def test_single_gates_bit_exact(n, mode):
    rng = np.random.default_rng(200 + n)
    psi = W.random_state(n, 300 + n)
    ref = oracle.q16_encode(psi, n)
    q = _dev(ref)
    for i, (t, ctrls, vals) in enumerate(_gate_cases(n, rng, 24)):
        U = oracle.gate_matrix("U", matrix=W.haar_unitary_2x2(400 + i))
        cm, cv = oracle.masks(ctrls, vals)
        sv.sv_apply_gate(q, t, ctrls, cv, np.asarray(W.haar_unitary_2x2(400 + i)), mode=mode)
        oracle.q16_apply_gate(ref, n, t, ctrls, vals, U)
        _assert_same(_host(q), ref, n, "gate %d: t=%d controls=%s values=%s" % (i, t, ctrls, vals))


def test_scheduled_and_masked_agree_bitwise_n20():
    n = 20
    psi = W.random_state(n, 21)
    base = oracle.q16_encode(psi, n)
    U = np.asarray(W.haar_unitary_2x2(22))
    for t, ctrls in ((19, (3, 11)), (2, (0, 7, 15)), (10, ()), (0, (19,))):
        a, b = _dev(base), _dev(base)
        sv.sv_apply_gate(a, t, ctrls, None, U, mode="auto")
        sv.sv_apply_gate(b, t, ctrls, None, U, mode="masked")
        assert torch.equal(a, b), (t, ctrls)
        want = oracle.q16_apply_gate(base.copy(), n, t, ctrls, (), oracle.gate_matrix("U", matrix=tuple(U)))
        _assert_same(_host(a), want, n, "t=%d controls=%s" % (t, ctrls))


def _named_matrices_agree(circ):
    """The float matrices both sides use are equal (each side computes the
    named gates' doubles itself; rounding to float must give the same)."""
    for g in circ.gates:
        mine = np.asarray(sv.sv_gate_matrix(g.kind, g.theta, g.matrix)).astype(np.float32)
        U = oracle.gate_matrix(g.kind, g.theta, g.matrix)
        ora = np.stack([U.real, U.imag], axis=-1).reshape(8).astype(np.float32)
        assert np.array_equal(mine, ora), g


@pytest.mark.parametrize("flags", [0, 4])  # unfused scheduled, masked
def test_random_circuit_bit_exact(flags):
    circ = W.random_gates_n12(seed=0)
    n = circ.n
    _named_matrices_agree(circ)
    want = oracle.q16_run_circuit(circ)
    q = sv.fixed_state(n)
    sv.sv_init(q, 0)
    sv.sv_apply_circuit(q, circ, flags=flags)
    _assert_same(_host(q), want, n, "random_gates_n12 flags %d" % flags)


def test_haar_circuit_with_graph_replays():
    rng = np.random.default_rng(31)
    n = 14
    gates = []
    for i in range(120):
        t = int(rng.integers(0, n))
        others = [q for q in range(n) if q != t]
        nc = int(rng.integers(0, 4))
        ctrls = tuple(int(c) for c in rng.choice(others, size=nc, replace=False)) if nc else ()
        vals = tuple(int(v) for v in rng.integers(0, 2, size=nc))
        gates.append(W.Gate("U", t, ctrls, vals, matrix=W.haar_unitary_2x2(1000 + i)))
    circ = W.Circuit(n, gates)
    psi = W.random_state(n, 32)
    start = oracle.q16_encode(psi, n)
    want = oracle.q16_run_circuit(circ, buf0=start)
    eager = _dev(start)
    sv.sv_apply_circuit(eager, circ, flags=0)
    _assert_same(_host(eager), want, n, "eager")
    plan = sv.Circuit(n, circ, dtype=sv.SV_CQ16, flags=sv.SV_GRAPH)
    q = _dev(start)
    for rep in range(3):  # replays with eager work and synchronisation between
        q.copy_(_dev(start))
        torch.cuda.synchronize()
        plan.run(q)
        torch.cuda.synchronize()
        assert torch.equal(q, eager), "replay %d" % rep
    assert plan.info()["passes"] == len(gates)
    plan.close()


def test_parameterised_circuit_within_bound():
    """Angles on the device: the matrices are computed there in double and
    rounded to float, so the result is checked against the double oracle
    within the format's bound (and against the fixed-point oracle, which
    must agree to within one code step per gate)."""
    circ = W.hea(8, 3, seed=33)
    n = circ.n
    params = torch.from_numpy(circ.params).cuda()
    q = sv.fixed_state(n)
    sv.sv_init(q, 0)
    sv.sv_apply_circuit(q, circ, params=params, flags=0)
    got = oracle.q16_decode(_host(q), n)
    exact = oracle.run_circuit(circ)
    G = len(circ.gates)
    assert np.linalg.norm(got - exact) <= (G + 1) * (math.sqrt(128) * 2.0 ** -15 + 1e-6)
    ref = oracle.q16_decode(oracle.q16_run_circuit(circ), n)
    assert np.abs(got - ref).max() <= 1e-3


def test_qft_error_against_double_oracle():
    """The QFT as drawn (no swaps): error of the fixed-point result against
    its closed form, within the rigorous bound, beside complex64's."""
    n = 16
    circ = W.qft(n)
    psi0 = W.random_state(n, 34)
    N = 1 << n
    rev = np.array([int(format(i, "0%db" % n)[::-1], 2) for i in range(N)])
    want = np.fft.ifft(psi0[rev]) * math.sqrt(N)
    q = _encode_gpu(psi0, n)
    sv.sv_apply_circuit(q, circ, flags=0)
    err = np.linalg.norm(oracle.q16_decode(_host(q), n) - want)
    G = len(circ.gates)
    assert err <= (G + 1) * (math.sqrt(128) * 2.0 ** -15 + 1e-6)
    assert err < 2e-2
    c64 = torch.from_numpy(psi0.astype(np.complex64)).cuda()
    sv.sv_apply_circuit(c64, circ, flags=0)
    err64 = np.linalg.norm(_host(c64).astype(np.complex128) - want)
    print("QFT n=%d: fixed-point error %.3e, complex64 error %.3e (2-norm)" % (n, err, err64))
    assert err64 < err  # 16-bit codes carry fewer bits than float


def test_full_size_n28_bit_exact():
    """The bench's configuration: n = 28 (1 GiB state), high and low targets,
    scheduled and masked kernels, whole-state comparison."""
    n = 28
    psi = W.random_state(n, 1)
    ref = oracle.q16_encode(psi, n)
    del psi
    q = _dev(ref)
    for t, ctrls, vals, mode in ((27, (0, 13), (1, 1), "auto"), (0, (14, 27), (1, 0), "masked"),
                                 (13, (), (), "auto")):
        U = W.haar_unitary_2x2(2)
        sv.sv_apply_gate(q, t, ctrls, oracle.masks(ctrls, vals)[1], np.asarray(U), mode=mode)
        oracle.q16_apply_gate(ref, n, t, ctrls, vals, oracle.gate_matrix("U", matrix=U))
        got = _host(q)
        assert np.array_equal(got, ref), "t=%d controls=%s %s: %s" % (t, ctrls, mode, _diff_report(got, ref, n))


def test_x_on_top_qubit_swaps_halves_n32():
    """n = 32 (16 GiB state): X on qubit 31 exchanges the two halves exactly
    (codes and scales), a property of any correct implementation."""
    n = 32
    q = sv.fixed_state(n)
    N = 1 << n
    codes = q[: 4 * N].view(torch.int16)
    gen = torch.Generator(device="cuda").manual_seed(35)
    codes.copy_(torch.randint(-32767, 32767, (2 * N,), device="cuda", dtype=torch.int16, generator=gen))
    scales = q[4 * N:].view(torch.int8)
    scales.copy_(torch.randint(-40, -20, (N // 64,), device="cuda", dtype=torch.int8, generator=gen))
    # make every block a valid encoding: largest magnitude at least 2^14
    codes.view(N // 64, 128)[:, 0] = 20000
    before = q.clone()
    sv.sv_apply_gate(q, 31, (), None, np.array([[0, 1], [1, 0]]))
    torch.cuda.synchronize()
    h = 2 * N  # bytes per half of the codes
    assert torch.equal(q[:h], before[h:4 * N]) and torch.equal(q[h:4 * N], before[:h])
    hs = N // 128
    assert torch.equal(q[4 * N:4 * N + hs], before[4 * N + hs:]) and torch.equal(q[4 * N + hs:], before[4 * N:4 * N + hs])
