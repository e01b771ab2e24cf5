"""GPU parity of the MFMA dense k-qubit block against the oracle: an explicit
2^k x 2^k matrix on the lowest k qubits (sv_apply_dense_low), and circuits
whose long stretches on those qubits become dense passes (SV_DENSE)."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def _unitary(k, seed):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def _dev(psi, dtype):
    import torch
    t = torch.from_numpy(psi)
    return (t if dtype == "c128" else t.to(torch.complex64)).cuda()


def _err(got, ref):
    return float(np.max(np.abs(got.astype(np.complex128) - ref)) / np.max(np.abs(ref)))


# the block works on whole groups of 64 rows of 2^k amplitudes, so it needs
# n >= k + 6; smaller states are rejected (test below)
DENSE_CASES = [(dt, k, n) for dt, k in (("c128", 4), ("c64", 4), ("c64", 5)) for n in (10, 11, 13, 20)
               if n >= k + 6]


@pytest.mark.parametrize("dtype,k,n", DENSE_CASES)
def test_dense_low_matrix(gpu, dtype, k, n):
    M = _unitary(k, 100 * n + k)
    psi = W.random_state(n, n + k)
    ref = oracle.apply_block_low(psi.copy(), n, k, M)
    d = _dev(psi, dtype)
    gpu.sv_apply_dense_low(d, k, M)
    e = _err(d.cpu().numpy(), ref)
    assert e <= (1e-12 if dtype == "c128" else 1e-5), (dtype, k, n, e)


def test_dense_low_rejects_unsupported(gpu):
    d = _dev(W.random_state(9, 1), "c128")
    with pytest.raises(gpu.SvError) as e:
        gpu.sv_apply_dense_low(d, 4, _unitary(4, 1))  # n < k + 6
    assert e.value.code == gpu.SV_ENOTSUP
    d = _dev(W.random_state(10, 1), "c64")
    with pytest.raises(gpu.SvError) as e:
        gpu.sv_apply_dense_low(d, 5, _unitary(5, 1))  # n < k + 6
    assert e.value.code == gpu.SV_ENOTSUP
    d = _dev(W.random_state(12, 1), "c128")
    with pytest.raises(gpu.SvError):
        gpu.sv_apply_dense_low(d, 5, _unitary(5, 1))  # k=5 is complex64 only


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_circuit_dense_passes(gpu, dtype):
    """Layers of many gates on qubits 0..3 (with device angles) separated by
    gates elsewhere: the plan turns each layer into one dense block."""
    import torch
    n = 14
    rng = np.random.default_rng(7)
    gates, p = [], 0
    for layer in range(4):
        for i in range(24):
            t = int(rng.integers(0, 4))
            others = [q for q in range(4) if q != t]
            c = int(rng.integers(0, 3))
            ctrls = tuple(int(q) for q in rng.choice(others, size=c, replace=False)) if c else ()
            kind = ("H", "RY", "RZ", "X", "P")[i % 5]
            if kind in ("RY", "RZ"):
                gates.append(W.Gate(kind, t, ctrls, (), param=p)); p += 1
            else:
                gates.append(W.Gate(kind, t, ctrls, (), 0.7))
        gates += [W.Gate("H", 4 + layer), W.Gate("X", 9, (4 + layer, 2))]
    circ = W.Circuit(n, gates, rng.uniform(0, 2 * np.pi, size=p))
    psi0 = W.random_state(n, 3)
    ref = oracle.run_circuit(circ, circ.params, psi0)
    params = torch.from_numpy(circ.params).cuda()
    gpu.sv_tune_set("dense_min_gates", 16)
    plan = gpu.Circuit(n, circ, dtype=0 if dtype == "c128" else 1, nparams=p, flags=gpu.SV_FUSE | gpu.SV_DENSE)
    info = plan.info()
    d = _dev(psi0, dtype)
    plan.run(d, params)
    plan.close()
    assert _err(d.cpu().numpy(), ref) <= (1e-12 if dtype == "c128" else 1e-5)
    assert info["passes"] <= 12, info
