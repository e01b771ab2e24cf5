"""Full-size parity for the n=28 controlled-gate sweep (complex128 state of
4 GiB, one Haar 2x2, target in {0, 13, 27}, 0-8 controls), in the same
launch configuration the benchmark times.  The oracle computes sampled output
amplitudes one by one from the host copy of the input; the scheduled and
masked kernels must also agree bit for bit over the whole state."""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def big(gpu):
    import torch
    n = 28
    _say("generating n=28 input")
    psi = W.random_state(n, seed=1)
    d_in = torch.from_numpy(psi).cuda()
    yield n, psi, d_in
    del d_in
    torch.cuda.empty_cache()


def _samples(n, t, ctrls, rng):
    N = 1 << n
    idx = [rng.integers(0, N, size=3072, dtype=np.uint64),
           np.arange(512, dtype=np.uint64), np.arange(N - 512, N, dtype=np.uint64)]
    sat = rng.integers(0, N, size=2048, dtype=np.uint64)
    for q in ctrls:
        sat |= np.uint64(1 << q)
    idx.append(sat)
    return np.unique(np.concatenate(idx))


def test_gate_sweep_sampled(gpu, big):
    import torch
    n, psi, d_in = big
    U = oracle.gate_matrix("U", matrix=W.sweep_unitary())
    Ulib = np.asarray(W.sweep_unitary(), dtype=np.float64)
    rng = np.random.default_rng(99)
    work = torch.empty_like(d_in)
    ref_full = torch.empty_like(d_in)
    worst = 0.0
    for t, ctrls in W.gate_sweep_cases(n):
        idx = _samples(n, t, ctrls, rng)
        exp = oracle.gate_amplitudes(psi, n, t, ctrls, (), U, idx)
        tidx = torch.from_numpy(idx.astype(np.int64)).cuda()
        cm = sum(1 << q for q in ctrls)
        modes = []
        for m in ("masked", "auto", "pair", "wave", "tile"):
            try:
                gpu.sv_gate_plan(n, gpu.SV_C128, t, cm, cm, m)
                modes.append(m)
            except gpu.SvError:
                pass
        for mode in modes:
            _say("sweep n=28 t=%d c=%d mode=%s" % (t, len(ctrls), mode))
            work.copy_(d_in)
            gpu.sv_apply_gate(work, t, ctrls, None, Ulib, mode=mode)
            got = work.index_select(0, tidx).cpu().numpy()
            err = float(np.max(np.abs(got - exp)) / np.max(np.abs(exp)))
            worst = max(worst, err)
            assert err <= 1e-12, (t, ctrls, mode, err)
            # amplitudes whose controls fail are untouched, bit for bit
            cm = sum(1 << q for q in ctrls)
            fail = (idx & np.uint64(cm)) != np.uint64(cm)
            assert np.array_equal(got[fail].view(np.uint8), psi[idx[fail]].view(np.uint8))
            if mode == "masked":
                ref_full.copy_(work)
            else:
                assert torch.equal(work.view(torch.float64), ref_full.view(torch.float64)), (t, ctrls, mode)
    _say("sweep worst rel err", worst)


def test_gate_sweep_c64_sampled(gpu, big):
    """complex64 variant of the sweep at n=28, error against the fp64 oracle."""
    import torch
    n, psi, d_in = big
    U = oracle.gate_matrix("U", matrix=W.sweep_unitary())
    Ulib = np.asarray(W.sweep_unitary(), dtype=np.float64)
    rng = np.random.default_rng(98)
    d64 = d_in.to(torch.complex64)
    work = torch.empty_like(d64)
    psi32 = psi.astype(np.complex64).astype(np.complex128)  # the input the c64 path actually sees
    worst = 0.0
    for t, ctrls in W.gate_sweep_cases(n)[::4]:
        idx = _samples(n, t, ctrls, rng)
        exp = oracle.gate_amplitudes(psi32, n, t, ctrls, (), U, idx)
        tidx = torch.from_numpy(idx.astype(np.int64)).cuda()
        for mode in ("auto", "masked"):
            work.copy_(d64)
            gpu.sv_apply_gate(work, t, ctrls, None, Ulib, mode=mode)
            got = work.index_select(0, tidx).cpu().numpy().astype(np.complex128)
            err = float(np.max(np.abs(got - exp)) / np.max(np.abs(exp)))
            worst = max(worst, err)
            assert err <= 1e-5, (t, ctrls, mode, err)
    _say("sweep c64 worst rel err vs fp64 oracle", worst)
    del d64, work
