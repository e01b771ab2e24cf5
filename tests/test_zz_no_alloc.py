"""The allocation-free expectation entry point (sv_expect_noalloc) against
sv_expect: same kernels and summation order, so the results must be equal
bit for bit, on two calls in a row (the second smaller), and both within
1e-12 of the oracle."""
import numpy as np
import pytest

import workloads as W


def _terms(n, nterms, seed):
    rng = np.random.default_rng(seed)
    out = [W.PauliTerm(float(rng.standard_normal()), 0, 0)]  # identity: the norm
    for _ in range(nterms - 1):
        x = int(rng.integers(0, 1 << n)) if rng.random() < 0.7 else 0
        z = int(rng.integers(0, 1 << n))
        out.append(W.PauliTerm(float(rng.standard_normal()), x, z))
    return out


@pytest.mark.gpu
def test_expect_noalloc_matches_expect(gpu):
    import torch

    import oracle
    sv = gpu
    for n, nterms, seed in ((20, 64, 101), (11, 5, 102)):  # the second call smaller
        print("noalloc case n=%d nterms=%d seed=%d" % (n, nterms, seed), flush=True)
        psi_h = W.random_state(n, seed)
        psi = torch.from_numpy(psi_h).cuda()
        H = _terms(n, nterms, seed)
        want = sv.sv_expect(psi, H)
        out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        got = sv.sv_expect_noalloc(psi, H, out)
        torch.cuda.synchronize()
        assert got.cpu().numpy().tobytes() == want.cpu().numpy().tobytes(), (got.item(), want.item())
        ref = oracle.expect(psi_h, n, H)
        assert abs(got.item() - ref) <= 1e-12 * max(1.0, abs(ref)), (got.item(), ref)


@pytest.mark.gpu
def test_expect_noalloc_complex64_and_limit(gpu):
    import torch

    import oracle
    sv = gpu
    n = 14
    psi_h = W.random_state(n, 7)
    psi = torch.from_numpy(psi_h.astype(np.complex64)).cuda()
    H = W.zz_x_hamiltonian(n, 8)
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    a = sv.sv_expect(psi, H).cpu().item()
    b = sv.sv_expect_noalloc(psi, H, out).cpu().item()
    assert a == b
    ref = oracle.expect(psi_h.astype(np.complex64).astype(np.complex128), n, H)
    assert abs(b - ref) <= 1e-9 * max(1.0, abs(ref))
    with pytest.raises(sv.SvError, match="allocation-free limit"):
        sv.sv_expect_noalloc(psi, _terms(n, 65, 9), out)
