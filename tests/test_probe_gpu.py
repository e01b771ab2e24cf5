"""The HBM probe (a measurement helper): read-modify-write and read-only
passes leave a state bit-identical, and the write pass zeroes exactly the
amplitudes whose index bits match the fixed pattern."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_probe_passes(gpu, dtype):
    import torch
    sv = gpu
    n = 16
    psi = W.random_state(n, 61)
    if dtype == "c64":
        psi = psi.astype(np.complex64)
    for mask, vals in ((0, 0), (1 << 7, 1 << 7), ((1 << 0) | (1 << 9) | (1 << 15), 1 << 9)):
        d = torch.from_numpy(psi).cuda()
        sv.sv_hbm_probe(d, mask, vals, "rmw")
        sv.sv_hbm_probe(d, mask, vals, "read")
        torch.cuda.synchronize()
        assert np.array_equal(d.cpu().numpy(), psi)
        sv.sv_hbm_probe(d, mask, vals, "write")
        got = d.cpu().numpy()
        k = np.arange(1 << n)
        sel = (k & mask) == vals
        assert np.all(got[sel] == 0) and np.array_equal(got[~sel], psi[~sel])
