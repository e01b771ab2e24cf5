"""The autotuner measures launch choices on the device, applies the fastest,
writes a cache that loads back, and never changes results."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("granule_bits_c128", "low_policy", "wave_auto", "tile_log2_c128", "tile_low_bits_c128", "dense_min_gates")


def test_autotune_roundtrip_and_results(gpu, tmp_path):
    import torch
    before = {k: gpu.sv_tune_get(k) for k in KEYS}
    cache = str(tmp_path / "tune.json")
    try:
        report = gpu.sv_autotune(18, gpu.SV_C128, cache_path=cache)
        print(report, flush=True)
        chosen = {k: gpu.sv_tune_get(k) for k in KEYS}
        assert "chosen" in report
        # circuits still match the oracle under the chosen knobs
        c = W.random_gates_n12(seed=4, n=14, ngates=300)
        ref = oracle.run_circuit(c)
        d = torch.empty(1 << 14, dtype=torch.complex128, device="cuda")
        gpu.sv_init(d, 0)
        gpu.sv_apply_circuit(d, c, flags=gpu.SV_FUSE)
        assert np.max(np.abs(d.cpu().numpy() - ref)) <= 1e-12
        # the cache restores the same choice
        for k, v in before.items():
            gpu.sv_tune_set(k, v)
        gpu.sv_tune_load(cache)
        assert {k: gpu.sv_tune_get(k) for k in KEYS} == chosen
    finally:
        for k, v in before.items():
            gpu.sv_tune_set(k, v)
