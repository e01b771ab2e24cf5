import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def _gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def gpu():
    if not _gpu_available():
        pytest.skip("no GPU visible")
    import paper_2411_18354_amd as sv
    return sv


@pytest.fixture(autouse=True)
def _restore_tuning():
    """Tests may change the library's launch knobs; each one ends with the
    values it started with."""
    try:
        import paper_2411_18354_amd as mod
        saved = {k: mod.sv_tune_get(k) for k in mod.TUNE_KEYS}
    except (ImportError, OSError):
        saved = None
    yield
    if saved is not None:
        for k, v in saved.items():
            mod.sv_tune_set(k, v)
