import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C ABI)")
    config.addinivalue_line("markers", "slow: full-size workloads")


def _ensure_cpu_libs():
    """Build the generator and oracle libraries if they are not built yet
    (tests use what is built; they compile only when nothing is)."""
    from paper_1910_05971_amd import build as b
    if not os.path.exists(b.GEN_LIB):
        b.build_gen()
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        import __graft_entry__ as ge
        ge._build_oracle()


_ensure_cpu_libs()


@pytest.fixture(scope="session")
def gpu_ok():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return True
