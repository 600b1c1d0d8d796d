import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library, loaded once; GPU tests fail loudly if it is missing."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test collected without a visible GPU")
    from paper_2606_12577_amd import cascade
    return cascade


def pytest_terminal_summary(terminalreporter):
    """Print the achieved parity ratios (error / bound) the GPU tests recorded."""
    try:
        import parity
    except ImportError:
        return
    for line in parity.summary_lines():
        terminalreporter.write_line(line)
