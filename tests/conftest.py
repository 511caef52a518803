import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the libsortrace C ABI)")


@pytest.fixture(scope="session")
def gpu():
    """The loaded libsortrace binding; GPU tests require a visible device."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1609_04471_amd import sortrace
    sortrace.load()  # raises if the HIP library is missing: never a silent fallback
    return sortrace
