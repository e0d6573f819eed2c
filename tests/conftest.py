import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line('markers', 'gpu: needs an MI355X (HIP device); run with -m gpu')
    config.addinivalue_line('markers', 'slow: longer CPU oracle runs')


@pytest.fixture(scope='session')
def gpu_lib():
    """The built HIP library, loaded through the Python binding; GPU tests only."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip('no HIP device')
    from paper_2401_15233_amd import solver
    return solver
