import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP) device")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        oracle.build(force=True)
    return oracle


@pytest.fixture(scope="session")
def synth_lib():
    import synth
    if not os.path.exists(os.path.join(ROOT, "synth", "libsynth.so")):
        synth.build(force=True)
    return synth


@pytest.fixture(scope="session")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2411_10258_amd as mdhp  # raises if libmdhp.so is missing
    from paper_2411_10258_amd import _lib
    _lib.load()
    return mdhp
