import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    # The oracle is compiled (only if its library is missing or stale) here,
    # before any test touches the GPU: a process that has initialised the GPU
    # must not start child processes, and oracle.lib() never compiles.
    import oracle
    oracle.build()


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture
def no_gpu_in_process():
    """Skip a test that starts child processes once this process has used
    the GPU (such a process must not start other programs)."""
    t = sys.modules.get("torch")
    if t is not None and t.cuda.is_initialized():
        pytest.skip("this process has used the GPU; child processes are not started from it")
