import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def tiny():
    import synth
    return synth.workload_tiny()


@pytest.fixture(scope="session")
def tiny_oracle(tiny):
    import oracle
    return oracle.Model.from_workload(tiny)


@pytest.fixture(scope="session")
def tiny_keys(tiny):
    import oracle
    return [oracle.shell_keys(tiny.verts, tiny.tris, N, tiny.dilate) for N in tiny.res]
