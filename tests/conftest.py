import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: long-running CPU case")


@pytest.fixture(scope="session")
def ctx():
    """One library context on cuda:0 for the GPU tests (fails loudly without the HIP library)."""
    import torch
    import paper_1207_1746_amd as G

    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    c = G.Context(0)
    yield c
    c.end()
    c.finalize()


def pytest_runtest_setup(item):
    # name the case before it touches the GPU, so a fault is attributable
    if item.get_closest_marker("gpu") is not None:
        sys.stdout.write(f"\n[gpu-case] {item.nodeid}\n")
        sys.stdout.flush()


@pytest.fixture
def sctx():
    """A library context on a side stream (graph capture needs a non-null
    stream); torch's current stream is the same stream inside the test."""
    import torch
    import paper_1207_1746_amd as G

    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        c = G.Context(0, stream=s)
        yield c
        c.end()
        c.finalize()
