import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")


def read_golden(name: str) -> dict:
    """key=value fixture lines (comments start with #)."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split("=", 1)
            out[k.strip()] = v.strip()
    return out


@pytest.fixture(scope="session")
def gpu_ctx():
    """A libpaf context on cuda:0.  A GPU test fails (it does not skip) when
    there is no GPU or no library: the parity claims need the HIP path."""
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1910_03936_amd as paf

    ctx = paf.Context(0)
    yield ctx
    ctx.close()
