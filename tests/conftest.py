import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def dev():
    """The GPU device; GPU tests fail loudly if the HIP library cannot be loaded."""
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test collected on a machine without a GPU")
    from paper_1908_05845_amd import smmo

    smmo.load_library()   # raises if libsmmo.so is missing
    return torch.device("cuda:0")


def pytest_terminal_summary(terminalreporter):
    """Break-decision ties met by the GPU parity checks of this session, and
    the end-to-end drift of unrestarted float32 runs from the float64
    trajectory (reported, not gated)."""
    mod = sys.modules.get("spring_parity")
    if mod is None:
        return
    t = mod.TIES
    if t["checked_spring_steps"]:
        terminalreporter.write_line(
            "spring break decisions: %d checked steps; springs within the tie band of the limit: %d; "
            "decided by the GPU otherwise than the float64 rule: %d" % (t["checked_spring_steps"], t["near"],
                                                                       t["flipped"]))
    for rec in mod.DRIFT:
        terminalreporter.write_line("float32 run vs float64 trajectory: %s" % rec)
