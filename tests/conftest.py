import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")


_CACHE = {}


def _frame(key, fn):
    if key not in _CACHE:
        _CACHE[key] = fn()
    return _CACHE[key]


@pytest.fixture(scope="session")
def cfg1_frame():
    from paper_2009_07515_amd import synth
    return _frame("cfg1", synth.config1_single_sector)


@pytest.fixture(scope="session")
def cfg2_frame():
    from paper_2009_07515_amd import synth
    return _frame("cfg2", synth.config2_pbpb_event)


@pytest.fixture(scope="session")
def small_pbpb_frame():
    """A 1000-primary Pb-Pb-like event (full TPC) that the oracle tracks in < 1 s."""
    from paper_2009_07515_amd import synth
    return _frame("small", lambda: synth.config2_pbpb_event(seed=4242, n_primary=1000))


@pytest.fixture(scope="session")
def row_x():
    from paper_2009_07515_amd import synth
    return synth.row_x()
