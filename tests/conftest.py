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


# the benchmark's tuning of the 2 ms frame (grid bins 2 x 4 cm, at most 4n + 64 bins per row)
CFG3_TUNING = dict(bin_y=2.0, bin_z=4.0, cap_mul=4, block=512, tl_block=256, chunk=2)
CFG3_GRID = dict(bin_y=2.0, bin_z=4.0, cap_mul=4, cap_add=64)


@pytest.fixture(scope="session")
def cfg3_frame():
    """The 2 ms continuous-readout Pb-Pb time frame (27.1M clusters), generated once."""
    from paper_2009_07515_amd import synth
    return _frame("cfg3", synth.config3_time_frame)


@pytest.fixture(scope="session")
def cfg3_oracle(cfg3_frame, row_x):
    """The FP64 oracle on the whole 2 ms frame with the benchmark's grid, sectors in
    parallel."""
    import oracle_sectors

    def run():
        f = cfg3_frame
        return oracle_sectors.track_frame_parallel(row_x, f.y, f.z, f.row_off, grid=CFG3_GRID)
    return _frame("cfg3_oracle", run)


@pytest.fixture(scope="session")
def cfg4_frames():
    """The 64 frames of the uneven batch (pp-like and Pb-Pb-like alternating), generated
    once in worker processes."""
    from paper_2009_07515_amd import synth
    return _frame("cfg4", lambda: synth.config4_batch(64))
