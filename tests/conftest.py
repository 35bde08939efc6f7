import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU oracle test")


@pytest.fixture
def wall_margin():
    """Factory of a context manager that records, over the oracle steps run
    inside it, the smallest index-space distance |b| from the wall line of the
    wall nodes' departure points found above the wall.  Whether a wall
    population is missing is a floating-point decision (FP32 in the kernel,
    FP64 in the oracle); parity over many steps is meaningful when this margin
    stays well outside the kernel's decision band (1e-5 cells)."""
    import contextlib

    import numpy as np

    @contextlib.contextmanager
    def recorder():
        import oracle.stream as S
        orig = S.departure_offsets
        seen = [np.inf]

        def spy(grid, X, Y, chx, chy, dt, wall_row=False):
            a, b, m = orig(grid, X, Y, chx, chy, dt, wall_row)
            wall = (grid.jj == 0) & grid.wall_col[None, :] & ~np.isnan(b)
            if np.any(wall):
                seen[0] = min(seen[0], float(np.min(np.abs(b[wall]))))
            return a, b, m

        S.departure_offsets = spy
        try:
            yield seen
        finally:
            S.departure_offsets = orig

    return recorder
