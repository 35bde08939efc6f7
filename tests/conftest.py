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
    inside it, the smallest index-space distance of the wall nodes' departure
    points (found or missing) from the line at which a population counts as
    missing (WALL_TOL below the wall line).  Both sides decide at that line,
    the oracle in FP64, the kernel in FP32 and, within 1e-5 of the line, in
    FP64; parity over many steps is meaningful when no point comes closer to
    it than the differences of two FP64 evaluations (~1e-13 cells)."""
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
                seen[0] = min(seen[0], float(np.min(np.abs(b[wall] + S.WALL_TOL))))
            return a, b, m

        S.departure_offsets = spy
        try:
            yield seen
        finally:
            S.departure_offsets = orig

    return recorder
