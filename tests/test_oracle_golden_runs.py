"""The stored oracle runs under tests/golden/ still describe the oracle as it
stands: its first steps, recomputed, repeat the stored body history bitwise
(a change to the oracle's arithmetic must rewrite the files with
tests/golden/make_oracle_runs.py)."""

import importlib.util
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
spec = importlib.util.spec_from_file_location("make_oracle_runs",
                                              os.path.join(GOLDEN, "make_oracle_runs.py"))
mk = importlib.util.module_from_spec(spec)
spec.loader.exec_module(mk)


@pytest.mark.parametrize("name", sorted(mk.RUNS))
def test_stored_run_repeats_its_first_steps(name):
    with np.load(mk.path_of(name), allow_pickle=False) as z:
        hist, meta = z["history"], json.loads(str(z["meta"]))
    c = mk.RUNS[name]()
    assert meta["steps"] == c.steps == hist.shape[0]
    assert meta["nodes"] == c.mesh.ni * c.mesh.nj
    _, h5, _, _, _ = mk.run(name, steps=4)
    assert np.array_equal(h5, hist[:4])
