"""The oracle reproduces its committed trajectory of the equal-mass 32x16x4 case
(tests/golden/equal_mass_32x16x4.json, written by tests/golden/make_golden.py
from the oracle alone). Guards against unintended changes of its arithmetic."""
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_reproduces_golden_trajectory(oracle_lib):
    import sys
    sys.path.insert(0, os.path.join(HERE, "golden"))
    import make_golden

    with open(os.path.join(HERE, "golden", "equal_mass_32x16x4.json")) as f:
        ref = json.load(f)
    got = make_golden.compute()
    assert got["dt"] == ref["dt"]
    np.testing.assert_allclose(got["residual_history"], ref["residual_history"], rtol=1e-12)
    for (s, v), (s2, v2) in zip(got["samples"], ref["samples"]):
        assert s == s2
        np.testing.assert_allclose(v, v2, rtol=1e-12, atol=1e-18)
