"""Writes tests/golden/equal_mass_32x16x4.json from the CPU oracle only.

The equal-mass 32x16x4 case (SinhSymTP, 8th order, m = 0.5 at z = +-1,
P = (0, +-0.1, 0), eta = 1, CFL 0.5): residual after every 100 of 1000 RK4
steps and u at a fixed set of stored points. The paper prints no values for
this case, so the file guards the oracle against unintended changes of its
arithmetic; regenerate it only together with a change justified in the
commit message.

Run: python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402

OUT = os.path.join(HERE, "equal_mass_32x16x4.json")
# (i2, i1, i0) of stored points in the extended layout (interior and outer)
SAMPLES = [(0, 0, 0), (1, 3, 5), (2, 8, 16), (3, 15, 31), (0, 7, 33), (2, 12, 35), (1, 0, 20)]


def compute():
    g = oracle.OracleGrid(oracle.SINHSYMTP, 32, 16, 4, 8, bscale=1.0)
    g.set_punctures([0.5, 0.5], [[0, 0, 1.0], [0, 0, -1.0]], [[0, 0.1, 0], [0, -0.1, 0]],
                    np.zeros((2, 3)))
    dt = g.suggest_dt(0.5)
    st, n, hist = g.relax(1.0, 1.0, dt, 1000, 0.0, 100)
    u, _ = g.state()
    ng = g.NG
    ext = u[ng:ng + 4, ng:ng + 16, ng:ng + 32 + ng]
    return {"dt": dt, "residual_history": hist.tolist(),
            "samples": [[list(s), float(ext[s])] for s in SAMPLES]}


if __name__ == "__main__":
    with open(OUT, "w") as f:
        json.dump(compute(), f, indent=1)
    print(f"wrote {OUT}")
