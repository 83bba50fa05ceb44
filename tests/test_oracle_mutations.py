"""The pins catch plausible mistakes: each case copies the oracle's source,
plants one mistake (a wrong factor, exponent, divisor or derivative), builds
the copy on the CPU and checks that the pin meant for that part fails on it,
while the unmodified oracle passes the same pin (``test_oracle_pins.py``)."""
from __future__ import annotations

import os

import pytest

import oracle
import test_oracle_pins as pins

# (name, text in the source, replacement, the pin that must fail)
MUTATIONS = [
    ("source factor 1/4 instead of 1/8", "g->ssrc[id] = aa / 8.0;", "g->ssrc[id] = aa / 4.0;",
     pins.check_boosted_puncture),
    ("source exponent -6 instead of -7", "std::pow(g.psi[id] + uval, -7.0)",
     "std::pow(g.psi[id] + uval, -6.0)", pins.check_boosted_puncture),
    ("singular conformal factor m/r instead of m/(2r)", "psi += m[p] / (2.0 * r);",
     "psi += m[p] / r;", pins.check_boosted_puncture),
    ("grid norm divided by the padded point count",
     "const double nint = (double)g.N[0] * g.N[1] * g.N[2];",
     "const double nint = (double)g.npad();", pins.check_grid_norm),
    ("grid norm without the square root", "return std::sqrt(tot / nint);", "return tot / nint;",
     pins.check_grid_norm),
    ("SinhSymTP dr/dxx0 = A' / r", "g.drdxx0[k] = A * Ap / r;", "g.drdxx0[k] = Ap / r;",
     pins.check_sinhsymtp_bc),
    ("SinhSymTP dr/dxx0 with sqrt(A^2 + b^2) for r", "g.drdxx0[k] = A * Ap / r;",
     "g.drdxx0[k] = A * Ap / std::sqrt(A * A + g.b * g.b);", pins.check_sinhsymtp_bc),
    ("SinhCylindrical dr/dxx1 = z'", "g.drdxx1[k] = Z * Zp / r;", "g.drdxx1[k] = Zp;",
     pins.check_sinhcylindrical_bc),
    ("SinhCylindrical dr/dxx0 = rho' / r", "g.drdxx0[k] = Ap * A / r;", "g.drdxx0[k] = Ap / r;",
     pins.check_sinhcylindrical_bc),
    ("SinhCylindrical z-face difference not mirrored on the lower face",
     "const int dir = a1 ? (i1 < NG ? -1 : 1) : 1;", "const int dir = 1;",
     pins.check_sinhcylindrical_bc),
    ("Cartesian face difference not mirrored on the lower faces",
     "const int dir = ii[d] < NG ? -1 : 1;   // outward along x_d", "const int dir = 1;",
     pins.check_cartesian_bc),
    ("Cartesian dr/dx_d = 1", "const double drdx = xd / r;", "const double drdx = 1.0;",
     pins.check_cartesian_bc),
    ("Cartesian face difference along x0 on every face",
     "while (ii[d] >= NG && ii[d] < NG + g.N[d]) ++d;", "while (false) ++d;",
     pins.check_cartesian_bc),
]


@pytest.mark.parametrize("name,old,new,check", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pin_catches_planted_mistake(tmp_path, name, old, new, check):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "hr_oracle.cpp")).read()
    assert src.count(old) == 1, f"mutation site not unique or missing: {old!r}"
    path = tmp_path / "hr_oracle_mutant.cpp"
    path.write_text(src.replace(old, new))
    so = oracle.compile_source(str(path), str(tmp_path / "libhr_oracle_mutant.so"))
    oracle.use_library(so)
    try:
        with pytest.raises(AssertionError):
            check(oracle)
    finally:
        oracle.use_library(None)
