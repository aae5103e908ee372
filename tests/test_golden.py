"""The oracle's strut integral against hand-derived exact values
(tests/golden/strut_integral_exact.txt: Sec. 3.2, Eqs. 5-6)."""
import os
from fractions import Fraction

import numpy as np

from oracle import field as OF

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "strut_integral_exact.txt")


def cases():
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if not line:
            continue
        tok = line.split()
        R = float(tok[0])
        a, b, p = (np.array([float(x) for x in tok[i:i + 3]]) for i in (1, 4, 7))
        exact = Fraction(int(tok[10]), int(tok[11]))
        yield R, a, b, p, exact, " ".join(tok[12:])


def test_golden_file_is_complete():
    assert len(list(cases())) == 10


def test_strut_integral_matches_exact_values():
    for R, a, b, p, exact, what in cases():
        got = float(OF.strut_integral(p[None], a, b, R)[0])
        assert abs(got - float(exact)) <= 1e-13 * max(1.0, float(exact)), (what, got, exact)
        # the edge's orientation does not matter
        back = float(OF.strut_integral(p[None], b, a, R)[0])
        assert abs(back - got) <= 1e-13 * max(1.0, abs(got)), what
