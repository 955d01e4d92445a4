"""Parser for the hand-worked fixtures in tests/golden/hand_worked.txt."""
import os
from fractions import Fraction

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def _row(tok):
    return [Fraction(t) for t in tok.split()]


def _mat(text):
    return [_row(r) for r in text.split(";")]


def load(name="hand_worked.txt"):
    cases, cur = {}, None
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, rest = line.partition(" ")
            if key == "case":
                cur = {"name": rest}
            elif key == "end":
                cases[cur["name"]] = cur
                cur = None
            elif key in ("A", "L", "U"):
                cur[key] = _mat(rest)
            elif key in ("ipiv",):
                cur[key] = [int(t) for t in rest.split()]
            elif key in ("info",):
                cur[key] = int(rest)
            elif key in ("b", "x"):
                cur[key] = _row(rest)
            elif key == "det":
                cur[key] = Fraction(rest)
            else:
                cur[key] = rest
    return cases


def as_f64(mat):
    """Fraction matrix (row-major lists) -> float64 column-major array (exact for dyadics)."""
    return np.asfortranarray(np.array([[float(x) for x in r] for r in mat], dtype=np.float64))
