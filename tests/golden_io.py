"""Reader for the small text fixtures under tests/golden/."""
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _num(tok):
    return float(Fraction(tok))


def load(name):
    """dict section -> 2D float array (rows of numbers)."""
    out, cur = {}, None
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if line.startswith("[") and line.endswith("]"):
                cur = line[1:-1]
                out[cur] = []
                continue
            out[cur].append([_num(t) for t in line.split()])
    return {k: np.array(v) for k, v in out.items()}
