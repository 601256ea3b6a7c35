"""The oracle's parameter-bound helpers against the worked numbers the
paper prints in Sec. 3.2 (Eq. 18-19), stored under tests/golden/."""

import os

import oracle.sfft_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "eq18_19_worked_examples.txt")


def _rows():
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if line:
            kind, dphi, l, val = line.split()
            yield kind, float(dphi), (None if l == "-" else float(l)), float(val)


def test_eq18_eq19_worked_examples():
    rows = list(_rows())
    assert len(rows) == 6
    for kind, dphi, l, val in rows:
        if kind == "l_upper":
            got = O.multiscale_upper_bound(dphi)
        else:
            got = O.extension_lower_bound(dphi, l)
        # the paper rounds these bounds loosely ("approximately"); the
        # printed value must be within 20% (or 0.2 absolute) of the formula
        assert abs(got - val) <= max(0.2 * val, 0.2), (kind, dphi, l, got, val)
