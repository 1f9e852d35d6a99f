"""Golden fixtures copied from the paper, with citations inside each file."""
import json
import math
import os

import pytest

from seeded_inputs import WORKLOADS, eps_table1_24

HERE = os.path.dirname(os.path.abspath(__file__))


def test_table1_24_site_radii():
    """The 24-site workload uses Table I's discretisation: E_b = -5, L = 128, M = 16 and the
    printed radii (including the T = 0.2 expression (14 ln 10) x 0.2 / 128 / 2)."""
    with open(os.path.join(HERE, "golden", "table1_delta.json")) as f:
        rows = [r for r in json.load(f)["rows"] if r["sites"] == 24]
    w = WORKLOADS["plain-N24"]
    for r in rows:
        T = math.inf if r["T"] == "inf" else r["T"]
        eps = 14 * math.log(10) * 0.2 / 128 / 2 if isinstance(r["eps"], str) else r["eps"]
        assert eps_table1_24(T) == pytest.approx(eps, rel=1e-15)
        assert (r["E_b"], r["L"], r["M"]) == (w["E_b"], w["L"], w["M"])
        # the low-temperature rows only cover the bottom of the spectrum
        assert (r["E_b"] + 2 * r["L"] * eps > 0) == (T >= 0.2)


def test_table1_windows_are_contiguous():
    """Every row of Table I covers [E_b, E_b + 2 eps L] with shells of width 2 eps."""
    with open(os.path.join(HERE, "golden", "table1_delta.json")) as f:
        rows = json.load(f)["rows"]
    for r in rows:
        eps = 14 * math.log(10) * 0.2 / 128 / 2 if isinstance(r["eps"], str) else r["eps"]
        assert r["M"] % 2 == 0  # even M keeps every contour node off the real axis
        assert 2 * r["L"] * eps > 2.0
