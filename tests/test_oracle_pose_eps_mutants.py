"""The pose-tolerance pins must catch plausible mistakes: each case plants one
mistake in a private copy of oracle/pose_eps.py and checks that at least one
pin of tests/test_oracle_pose_eps.py fails on it."""

import importlib.util
import os
import sys
import tempfile

import pytest

from oracle import pose_eps
from tests import test_oracle_pose_eps as pins

PINS = [getattr(pins, n) for n in dir(pins) if n.startswith("test_")]

MUTANTS = {
    "depth_R_not_transposed": ("X1 = R0.T @ (ray - rho", "X1 = R0 @ (ray - rho"),
    "depth_wrong_sign": ("(ray - rho * np.asarray", "(ray + rho * np.asarray"),
    "variance_not_sqrt": ("return np.sqrt(best)", "return best"),
    "one_sided_difference": (
        "- distance(F_of(-e, K1, K2, R0, t0), x1, x2)) / (2.0 * STEP)",
        "- distance(F_of(0.0 * e, K1, K2, R0, t0), x1, x2)) / (2.0 * STEP)"),
    "nearest_pair_of_crossings": ("if dd > far:", "if best is None or dd < far:"),
    "unsigned_distance": ("return (l[0] * x2[0] + l[1] * x2[1] + l[2]) / np.hypot(l[0], l[1])",
                          "return abs(l[0] * x2[0] + l[1] * x2[1] + l[2]) / np.hypot(l[0], l[1])"),
    "no_segment_fallback": ("    if not pts:\n        pts = samples(line, W1, H1)\n", ""),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pose_pins_catch_planted_mistake(name, monkeypatch):
    old, new = MUTANTS[name]
    src = open(pose_eps.__file__).read()
    assert src.count(old) == 1, name
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "pose_eps_mutant.py")
        with open(path, "w") as fh:
            fh.write(src.replace(old, new))
        spec = importlib.util.spec_from_file_location("pose_eps_mutant", path)
        mutant = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mutant)
    monkeypatch.setattr(pins, "P", mutant)
    caught = []
    for pin in PINS:
        try:
            pin()
        except (AssertionError, IndexError, ValueError, TypeError, ZeroDivisionError):
            caught.append(pin.__name__)
    assert caught, f"no pin caught mutant {name}"
    assert "pose_eps_mutant" not in sys.modules
