"""The tiling table (csrc/zeus_tiling.inc) and the autotuner's rule
construction: every rule names a tiling that can run the dimensions it covers,
and merging probe choices into ranges keeps each probe's choice."""
import os
import re

from paper_2603_28770_amd import autotune as A

INC = os.path.join(os.path.dirname(A.__file__), "csrc", "zeus_tiling.inc")


def _rules():
    text = open(INC).read()
    return [tuple(int(v) for v in m.groups())
            for m in re.finditer(r"\{\s*(-?\d+),\s*(-?\d+),\s*(-?\d+),\s*(-?\d+),\s*(-?\d+)\s*\}", text)]


def test_table_rules_are_valid():
    for obj, prec, dmin, dmax, lanes in _rules():
        if obj < 0:  # placeholder row
            continue
        assert 0 <= obj <= 6 and prec in (0, 1) and 1 <= dmin <= dmax <= 64
        assert lanes == 256 or (lanes in (2, 4, 8, 16, 32, 64) and lanes >= dmax)


def test_candidates_cover_every_tiling():
    assert A.candidates(3) == [4, 8, 16, 32, 64, 256]
    assert A.candidates(10) == [16, 32, 64, 256]
    assert A.candidates(64) == [64, 256]


def test_rules_from_merges_runs_and_keeps_choices():
    best = {("rastrigin", "fp64"): [(2, 4), (4, 4), (8, 8), (16, 16), (32, 32), (48, 64), (64, 64)],
            ("ackley", "mixed"): [(2, 4), (4, 256), (8, 256)]}
    rules = A.rules_from(best)
    assert [1, 0, 1, 4, 4] in rules and [1, 0, 5, 8, 8] in rules and [1, 0, 33, 64, 64] in rules
    assert [2, 1, 3, 8, 256] in rules

    def lanes_for(obj, prec, d):
        for o, p, lo, hi, lanes in rules:
            if o == obj and p == prec and lo <= d <= hi:
                return lanes
    for (obj, prec), pts in best.items():
        for d, lanes in pts:
            assert lanes_for(A.OBJECTIVES[obj], A.PRECISIONS[prec], d) == lanes
