"""The one-pass scan and the profile scan reproduce the enumerated fixtures."""
import glob
import json
import os

import numpy as np
import pytest

import oracle as O

FIX = sorted(glob.glob(os.path.join(os.path.dirname(__file__), "golden", "*.json")))


def load(path):
    d = json.load(open(path))
    e = np.array(d["edges"], np.uint32).reshape(-1, 4)
    return d, e


@pytest.mark.parametrize("path", FIX, ids=[os.path.basename(p) for p in FIX])
def test_golden_fixture(path, oracle_mod):
    d, e = load(path)
    se = O.sort_by_departure(d["n"], e[:, 0], e[:, 1], e[:, 2], e[:, 3])
    ea = O.earliest_arrival(se, d["source"], d["t_alpha"], d["t_omega"])
    pea, pld, pf = O.profile(se, d["source"], d["t_alpha"], d["t_omega"])
    assert ea.tolist() == d["ea"] == pea.tolist()
    assert pld.tolist() == d["ld"]
    assert pf.tolist() == d["fastest"]


def test_fixtures_present():
    assert len(FIX) >= 5
