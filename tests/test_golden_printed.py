"""The paper's printed values stored under tests/golden/ (the circuit-level
threshold figure's rotated BP4MF and unrotated BP4M panels, and the B-BP4MF
threshold figure's code-capacity panel):
each file holds the full d x p grid the panel prints, every printed curve
rises with p, and at the lowest p the largest distance is below the smallest.
These files are what bench.py's printed-panel sweeps and the readings study
(oracle/readings.py --bbp4mf) compare against."""
import os

import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    pts = {}
    for ln in open(os.path.join(GOLDEN, name)):
        if ln.startswith("#") or not ln.strip():
            continue
        d, p, v = ln.split()
        pts[(int(d), round(float(p), 3))] = float(v)
    return pts


@pytest.mark.parametrize("name", ["paper_circuit_bp4mf_rotated.txt", "paper_circuit_bp4m_unrotated.txt"])
def test_printed_circuit_panel_grid_and_monotone(name):
    pts = load(name)
    ds = (3, 5, 7, 9, 11)
    ps = [round(0.001 * k, 3) for k in range(2, 13)]
    assert set(pts) == {(d, p) for d in ds for p in ps}
    for d in ds:
        ys = [pts[(d, p)] for p in ps]
        assert all(0.0 < y < 0.5 for y in ys)
        assert all(a < b for a, b in zip(ys, ys[1:])), (d, ys)
    # below threshold the larger distance has the smaller rate (both panels'
    # crossings lie above p = 0.004)
    for p in (0.002, 0.003):
        assert pts[(11, p)] < pts[(3, p)]


def test_printed_bbp4mf_code_capacity_grid_and_monotone():
    pts = load("paper_bbp4mf_code_capacity_unrotated.txt")
    ds = (5, 9, 13)
    ps = [round(0.01 * k, 2) for k in range(3, 19)]
    assert set(pts) == {(d, p) for d in ds for p in ps}
    for d in ds:
        ys = [pts[(d, p)] for p in ps]
        assert all(0.0 < y < 0.5 for y in ys)
        assert all(a < b for a, b in zip(ys, ys[1:])), (d, ys)
    for p in (0.03, 0.05, 0.08):
        assert pts[(13, p)] < pts[(9, p)] < pts[(5, p)]
