"""The campaign harness's summaries.  RoFT (the equation after Fig. 1 of the
paper) is pinned by every row the paper prints in Tables 2 and 3: the
printed value must follow from the printed iteration means and the caption's
baseline up to the rounding of the printed numbers."""
import csv
import os

import pytest

from paper_2103_07210_amd.campaign import roft, summarize

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_tables_2_3_roft.csv")


def _rows():
    with open(GOLDEN) as f:
        lines = [l for l in f if not l.startswith("#")]
    return list(csv.DictReader(lines))


def test_roft_reproduces_paper_tables():
    rows = _rows()
    assert len(rows) == 42
    for r in rows:
        base = float(r["baseline"])
        got = roft(float(r["gcr"]), float(r["ft_gcr"]), base)
        # the means are printed to 2 decimals (half-unit 0.005 each), the
        # RoFT itself to 2 decimals
        bound = 100.0 * 0.01 / base + 0.005
        assert abs(got - float(r["roft_printed"])) <= bound, r
    # the formula's orientation matters: swapped arguments fail
    r = rows[28]
    assert abs(roft(float(r["ft_gcr"]), float(r["gcr"]), 21) - float(r["roft_printed"])) > 1.0


def test_summarize_counts_detections_and_extra_steps():
    recs = [
        dict(events_applied=1, detections=1, steps=102, steps_off=110, err=0.0, err_off=1e-3, vec="r"),
        dict(events_applied=1, detections=0, steps=100, steps_off=100, err=1e-9, err_off=1e-9, vec="x"),
        dict(events_applied=0, detections=0, steps=100, steps_off=100, err=0.0, err_off=0.0, vec="p"),
        dict(events_applied=1, detections=1, steps=104, steps_off=101, err=0.0, err_off=2e-6, vec="ap"),
    ]
    s = summarize(recs, clean_steps=100)
    assert s["runs"] == 4 and s["runs_with_fault"] == 3
    assert s["detection_rate"] == pytest.approx(2 / 3)
    assert s["extra_steps_mean"] == pytest.approx(2.0) and s["extra_steps_max"] == 4
    assert s["bitwise_equal_to_fault_free"] == 2
    assert s["roft_percent"] == pytest.approx(100 * ((110 + 100 + 101) / 3 - (102 + 100 + 104) / 3) / 100)
    assert s["detection_rate_by_vector"] == {"r": 1.0, "x": 0.0, "ap": 1.0}


def test_octahedral_process_bands_and_grid_text():
    """On O_N a process owns a contiguous range of points (latitude bands of
    the ring-by-ring numbering) at every level; the bands partition the
    mesh.  'O40' names the paper's O40 with its 51 levels (Table 1)."""
    import numpy as np
    from paper_2103_07210_amd import inputs as I
    from paper_2103_07210_amd.campaign import grid_label, parse_grid
    pb = I.OctProblem(4, 3)
    procs = 5
    owned = np.concatenate([I.process_entries(pb, procs, r) for r in range(procs)])
    assert np.array_equal(np.sort(owned), np.arange(pb.n))
    band = I.process_entries(pb, procs, 2)
    pts = np.unique(band % pb.points)
    assert pts.size * pb.nz == band.size and np.all(np.diff(pts) == 1)
    o40 = parse_grid("O40")
    assert (o40.N, o40.nz, o40.n) == (40, 51, 399840)
    assert grid_label(parse_grid("O16x8")) == ["O16", 8]
    assert grid_label(parse_grid("64,32,8")) == [64, 32, 8]
