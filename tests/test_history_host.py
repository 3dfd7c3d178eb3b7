"""Host logic of the error-history harness (no GPU): markers of an error curve."""
import numpy as np

from paper_2110_01481_amd.history import markers


def test_markers_minimum_and_stops():
    e = np.array([0.9, 0.5, 0.31, 0.3, 0.3, 0.34, 0.5])
    k_min, e_min, e_dp, e_ncp = markers(e, 3, 2)
    assert (k_min, e_min) == (4, 0.3)          # first of equal values
    assert e_dp == 0.31 and e_ncp == 0.5


def test_markers_missing_or_out_of_range_stops():
    e = np.array([0.9, 0.5])
    assert markers(e, None, 0)[2:] == (None, None)   # k = 0 is x_0: no curve entry
    assert markers(e, 3, None)[2] is None
    k_min, e_min, e_dp, e_ncp = markers(np.zeros(0), 1, 1)
    assert k_min == 0 and np.isnan(e_min) and e_dp is None and e_ncp is None
