"""Pins for the oracle's bookkeeping helpers: the borderline margin that
excuses GPU/oracle active-set differences (C9 reading), and the error rates.

Every expected value below is worked out by hand, so that a wrong k, a min
over the wrong axis or a dropped endpoint fails."""

import numpy as np
import pytest

from oracle.metrics import margin, rel_err, set_recall


def test_margin_hand_cases():
    # cell 0: bound [-2, 2]; distances to 0.5: 2.5, 1.5; to 3: 5, 1 -> 1
    # cell 1: bound [0, 2];  distances to 0.5: 0.5, 1.5; to 3: 3, 1 -> 0.5
    # cell 2: bound [4, 4] (zero spread); distances 3.5 and 1 -> 1
    centre = np.array([0.0, 1.0, 4.0])
    spread = np.array([1.0, 0.5, 0.0])
    m = margin(centre, spread, 2.0, [0.5, 3.0])
    np.testing.assert_allclose(m, [1.0, 0.5, 1.0], rtol=0, atol=1e-15)


def test_margin_uses_k_and_both_endpoints():
    # k scales the spread: bound [1 - 3*0.25, 1 + 3*0.25] = [0.25, 1.75]
    m = margin(np.array([1.0]), np.array([0.25]), 3.0, [1.7])
    assert m[0] == pytest.approx(0.05, abs=1e-15)  # upper endpoint is the closer one
    m = margin(np.array([1.0]), np.array([0.25]), 3.0, [0.3])
    assert m[0] == pytest.approx(0.05, abs=1e-15)  # lower endpoint
    # an iso-value exactly on an endpoint gives margin 0
    m = margin(np.array([1.0]), np.array([0.25]), 3.0, [0.25])
    assert m[0] == 0.0
    # an iso-value inside the bound but far from both endpoints still counts
    # its distance to the nearer endpoint, not to the centre
    m = margin(np.array([0.0]), np.array([1.0]), 1.0, [0.0])
    assert m[0] == pytest.approx(1.0)


def test_margin_min_over_isovalues_per_cell():
    # the min runs over iso-values within each cell, never across cells
    centre = np.array([0.0, 10.0])
    spread = np.array([0.0, 0.0])
    m = margin(centre, spread, 1.0, [0.25, 9.0])
    np.testing.assert_allclose(m, [0.25, 1.0])


def test_rel_err_and_recall_hand_cases():
    np.testing.assert_allclose(rel_err([1.5, 0.01], [1.0, 0.0], 0.5), [0.5, 0.02])
    assert set_recall([1, 2, 3, 7], [2, 3, 4, 5]) == pytest.approx(0.5)
    assert set_recall([1], []) == 1.0
