"""Host logic of the evaluation harness: the performance measures of
Sec. V-A on hand-made inputs."""

import numpy as np

from paper_2306_08514_amd import evaluate as ev


def test_localisation_error_near_and_far_field():
    grid = np.array([[0.0, 0.0, 0.0], [3.0, 4.0, 0.0], [0.0, 0.0, -1.0], [1.0, 0.0, 0.0]])
    d = ev.localisation_error(grid, np.array([1, 0]), np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0]]), False)
    np.testing.assert_allclose(d, [5.0, 0.0])
    a = ev.localisation_error(grid, np.array([2, 3]), np.array([[1.0, 0.0, 0.0], [1.0, 0.0, 0.0]]), True)
    np.testing.assert_allclose(a, [90.0, 0.0], atol=1e-12)


def test_accuracy_counts_frames_within_threshold():
    r = ev.accuracy(np.array([0.01, 0.05, 0.1, 0.3]), (0.04, 0.08, 0.16))
    assert r == {"0.04": 0.25, "0.08": 0.5, "0.16": 0.75}


def test_map_error_db_is_ten_log_of_squared_norm_ratio():
    z_ref = np.array([[3.0, 4.0], [1.0, 0.0]])
    z = np.array([[3.0, 4.5], [1.0, 0.0]])
    e = ev.map_error_db(z, z_ref)
    np.testing.assert_allclose(e[0], 10 * np.log10(0.25 / 25.0))
    assert e[1] == -np.inf


def test_sweeps_cover_every_form():
    assert set(ev.SWEEPS) == {"fd", "td", "si", "slri", "slri_global", "sspi", "sspi_global", "lr"}
