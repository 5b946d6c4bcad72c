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


# --------------------------------------------------- eps_H against the oracle ---

import pytest

import oracle as o
from paper_2306_08514_amd import native, scenes


def _sbar(n_p, K):
    """Sampling rows exp(j pi k n / K), n = -N_p..N_p, k = 1..K-1."""
    n = np.arange(-n_p, n_p + 1, dtype=np.float64)
    k = np.arange(1, K, dtype=np.float64)
    return np.exp(1j * np.pi * np.outer(n, k) / K)


def _oracle_eps_h(form, x, Np, K, rq):
    """eps_H of (64) with H_type = Lambda_type S formed densely from the
    oracle's own fits."""
    P, J = x.shape
    if form == "slri_global":
        tall, fat = o.slri_global_factors(x, Np, rq)
        lam_all = tall @ fat
    elif form == "sspi_global":
        lam_all = o.sspi_global_select(x, Np, rq * J * P)
    blocks, c0 = [], 0
    for p in range(P):
        n_p = int(Np[p])
        w = 2 * n_p + 1
        if form == "si":
            lam = o.interp_matrix(x[p], n_p)
        elif form == "td":
            lam = np.zeros((J, w))
            r = np.clip(np.sign(x[p]) * np.floor(np.abs(x[p]) + 0.5), -n_p, n_p).astype(int)
            lam[np.arange(J), r + n_p] = 1.0
        elif form == "slri":
            U, V, _ = o.slri_factors(x, Np, rq)[p]
            lam = U @ V.T
        elif form == "sspi":
            lags, wts = o.sspi_select(x[p], n_p, rq)
            lam = np.zeros((J, w))
            np.add.at(lam, (np.repeat(np.arange(J), lags.shape[1]), (lags + n_p).ravel()), wts.ravel())
        else:
            lam = lam_all[:, c0:c0 + w]
        blocks.append(lam @ _sbar(n_p, K))
        c0 += w
    return o.eps_h_db(np.concatenate(blocks, axis=1), o.steering_matrix(x, K))


@pytest.mark.parametrize("name,stride", [("square4_plane1k", 4), ("uca8_room125k", 10)])
@pytest.mark.parametrize("form,variant,rq,glob", [("si", "si", 0, False), ("td", "td", 0, False),
                                                   ("slri", "slri", 4, False), ("slri", "slri", 8, False),
                                                   ("sspi", "sspi", 2, False), ("sspi", "sspi", 4, False),
                                                   ("slri_global", "slri", 24, True),
                                                   ("sspi_global", "sspi", 2, True)])
def test_harness_eps_h_matches_oracle_dense(name, stride, form, variant, rq, glob):
    """The harness's eps_H (per-(location, pair) closed form on the library's
    host-plan fit) against the oracle's dense ||Lambda S - H||^2 / ||H||^2."""
    try:
        native.lib()
    except OSError:
        pytest.skip("library not built")
    cfg = scenes.workload(name, grid_stride=stride)
    x = o.tdoa_samples(cfg["mics"], cfg["grid"], cfg["fs"], cfg["c"])
    Np = o.max_lags(cfg["mics"], cfg["fs"], cfg["c"], 2)
    K = cfg["N"] // 2
    got = ev.eps_h_db(native, cfg, variant, rq, global_fit=glob)
    ref = _oracle_eps_h(form, x, Np, K, rq)
    assert abs(got - ref) <= 1e-6 * max(1.0, abs(ref)), (got, ref)


def test_dirichlet_sum_matches_the_plain_sum():
    K = 37
    t = np.array([0.0, 0.3, -1.7, 2.0, 5.5, 2 * K, -2 * K + 0.25, 11.0])
    k = np.arange(1, K)
    ref = np.cos(np.pi * np.outer(t, k) / K).sum(axis=1)
    np.testing.assert_allclose(ev.dirichlet_sum(t, K), ref, rtol=0, atol=1e-11)
