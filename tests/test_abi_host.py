"""CPU tests of the C ABI: the library loads, exports every declared symbol,
validates its arguments, and its FP64 host plan (pairs, TDOAs, lag ranges,
SLRI factors, SSPI windows) agrees with the oracle.  No device calls."""

import ctypes
import os
import re

import numpy as np
import pytest

import oracle as o
from paper_2306_08514_amd import native, scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_or_skip():
    if not os.path.exists(native.LIB_PATH):
        pytest.skip("libsrp.so not built")
    return native.lib()


def test_library_exports_every_declared_symbol():
    L = _lib_or_skip()
    hdr = open(os.path.join(ROOT, "include", "srp.h")).read()
    declared = set(re.findall(r"^\s*(?:srp_status|void|const char\*)\s+(srp_\w+)\s*\(", hdr, re.M))
    assert declared == set(native.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def _host_plan(variant, rq, name="square4_plane1k", stride=4, **kw):
    cfg = scenes.workload(name, grid_stride=stride)
    p = native.Plan(cfg["mics"], cfg["grid"], cfg["fs"], cfg["N"], variant, rq, device=-1, **kw)
    return p, cfg


def test_host_plan_geometry_matches_oracle():
    _lib_or_skip()
    p, cfg = _host_plan("sspi", 4, name="uca8_room125k", stride=7)
    x_ref = o.tdoa_samples(cfg["mics"], cfg["grid"], cfg["fs"], cfg["c"])
    x = p.export("tdoa").reshape(x_ref.shape)
    np.testing.assert_allclose(x, x_ref, rtol=0, atol=1e-11)
    np.testing.assert_array_equal(p.export("np"), o.max_lags(cfg["mics"], cfg["fs"], cfg["c"], 2))
    np.testing.assert_array_equal(p.export("pairs").reshape(-1, 2), np.array(o.pairs(8)))
    info = p.info()
    assert info["PN"] == 660 and info["P"] == 28 and info["K"] == 512
    assert info["mean_n"] == pytest.approx(660 / 28)
    assert info["device_bytes"] == 0


def test_host_plan_far_field_geometry_matches_oracle():
    _lib_or_skip()
    mics = scenes.uca(8, 0.3)
    u = scenes.half_sphere_directions(4.0)
    p = native.Plan(mics, u, 16000.0, 1024, "sspi", 4, device=-1, far_field=True)
    x_ref = o.tdoa_samples_far_field(mics, u, 16000.0, 343.0)
    np.testing.assert_allclose(p.export("tdoa").reshape(x_ref.shape), x_ref, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(p.export("np"), o.max_lags(mics, 16000.0, 343.0, 2))
    p.close()
    with pytest.raises(native.SrpError):
        native.Plan(mics, 1.5 * u, 16000.0, 1024, "fd", device=-1, far_field=True)


def test_host_plan_slri_factors_match_oracle_svd():
    """U_p V_p^T (the rank-R truncation, unique when sigma_R > sigma_{R+1})
    agrees with numpy's SVD; singular values agree."""
    _lib_or_skip()
    R = 5
    p, cfg = _host_plan("slri", R, name="uca8_room125k", stride=5)
    x = o.tdoa_samples(cfg["mics"], cfg["grid"], cfg["fs"], cfg["c"])
    Np = o.max_lags(cfg["mics"], cfg["fs"], cfg["c"], 2)
    fac = o.slri_factors(x, Np, R)
    P, J = x.shape
    nmax = 2 * Np.max() + 1
    U = p.export("slri_u").reshape(P, J, R)
    V = p.export("slri_v").reshape(P, nmax, R)
    S = p.export("slri_s").reshape(P, nmax)
    for q in range(P):
        n = 2 * Np[q] + 1
        Uo, Vo, so = fac[q]
        np.testing.assert_allclose(S[q, :n], so, rtol=1e-9, atol=1e-12 * so[0])
        prod = U[q] @ V[q, :n].T
        ref = Uo @ Vo.T
        assert np.linalg.norm(prod - ref) <= 1e-9 * np.linalg.norm(ref)


@pytest.mark.parametrize("R", [8, 40, 154])
def test_host_plan_global_slri_matches_oracle_svd(R):
    """Global fit of (54): singular values and the rank-R product U V^T of
    the stacked Lambda against numpy's SVD (factors are unique only up to
    signs and rotations within equal singular values, so products are
    compared); R = PN reproduces Lambda itself."""
    _lib_or_skip()
    p, cfg = _host_plan("slri", R, stride=2, global_fit=True)
    x = o.tdoa_samples(cfg["mics"], cfg["grid"], cfg["fs"], cfg["c"])
    Np = o.max_lags(cfg["mics"], cfg["fs"], cfg["c"], 2)
    PN, J = int(sum(2 * Np + 1)), x.shape[1]
    assert p.info()["rank_or_q"] == min(R, PN)
    tall, fat = o.slri_global_factors(x, Np, R)
    U = p.export("slri_u").reshape(J, -1)
    V = p.export("slri_v").reshape(PN, -1)
    sv = p.export("slri_s")
    lam = np.concatenate([o.interp_matrix(x[q], n) for q, n in enumerate(Np)], axis=1)
    s_ref = np.linalg.svd(lam, compute_uv=False)
    k = min(R, len(s_ref))
    np.testing.assert_allclose(sv[:k], s_ref[:k], rtol=1e-9, atol=1e-9 * s_ref[0])
    np.testing.assert_allclose(U @ V.T, tall @ fat, rtol=0, atol=1e-9 * s_ref[0])
    if R >= PN:
        np.testing.assert_allclose(U @ V.T, lam, rtol=0, atol=1e-9)
    p.close()


@pytest.mark.parametrize("name,stride", [("square4_plane1k", 2), ("uca8_room125k", 3)])
@pytest.mark.parametrize("qbar", [1, 2, 4])
def test_host_plan_global_sspi_matches_oracle_selection(qbar, name, stride):
    """Global selection of (55): the kept entries of the stacked Lambda are
    the oracle's Q_Lambda = qbar J P largest magnitudes, with their values,
    exactly Q_Lambda of them (the room grid has exact magnitude ties at the
    threshold for qbar = 2 and 4, settled in the stacked matrix's order)."""
    _lib_or_skip()
    p, cfg = _host_plan("sspi", qbar, name=name, stride=stride, global_fit=True)
    x = o.tdoa_samples(cfg["mics"], cfg["grid"], cfg["fs"], cfg["c"])
    Np = o.max_lags(cfg["mics"], cfg["fs"], cfg["c"], 2)
    J, P = x.shape[1], len(Np)
    ref = o.sspi_global_select(x, Np, qbar * J * P)
    Q = p.info()["rank_or_q"]
    start = p.export("sspi_start").reshape(J, P)
    w = p.export("sspi_w").reshape(J, P, Q)
    off = np.concatenate([[0], np.cumsum(2 * Np + 1)])
    dense = np.zeros_like(ref)
    for q in range(P):
        for t in range(Q):
            nz = w[:, q, t] != 0
            cols = off[q] + start[nz, q] + t + Np[q]
            dense[np.nonzero(nz)[0], cols] = w[nz, q, t]
    assert np.count_nonzero(dense) == np.count_nonzero(ref) == qbar * J * P
    np.testing.assert_array_equal(dense != 0, ref != 0)
    np.testing.assert_allclose(dense, ref, rtol=0, atol=1e-14)
    assert 1 <= Q <= 16
    p.close()


def test_global_fit_is_refused_for_other_forms():
    _lib_or_skip()
    cfg = scenes.workload("square4_plane1k", grid_stride=4)
    for variant in ("fd", "si", "td"):
        with pytest.raises(native.SrpError):
            native.Plan(cfg["mics"], cfg["grid"], cfg["fs"], cfg["N"], variant, 4, device=-1, global_fit=True)


def test_host_plan_slri_large_lag_counts_match_oracle_svd():
    """Pairs with up to 499 lags take the tridiagonal + QL eigensolver: the
    first eight microphones of the 2 m disc array at 48 kHz on a 200-point
    subgrid (rank-deficient Lambda_p, J < 2 N_p + 1)."""
    _lib_or_skip()
    R = 8
    cfg = scenes.workload("disc32_box200k", grid_stride=10)
    mics = cfg["mics"][:8]
    p = native.Plan(mics, cfg["grid"], cfg["fs"], cfg["N"], "slri", R, device=-1)
    x = o.tdoa_samples(mics, cfg["grid"], cfg["fs"], cfg["c"])
    Np = o.max_lags(mics, cfg["fs"], cfg["c"], 2)
    assert (2 * Np + 1).max() > 200
    fac = o.slri_factors(x, Np, R)
    P, J = x.shape
    nmax = 2 * Np.max() + 1
    U = p.export("slri_u").reshape(P, J, R)
    V = p.export("slri_v").reshape(P, nmax, R)
    S = p.export("slri_s").reshape(P, nmax)
    for q in range(P):
        n = 2 * Np[q] + 1
        Uo, Vo, so = fac[q]
        np.testing.assert_allclose(S[q, :R], so[:R], rtol=1e-9)
        # the remaining singular values come from the squared spectrum of
        # the Gram matrix: absolute accuracy ~ sqrt(eps) sigma_1
        k = min(n, J)
        np.testing.assert_allclose(S[q, :k], so[:k], atol=1e-6 * so[0])
        prod = U[q] @ V[q, :n].T
        ref = Uo @ Vo.T
        assert np.linalg.norm(prod - ref) <= 1e-9 * np.linalg.norm(ref)


def test_host_plan_slri_rank_deficient_grams_all_converge():
    """All 496 pairs of the 32-microphone disc array on a 200-candidate
    subgrid: Gram matrices of rank 200 with up to 499 lags, hundreds of
    (near-)zero eigenvalues.  Pairs whose QL iteration once failed to
    deflate are checked against numpy's SVD."""
    _lib_or_skip()
    R = 8
    cfg = scenes.workload("disc32_box200k", grid_stride=10)
    p = native.Plan(cfg["mics"], cfg["grid"], cfg["fs"], cfg["N"], "slri", R, device=-1)
    x = o.tdoa_samples(cfg["mics"], cfg["grid"], cfg["fs"], cfg["c"])
    Np = o.max_lags(cfg["mics"], cfg["fs"], cfg["c"], 2)
    P, J = x.shape
    nmax = 2 * Np.max() + 1
    U = p.export("slri_u").reshape(P, J, R)
    V = p.export("slri_v").reshape(P, nmax, R)
    for q in (0, 381, 434, 456, 459, P - 1):
        n = 2 * Np[q] + 1
        lam = o.interp_matrix(x[q], Np[q])
        Uo, so, Vt = np.linalg.svd(lam, full_matrices=False)
        ref = (Uo[:, :R] * so[:R]) @ Vt[:R]
        prod = U[q] @ V[q, :n].T
        assert np.linalg.norm(prod - ref) <= 1e-9 * np.linalg.norm(ref), q


def test_host_plan_sspi_windows_match_oracle_selection():
    _lib_or_skip()
    Q = 4
    p, cfg = _host_plan("sspi", Q, name="uca8_room125k", stride=5)
    x = o.tdoa_samples(cfg["mics"], cfg["grid"], cfg["fs"], cfg["c"])
    Np = o.max_lags(cfg["mics"], cfg["fs"], cfg["c"], 2)
    P, J = x.shape
    st = p.export("sspi_start").reshape(J, P)
    w = p.export("sspi_w").reshape(J, P, Q)
    for q in range(P):
        lags, wts = o.sspi_select(x[q], Np[q], Q)
        np.testing.assert_array_equal(st[:, q], lags[:, 0])
        np.testing.assert_allclose(w[:, q, :], wts, rtol=0, atol=1e-14)


def test_host_plans_of_si_and_td():
    """TD keeps one unit-weight tap at the TDOA rounded half away from zero;
    SI keeps every lag (U_p = Lambda_p)."""
    _lib_or_skip()
    cfg = scenes.workload("uca8_room125k", grid_stride=7)
    x = o.tdoa_samples(cfg["mics"], cfg["grid"], cfg["fs"], cfg["c"])
    Np = o.max_lags(cfg["mics"], cfg["fs"], cfg["c"], 2)
    P, J = x.shape
    td = native.Plan(cfg["mics"], cfg["grid"], cfg["fs"], cfg["N"], "td", device=-1)
    st = td.export("sspi_start").reshape(J, P)
    np.testing.assert_array_equal(st.T, np.sign(x) * np.floor(np.abs(x) + 0.5))
    np.testing.assert_array_equal(td.export("sspi_w"), 1.0)
    si = native.Plan(cfg["mics"], cfg["grid"], cfg["fs"], cfg["N"], "si", device=-1)
    R = si.info()["rank_or_q"]
    assert R == 2 * Np.max() + 1
    U = si.export("slri_u").reshape(P, J, R)
    for q in range(P):
        lam = o.interp_matrix(x[q], Np[q])
        np.testing.assert_allclose(U[q][:, :lam.shape[1]], lam, rtol=0, atol=1e-12)


def test_mac_counts_follow_complexity_model():
    _lib_or_skip()
    cfg = scenes.workload("uca8_room125k", grid_stride=5)
    J = cfg["grid"].shape[0]
    fd = native.Plan(cfg["mics"], cfg["grid"], cfg["fs"], cfg["N"], "fd", device=-1)
    assert fd.info()["macs_per_map"] == 2 * J * 28 * 511
    sl = native.Plan(cfg["mics"], cfg["grid"], cfg["fs"], cfg["N"], "slri", 8, device=-1)
    c = o.complexity(J=J, P=28, K=512, N=660 / 28, R_lambda=28 * 8, sampling="direct")
    # per-pair rank R is a block-diagonal fat factor: R PN_p per pair
    assert sl.info()["macs_per_map"] == pytest.approx(J * 28 * 8 + 8 * 660 + 2 * 660 * 511)
    assert c["C_samp"] == 2 * 660 * 511
    sp = native.Plan(cfg["mics"], cfg["grid"], cfg["fs"], cfg["N"], "sspi", 4, device=-1)
    assert sp.info()["macs_per_map"] == pytest.approx(J * 28 * 4 + 2 * 660 * 511)


@pytest.mark.parametrize("kw,code", [
    (dict(N=511), -1),                          # odd N
    (dict(N=16), -1),                           # 2 N_p + 1 = 31 > N (lags alias)
    (dict(fs=-1.0), -1),
    (dict(variant="slri", rq=0), -1),
    (dict(variant="slri", rq=33), -3),
    (dict(variant="sspi", rq=17), -3),
    (dict(variant="slri", rq=4, dtype="f64"), -3),
    (dict(M=1), -1),
    (dict(variant="lr", rq=8), -3),             # LR-SRP fits on the device only
])
def test_invalid_arguments_return_error_codes(kw, code):
    _lib_or_skip()
    cfg = scenes.workload("square4_plane1k", grid_stride=8)
    mics = cfg["mics"][: kw.get("M", 4)]
    with pytest.raises(native.SrpError) as ei:
        native.Plan(mics, cfg["grid"], kw.get("fs", cfg["fs"]), kw.get("N", cfg["N"]),
                    kw.get("variant", "fd"), kw.get("rq", 0), dtype=kw.get("dtype", "f32"),
                    device=-1)
    assert ei.value.code == code
    assert native.lib().srp_last_error().decode() != ""


def test_non_finite_geometry_and_null_out():
    L = _lib_or_skip()
    cfg = scenes.workload("square4_plane1k", grid_stride=8)
    grid = cfg["grid"].copy()
    grid[3, 1] = np.nan
    with pytest.raises(native.SrpError) as ei:
        native.Plan(cfg["mics"], grid, cfg["fs"], cfg["N"], "fd", device=-1)
    assert ei.value.code == -1
    # NULL out pointer
    m = np.ascontiguousarray(cfg["mics"])
    g = np.ascontiguousarray(cfg["grid"])
    dp = ctypes.POINTER(ctypes.c_double)
    rc = L.srp_plan(m.ctypes.data_as(dp), 4, g.ctypes.data_as(dp), g.shape[0], 16000.0, 512, 0, 0, None, None)
    assert rc == -1


def test_host_only_plan_refuses_compute_and_export_of_missing_data():
    L = _lib_or_skip()
    p, _ = _host_plan("fd", 0)
    rc = L.srp_compute(p._h, ctypes.c_void_p(16), 4, ctypes.c_void_p(16), 0, None, 0, None)
    assert rc == -1
    assert L.srp_compute(p._h, None, 0, None, 0, None, 0, None) == 0   # L = 0 is a no-op
    # a row pitch below J is rejected before any device access
    rc = L.srp_compute(p._h, ctypes.c_void_p(16), 4, ctypes.c_void_p(16), p.J - 1, None, 0, None)
    assert rc == -1 and b"ld_maps" in L.srp_last_error()
    assert p.info()["map_pitch"] == (p.J + 127) // 128 * 128
    with pytest.raises(native.SrpError):
        p.export("slri_u")
    L.srp_destroy(None)   # safe on NULL


def test_host_plans_report_the_sspi_tile_split():
    """Host-only plans run no kernels: an SSPI plan reports every candidate
    tile on the gather and none on the matrix cores; other forms report
    neither."""
    _lib_or_skip()
    p, cfg = _host_plan("sspi", 4, name="uca8_room125k", stride=3, dtype="bf16")
    info = p.info()
    assert info["sspi_dense_tiles"] == 0
    assert info["sspi_gather_tiles"] == (len(cfg["grid"]) + 255) // 256
    assert info["sspi_band_tiles"] == 0
    q, _ = _host_plan("slri", 4)
    assert q.info()["sspi_dense_tiles"] == 0 and q.info()["sspi_gather_tiles"] == 0
    assert q.info()["sspi_band_tiles"] == 0

def test_td_endfire_candidates_stay_in_the_sampled_range():
    """With N_aux = 0, N_p = floor(d fs / c): a candidate on a pair's axis
    beyond the array has |x_p| = d fs / c, which rounds to N_p + 1 when its
    fraction is at least 1/2.  The TD plan's lag must stay at +-N_p (the
    end of the sampled range), as in the oracle."""
    _lib_or_skip()
    fs, c = 16000.0, 343.0
    d = 0.212                                   # d fs / c = 9.889: N_p = 9
    mics = np.array([[0.0, 0.0, 0.0], [d, 0.0, 0.0]])
    grid = np.array([[3.0, 0.0, 0.0], [-3.0, 0.0, 0.0], [0.05, 1.0, 0.0], [d + 1.0, 0.0, 0.0]])
    x = o.tdoa_samples(mics, grid, fs, c)
    Np = o.max_lags(mics, fs, c, 0)
    assert Np[0] == 9 and np.abs(x[0, [0, 1, 3]]).min() > 9.5
    p = native.Plan(mics, grid, fs, 64, "td", 0, n_aux=0, device=-1)
    start = p.export("sspi_start").astype(np.int64).reshape(len(grid), 1)[:, 0]
    n = np.clip(np.sign(x[0]) * np.floor(np.abs(x[0]) + 0.5), -9, 9)
    np.testing.assert_array_equal(start, n)
    assert start[0] == -9 and start[1] == 9 and start[3] == -9
    p.close()
