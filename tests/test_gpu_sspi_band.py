"""GPU parity of the SSPI band product (eq. (58) on the matrix cores for
apertures whose per-tile lag windows do not fit the dense-window
contraction), on the large-aperture geometry of disc32_box200k (496 pairs,
up to 499 lags per pair, fs 48 kHz, N = 2048):

* a 3125-candidate subgrid (13 tiles, the last one ragged) with 70 frames
  (two 64-frame blocks, the second ragged): every output against the FP64
  oracle for Q = 1, 3, 4 and 8, BF16 and FP16 weights, and TD;
* a 200-candidate subgrid with 6 frames (one tile with a dead subtile), and
  global SSPI there;
* bitwise batch invariance: a frame's map alone, at any offset, equals the
  same frame's map inside a batch.

Every check bounds the relative L2 error and every element relative to the
map's largest oracle magnitude."""

import numpy as np
import pytest

import oracle as o
from mapcheck import check_maps
from paper_2306_08514_amd import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"bf16": 1e-2, "f16": 1e-2}
_REFS = {}  # oracle maps of the stride-4 subgrid per Q, shared by both dtypes


@pytest.fixture(scope="module")
def native():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_08514_amd import native as nat
    nat.lib()
    return nat


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def sub4():
    cfg = scenes.workload("disc32_box200k", L=70, grid_stride=4)
    Y = scenes.make_frames(cfg)
    Np = o.max_lags(cfg["mics"], cfg["fs"], cfg["c"], 2)
    xi = o.gcc_samples_ifft(o.phat(Y), Np, cfg["N"] // 2)
    x = o.tdoa_samples(cfg["mics"], cfg["grid"], cfg["fs"], cfg["c"])
    return cfg, Y, xi, x, Np


def _plan(native, cfg, variant, rq, dtype, **kw):
    return native.Plan(cfg["mics"], cfg["grid"], cfg["fs"], cfg["N"], variant, rq, dtype=dtype, c=cfg["c"], **kw)


def _tiles(cfg):
    return (cfg["grid"].shape[0] + 255) // 256


@pytest.mark.parametrize("q", [1, 3, 4, 8])
@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_band_subgrid_all_outputs(native, sub4, q, dtype):
    cfg, Y, xi, x, Np = sub4
    _announce(f"disc32 stride-4 subgrid sspi band Q={q} {dtype} L={len(Y)}")
    p = _plan(native, cfg, "sspi", q, dtype)
    info = p.info()
    assert info["sspi_band_tiles"] == _tiles(cfg) and info["sspi_gather_tiles"] == 0, info
    assert info["sspi_dense_tiles"] == 0
    z = p.compute(torch.from_numpy(Y).cuda()).cpu().numpy()
    if q not in _REFS:
        _REFS[q] = o.sspi_map(xi, [o.sspi_select(x[k], Np[k], q) for k in range(len(Np))], Np)
    check_maps(z, _REFS[q], TOL[dtype], f"disc32 band sspi Q={q} {dtype}")


def test_band_td(native, sub4):
    cfg, Y, xi, x, Np = sub4
    _announce("disc32 stride-4 subgrid td band bf16")
    t = _plan(native, cfg, "td", 0, "bf16")
    assert t.info()["sspi_band_tiles"] == _tiles(cfg)
    z = t.compute(torch.from_numpy(Y).cuda()).cpu().numpy()
    check_maps(z, o.td_map(xi, x, Np), TOL["bf16"], "disc32 band td bf16")


@pytest.fixture(scope="module")
def sub10():
    cfg = scenes.workload("disc32_box200k", L=6, grid_stride=10)
    Y = scenes.make_frames(cfg)
    Np = o.max_lags(cfg["mics"], cfg["fs"], cfg["c"], 2)
    xi = o.gcc_samples_ifft(o.phat(Y), Np, cfg["N"] // 2)
    x = o.tdoa_samples(cfg["mics"], cfg["grid"], cfg["fs"], cfg["c"])
    return cfg, Y, xi, x, Np


def test_band_global_sspi(native, sub10):
    cfg, Y, xi, x, Np = sub10
    _announce(f"disc32 stride-10 subgrid global sspi qbar=2 bf16 J={cfg['grid'].shape[0]}")
    g = _plan(native, cfg, "sspi", 2, "bf16", global_fit=True)
    info = g.info()
    ref = o.sspi_global_map(xi, o.sspi_global_select(x, Np, 2 * x.shape[1] * len(Np)))
    z = g.compute(torch.from_numpy(Y).cuda()).cpu().numpy()
    # windows of more than eight taps stay on the gather
    assert info["sspi_band_tiles"] + info["sspi_gather_tiles"] == _tiles(cfg), info
    check_maps(z, ref, TOL["bf16"], f"disc32 global sspi bf16 (band tiles {info['sspi_band_tiles']})")


def test_band_dead_subtile_and_few_frames(native, sub10):
    cfg, Y, xi, x, Np = sub10
    _announce(f"disc32 stride-10 subgrid sspi band J={cfg['grid'].shape[0]} L=6")
    p = _plan(native, cfg, "sspi", 4, "bf16")
    assert p.info()["sspi_band_tiles"] == 1
    z = p.compute(torch.from_numpy(Y).cuda()).cpu().numpy()
    ref = o.sspi_map(xi, [o.sspi_select(x[k], Np[k], 4) for k in range(len(Np))], Np)
    check_maps(z, ref, TOL["bf16"], "disc32 band sspi few frames")


def test_band_maps_do_not_depend_on_the_batch(native, sub4):
    """Each frame goes through the same products whatever its block and
    row: alone, at any offset, its map is bitwise the batch's."""
    cfg, Y, _, _, _ = sub4
    _announce("disc32 band batch invariance bf16")
    p = _plan(native, cfg, "sspi", 4, "bf16")
    full = p.compute(torch.from_numpy(Y).cuda()).cpu().numpy()
    for a, b in ((0, 1), (5, 6), (33, 40), (63, 70), (64, 65)):
        part = p.compute(torch.from_numpy(np.ascontiguousarray(Y[a:b])).cuda()).cpu().numpy()
        np.testing.assert_array_equal(part, full[a:b])
