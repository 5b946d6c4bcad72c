"""GPU parity of SSPI (55)/(58) with 16-bit weights where the lag windows of a
256-candidate tile are evaluated as a dense contraction on the matrix cores
and the remaining tiles by the gather, through the C ABI against the FP64
oracle.  The plan reports how many tiles each path took; the workloads here
are chosen so that both paths run inside one plan."""

import numpy as np
import pytest

import oracle as o
from mapcheck import check_maps
from paper_2306_08514_amd import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "bf16": 1e-2, "f16": 1e-2}


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
def room_slice():
    """A contiguous run of the full-resolution room-125k grid (J = 7700, not a
    tile multiple) that passes under the ceiling array, 19 frames: most
    tiles have narrow lag windows, the tiles closest to the array do not."""
    cfg = scenes.workload("uca8_room125k", L=19)
    cfg["grid"] = cfg["grid"][58880:58880 + 7700]
    Y = scenes.make_frames(cfg)
    return cfg, Y


@pytest.fixture(scope="module")
def sq4():
    cfg = scenes.workload("square4_plane1k", L=41)
    return cfg, scenes.make_frames(cfg)


def _ref(cfg, Y, Q, form="sspi", global_fit=False):
    x = o.tdoa_samples(cfg["mics"], cfg["grid"], cfg["fs"], cfg["c"])
    Np = o.max_lags(cfg["mics"], cfg["fs"], cfg["c"], 2)
    xi = o.gcc_samples_ifft(o.phat(Y), Np, cfg["N"] // 2)
    if form == "td":
        return o.td_map(xi, x, Np)
    if global_fit:
        return o.sspi_global_map(xi, o.sspi_global_select(x, Np, Q * x.shape[1] * len(Np)))
    return o.sspi_map(xi, [o.sspi_select(x[p], Np[p], Q) for p in range(len(Np))], Np)


def _plan(native, cfg, variant, rq, dtype, **kw):
    return native.Plan(cfg["mics"], cfg["grid"], cfg["fs"], cfg["N"], variant, rq, dtype=dtype, **kw)


def _tiles(cfg):
    return (len(cfg["grid"]) + 255) // 256


def _check(z, ref, tol, label):
    check_maps(z, ref, tol, label)


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
@pytest.mark.parametrize("Q", [1, 3, 4, 8])
def test_split_tiles_match_oracle(native, room_slice, dtype, Q):
    cfg, Y = room_slice
    _announce(f"sspi dense/gather split Q={Q} {dtype} J={len(cfg['grid'])}")
    p = _plan(native, cfg, "sspi", Q, dtype)
    info = p.info()
    assert info["sspi_dense_tiles"] + info["sspi_gather_tiles"] == _tiles(cfg)
    # the windows widen with Q: one tap fits every tile here; from three
    # taps on, the tiles right under the array stay on the gather
    assert info["sspi_dense_tiles"] > 0, info
    if Q >= 3:
        assert info["sspi_gather_tiles"] > 0, (info["sspi_dense_tiles"], info["sspi_gather_tiles"])
    z = p.compute(torch.from_numpy(Y).cuda()).cpu().numpy()
    _check(z, _ref(cfg, Y, Q), TOL[dtype], f"split Q={Q} {dtype}")
    p.close()


def test_all_dense_small_array_and_f32_gather(native, sq4):
    """A 0.2 m square: every tile fits; FP32 weights always take the gather."""
    cfg, Y = sq4
    _announce("sspi all-dense square4 bf16 / f32 gather")
    Yt = torch.from_numpy(Y).cuda()
    ref = _ref(cfg, Y, 4)
    p = _plan(native, cfg, "sspi", 4, "bf16")
    assert p.info()["sspi_dense_tiles"] == _tiles(cfg) and p.info()["sspi_gather_tiles"] == 0
    _check(p.compute(Yt).cpu().numpy(), ref, TOL["bf16"], "square4 dense bf16")
    q = _plan(native, cfg, "sspi", 4, "f32")
    assert q.info()["sspi_dense_tiles"] == 0 and q.info()["sspi_gather_tiles"] == _tiles(cfg)
    _check(q.compute(Yt).cpu().numpy(), ref, TOL["f32"], "square4 gather f32")


def test_global_and_td_on_split_tiles(native, room_slice):
    cfg, Y = room_slice
    Yt = torch.from_numpy(Y).cuda()
    _announce("global sspi qbar=4 bf16 on the room slice")
    p = _plan(native, cfg, "sspi", 4, "bf16", global_fit=True)
    info = p.info()
    assert info["sspi_dense_tiles"] + info["sspi_gather_tiles"] == _tiles(cfg)
    _check(p.compute(Yt).cpu().numpy(), _ref(cfg, Y, 4, global_fit=True), TOL["bf16"], "global sspi bf16")
    _announce("td bf16 on the room slice")
    t = _plan(native, cfg, "td", 0, "bf16")
    _check(t.compute(Yt).cpu().numpy(), _ref(cfg, Y, 1, form="td"), TOL["bf16"], "td bf16")


def test_split_maps_do_not_depend_on_the_batch(native, room_slice):
    """Each frame's map is the same bit for bit alone, at any batch offset
    and in any batch size (frame groups of 32 never mix frames)."""
    cfg, Y = room_slice
    _announce("sspi split batch invariance bf16")
    p = _plan(native, cfg, "sspi", 4, "bf16")
    full = p.compute(torch.from_numpy(Y).cuda()).cpu().numpy()
    for a, b in ((0, 1), (5, 6), (3, 19), (18, 19)):
        part = p.compute(torch.from_numpy(np.ascontiguousarray(Y[a:b])).cuda()).cpu().numpy()
        np.testing.assert_array_equal(part, full[a:b])


def test_split_tiles_across_streams_and_frame_chunks(native, room_slice):
    """Maps of a plan with both tile kinds match across frame chunks that
    reuse the workspace (frame tile 64 < 150 frames) and when two calls on
    one plan run on two streams with their own workspaces."""
    cfg, Y1 = room_slice
    Y = np.concatenate([Y1] * 8)[:150]
    _announce(f"sspi split frame chunks / two streams bf16 L={len(Y)}")
    ref = _ref(cfg, Y1, 4)
    p = _plan(native, cfg, "sspi", 4, "bf16", frame_tile=64)
    assert p.info()["sspi_gather_tiles"] > 0
    Yt = torch.from_numpy(Y).cuda()
    z = p.compute(Yt).cpu().numpy()
    for k in range(len(Y)):
        _check(z[k:k + 1], ref[k % len(Y1):k % len(Y1) + 1], TOL["bf16"], f"chunked frame {k}")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for s, part in ((s1, Yt[:100]), (s2, Yt[40:150])):
        with torch.cuda.stream(s):
            ws = torch.empty(p.workspace_size(part.shape[0]), dtype=torch.uint8, device="cuda")
            outs.append((p.compute(part, workspace=ws, stream=s), ws))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(outs[0][0].cpu().numpy(), z[:100])
    np.testing.assert_array_equal(outs[1][0].cpu().numpy(), z[40:150])


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_dense_path_small_shapes(native, sq4, dtype):
    """One pair and one candidate, one ragged tile (J = 300), a single frame
    and an empty batch on the dense-window path."""
    cfg, Y = sq4
    _announce(f"sspi dense small shapes {dtype}")
    cfg2 = dict(cfg)
    cfg2["mics"] = cfg["mics"][:2]
    cfg2["grid"] = cfg["grid"][5:6]
    Y2 = np.ascontiguousarray(Y[:5, :2])
    q = _plan(native, cfg2, "sspi", 2, dtype)
    assert q.info()["sspi_dense_tiles"] == 1
    z = q.compute(torch.from_numpy(Y2).cuda()).cpu().numpy().astype(np.float64)
    ref2 = _ref(cfg2, Y2, 2)
    # one value per map: the error against the largest of the five frames
    assert np.abs(z - ref2).max() <= TOL[dtype] * np.abs(ref2).max(), "M=2 J=1"
    cfg3 = dict(cfg)
    cfg3["grid"] = cfg["grid"][:300]
    p = _plan(native, cfg3, "sspi", 4, dtype)
    assert p.info()["sspi_dense_tiles"] == 2
    ref = _ref(cfg3, Y, 4)
    _check(p.compute(torch.from_numpy(Y).cuda()).cpu().numpy(), ref, TOL[dtype], "J=300")
    _check(p.compute(torch.from_numpy(Y[7:8]).cuda()).cpu().numpy(), ref[7:8], TOL[dtype], "L=1")
    empty = torch.empty((0,) + Y.shape[1:], dtype=torch.complex64, device="cuda")
    assert p.compute(empty).shape == (0, 300)
