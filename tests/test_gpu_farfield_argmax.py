"""GPU parity of far-field plans (grid rows are unit directions, Sec. II-A)
and of the device peak picking of (10)-(11), through the C ABI, against the
FP64 oracle and numpy."""

import numpy as np
import pytest

import oracle as o
from paper_2306_08514_amd import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "bf16": 1e-2}


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
def plane_wave():
    """UCA-8 (0.3 m) at the origin, a 1/f plane wave from 300 m along a grid
    direction of the 2-degree lower half sphere, white noise at 20 dB; 29
    frames of N = 1024 at 16 kHz."""
    mics = scenes.uca(8, 0.3)
    u = scenes.half_sphere_directions(2.0)
    j0 = 10 * 180 + 20            # depression 20 deg, azimuth 40 deg
    rng = np.random.default_rng(scenes.SEED_BASE + 50)
    N, hop, L = 1024, 512, 29
    x = scenes.render(rng, mics, [300.0 * u[j0]], 16000.0, (L - 1) * hop + N, 20.0)
    Y = scenes.stft_frames(x, N, hop, L).astype(np.complex64)
    return dict(mics=mics, grid=u, fs=16000.0, N=N, c=343.0, j0=j0), Y


def _oracle_ff(variant, Y, cfg, rq):
    x = o.tdoa_samples_far_field(cfg["mics"], cfg["grid"], cfg["fs"], cfg["c"])
    Np = o.max_lags(cfg["mics"], cfg["fs"], cfg["c"], 2)
    K = cfg["N"] // 2
    psi = o.phat(Y)
    if variant == "fd":
        return o.fd_map(psi, x, K)
    xi = o.gcc_samples_ifft(psi, Np, K)
    if variant == "slri":
        return o.slri_map(xi, o.slri_factors(x, Np, rq))
    sel = [o.sspi_select(x[p], Np[p], rq) for p in range(len(Np))]
    return o.sspi_map(xi, sel, Np)


@pytest.mark.parametrize("variant,rq,dtype", [("fd", 0, "f32"), ("slri", 8, "f32"), ("sspi", 4, "f32"),
                                              ("fd", 0, "bf16"), ("slri", 8, "bf16")])
def test_far_field_maps(native, plane_wave, variant, rq, dtype):
    cfg, Y = plane_wave
    _announce(f"far-field {variant} {dtype} J={len(cfg['grid'])}")
    p = native.Plan(cfg["mics"], cfg["grid"], cfg["fs"], cfg["N"], variant, rq, dtype=dtype, far_field=True)
    maps = p.compute(torch.from_numpy(Y).cuda())
    idx, val = native.argmax(maps)
    z = maps.cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    ref = _oracle_ff(variant, Y, cfg, rq)
    rel = o.rel_error(z, ref)
    assert rel.max() <= TOL[dtype], f"max rel error {rel.max():.3e}"
    # device peak = numpy's argmax of the same maps, bit for bit
    np.testing.assert_array_equal(idx.cpu().numpy(), o.argmax_map(z))
    np.testing.assert_array_equal(val.cpu().numpy(), z[np.arange(len(z)), o.argmax_map(z)])
    # the plane wave is localised: FD's median pick is the source direction
    # up to one grid step; the reduced forms (R = 8, Q = 4 on a 0.3 m UCA)
    # carry their approximation error into the pick, within 10 deg
    u = cfg["grid"]
    ang = np.degrees(np.arccos(np.clip(u[idx.cpu().numpy()] @ u[cfg["j0"]], -1, 1)))
    assert np.median(ang) <= (2.5 if variant == "fd" else 10.0), ang
    p.close()


def _np_peak(z):
    """argmax ignoring NaN, ties to the smallest index, -1 for all-NaN rows."""
    out = np.full(len(z), -1, dtype=np.int64)
    for i, r in enumerate(z):
        ok = ~np.isnan(r)
        if ok.any():
            m = r[ok].max()
            out[i] = int(np.nonzero(ok & (r == m))[0][0])
    return out


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_argmax_ties_nan_pitch(native, dt):
    rng = np.random.default_rng(scenes.SEED_BASE + 51)
    L, J, pitch = 67, 5003, 5120
    z = rng.standard_normal((L, J)).astype(dt)
    z[3, [17, 4000, 4999]] = 9.0                  # three-way tie
    z[5, :] = 1.25                                # all equal
    z[7, ::2] = np.nan                            # NaN never wins
    z[8, :] = np.nan                              # all NaN
    z[9, J - 1] = 50.0                            # peak in the ragged tail
    z[10, :] = -np.inf
    z[10, 2500] = -1e30
    buf = torch.full((L, pitch), 1e9, dtype=torch.float64 if dt == np.float64 else torch.float32,
                     device="cuda")               # padding beyond J must be ignored
    buf[:, :J] = torch.from_numpy(z).cuda()
    _announce(f"argmax {dt.__name__} L={L} J={J} pitch={pitch}")
    idx, val = native.argmax(buf[:, :J])
    idx = idx.cpu().numpy()
    val = val.cpu().numpy()
    ref = _np_peak(z)
    np.testing.assert_array_equal(idx, ref)
    ok = ref >= 0
    np.testing.assert_array_equal(val[ok], z[ok, ref[ok]].astype(np.float64))
    assert idx[3] == 17 and idx[5] == 0 and idx[8] == -1 and idx[9] == J - 1 and idx[10] == 2500
    # single row, single column, and an empty batch
    one = torch.tensor([[3.0, 7.0, 7.0]], device="cuda")
    assert native.argmax(one)[0].item() == 1
    col = torch.tensor([[2.0], [-1.0]], device="cuda")
    assert native.argmax(col)[0].tolist() == [0, 0]
    e_idx, e_val = native.argmax(torch.empty((0, 10), device="cuda"))
    assert e_idx.numel() == 0 and e_val.numel() == 0
