"""GPU parity on the large-aperture workload disc32_box200k: M = 32 (496
pairs, up to 2 N_p + 1 = 499 lags per pair, so the GCC samples come from the
iFFT form and the SLRI fits from the FP64 MFMA Gram matrices), fs 48 kHz,
N = 2048.

* a 200-candidate subgrid, every output against the FP64 oracle;
* the full 200,000-candidate grid with L = 256 frames (the launch
  configuration of the benchmark's large-aperture leg): SSPI at sampled
  candidates the oracle evaluates one by one, SLRI against stored oracle
  maps written by tests/golden/make_disc32_slri.py (oracle only);
* conv. FD-SRP with the steering generated inside the product (the only FD
  form at this size: a resident H would take 406 GB in BF16), a
  contraction over 2 P (K-1) = 1,014,816, on the subgrid (6 and 150
  frames: both generating kernels) and at sampled candidates of the full
  grid.

Every check bounds the relative L2 error and every element relative to the
map's largest oracle magnitude."""

import os

import numpy as np
import pytest

import oracle as o
from mapcheck import check_maps
from paper_2306_08514_amd import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "bf16": 1e-2, "f16": 1e-2}
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "disc32_slri_r8.npz")


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
def small():
    cfg = scenes.workload("disc32_box200k", L=6, grid_stride=10)
    return cfg, scenes.make_frames(cfg)


@pytest.mark.parametrize("variant,rq", [("slri", 8), ("sspi", 4)])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_subgrid_all_outputs(native, small, variant, rq, dtype):
    cfg, Y = small
    _announce(f"disc32 subgrid {variant} {rq} {dtype}")
    p = native.Plan(cfg["mics"], cfg["grid"], cfg["fs"], cfg["N"], variant, rq, dtype=dtype)
    info = p.info()
    assert info["P"] == 496 and info["sampling_fft"] == 1
    z = p.compute(torch.from_numpy(Y).cuda()).cpu().numpy()
    x = o.tdoa_samples(cfg["mics"], cfg["grid"], cfg["fs"], cfg["c"])
    Np = o.max_lags(cfg["mics"], cfg["fs"], cfg["c"], 2)
    xi = o.gcc_samples_ifft(o.phat(Y), Np, cfg["N"] // 2)
    if variant == "slri":
        ref = o.slri_map(xi, o.slri_factors(x, Np, rq))
    else:
        ref = o.sspi_map(xi, [o.sspi_select(x[q], Np[q], rq) for q in range(len(Np))], Np)
    check_maps(z, ref, TOL[dtype], f"disc32 subgrid {variant} {dtype}")


@pytest.fixture(scope="module")
def full():
    cfg = scenes.workload("disc32_box200k")
    Y = scenes.make_frames(cfg)
    return cfg, Y, torch.from_numpy(Y).cuda()


def test_full_size_sspi_sampled(native, full):
    cfg, Y, Yt = full
    _announce("disc32 full sspi bf16")
    p = native.Plan(cfg["mics"], cfg["grid"], cfg["fs"], cfg["N"], "sspi", 4, dtype="bf16")
    z = p.compute(Yt)
    rng = np.random.default_rng(21)
    frames = np.array([0, 100, 255])
    cols = np.sort(rng.choice(cfg["grid"].shape[0], 2000, replace=False))
    zs = z[torch.from_numpy(frames).cuda()][:, torch.from_numpy(cols).cuda()].cpu().numpy()
    x = o.tdoa_samples(cfg["mics"], cfg["grid"][cols], cfg["fs"], cfg["c"])
    Np = o.max_lags(cfg["mics"], cfg["fs"], cfg["c"], 2)
    xi = o.gcc_samples_ifft(o.phat(Y[frames]), Np, cfg["N"] // 2)
    ref = o.sspi_map(xi, [o.sspi_select(x[q], Np[q], 4) for q in range(len(Np))], Np)
    # the argmax over the sampled candidates agrees up to the error band
    check_maps(zs, ref, TOL["bf16"], "disc32 full sspi bf16 sampled")


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="stored oracle maps not generated")
def test_full_size_slri_against_stored_oracle_maps(native, full):
    cfg, Y, Yt = full
    _announce("disc32 full slri bf16")
    g = np.load(GOLDEN)
    p = native.Plan(cfg["mics"], cfg["grid"], cfg["fs"], cfg["N"], "slri", int(g["R"]), dtype="bf16")
    z = p.compute(Yt)
    frames, cols = g["frames"], g["cols"]
    zs = z[torch.from_numpy(frames).cuda()][:, torch.from_numpy(cols).cuda()].cpu().numpy()
    check_maps(zs, g["z"], TOL["bf16"], "disc32 full slri bf16 sampled")


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_fd_generated_subgrid_all_outputs(native, small, dtype):
    """Generated steering at P = 496, K - 1 = 1023: per 64-bin slice the
    rotation is seeded in FP64 and advanced in FP32, so the chain's error is
    checked at the longest contraction any workload runs."""
    cfg, Y = small
    _announce(f"disc32 subgrid fd generated {dtype}")
    p = native.Plan(cfg["mics"], cfg["grid"], cfg["fs"], cfg["N"], "fd", 0, dtype=dtype,
                    fd_steering="generated")
    assert p.info()["fd_generated"] == 1
    z = p.compute(torch.from_numpy(Y).cuda()).cpu().numpy()
    x = o.tdoa_samples(cfg["mics"], cfg["grid"], cfg["fs"], cfg["c"])
    ref = o.fd_map(o.phat(Y), x, cfg["N"] // 2)
    check_maps(z, ref, TOL[dtype], f"disc32 subgrid fd generated {dtype}")
    p.close()


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_fd_generated_subgrid_large_batch(native, dtype):
    """More than 128 frames per call run the 16-bit kernel that generates the
    steering between its matrix instructions; on one candidate tile the
    contraction is also split at pair boundaries.  Every output of 150 frames
    (one ragged frame tile) against the oracle, and bitwise against the same
    frames in batches that run the small-batch kernel."""
    cfg = scenes.workload("disc32_box200k", L=150, grid_stride=10)
    Y = scenes.make_frames(cfg)
    _announce(f"disc32 subgrid fd generated L=150 {dtype}")
    p = native.Plan(cfg["mics"], cfg["grid"], cfg["fs"], cfg["N"], "fd", 0, dtype=dtype,
                    fd_steering="generated")
    z = p.compute(torch.from_numpy(Y).cuda()).cpu().numpy()
    # batches of at most 128 frames run the other generating kernel: the
    # same steering values and products, so the same maps bit for bit
    for a, b in ((0, 64), (100, 150)):
        part = p.compute(torch.from_numpy(np.ascontiguousarray(Y[a:b])).cuda()).cpu().numpy()
        np.testing.assert_array_equal(part, z[a:b])
    p.close()
    x = o.tdoa_samples(cfg["mics"], cfg["grid"], cfg["fs"], cfg["c"])
    ref = o.fd_map(o.phat(Y), x, cfg["N"] // 2)
    check_maps(z, ref, TOL[dtype], f"disc32 subgrid fd generated L=150 {dtype}")


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_fd_generated_full_size_sampled(native, full, dtype):
    """The full grid in the launch configuration of the serving mix's M = 32
    FD requests and the large-aperture leg (L = 256), against the oracle at
    500 sampled candidates of three frames."""
    cfg, Y, Yt = full
    _announce(f"disc32 full fd generated {dtype}")
    p = native.Plan(cfg["mics"], cfg["grid"], cfg["fs"], cfg["N"], "fd", 0, dtype=dtype)
    assert p.info()["fd_generated"] == 1
    z = p.compute(Yt)
    rng = np.random.default_rng(23)
    frames = np.array([3, 128, 254])
    cols = np.sort(rng.choice(cfg["grid"].shape[0], 500, replace=False))
    zs = z[torch.from_numpy(frames).cuda()][:, torch.from_numpy(cols).cuda()].cpu().numpy()
    del z
    p.close()
    x = o.tdoa_samples(cfg["mics"], cfg["grid"][cols], cfg["fs"], cfg["c"])
    ref = o.fd_map(o.phat(Y[frames]), x, cfg["N"] // 2)
    check_maps(zs, ref, TOL[dtype], f"disc32 full fd generated {dtype} sampled")
