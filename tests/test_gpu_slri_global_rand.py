"""GPU checks of the global SLRI fit (eq. (54)) by randomized subspace
iteration, the fit the device uses when the stacked Lambda is too wide for
the PN x PN Gram eigendecomposition (PN > 4096), against the oracle's exact
SVD of the same Lambda:

* the fitted V has orthonormal columns;
* Eckart-Young: the fit's error ||Lambda - Lambda V V^T||_F^2 is within 1 %
  of the optimum, the discarded singular energy sum_{i > R} sigma_i^2;
* the leading quarter of the R singular values matches the exact ones to
  1e-4 relative (two power iterations: the values converge more slowly than
  the subspace, 6e-6 on the room case);
* the maps equal the oracle's rank-R map built from the same V (every
  output, the map tolerances of the other parity tests).

Two cases: the 0.3 m UCA on a 4913-candidate room subgrid with the
randomized fit forced (PN = 660), and the 0.5 m UCA of the serving mix
(120 pairs, PN = 4232 > 4096) on its 1024-candidate grid, where the plan
switches to the randomized fit by itself."""

import numpy as np
import pytest

import oracle as o
from mapcheck import check_maps
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


def _case(name):
    if name == "room_forced":
        cfg = scenes.workload("uca8_room125k", L=12, grid_stride=3)
        return cfg["mics"], cfg["grid"], cfg["fs"], cfg["N"], cfg["c"], 140, "randomized", scenes.make_frames(cfg)
    mics, fs, N = scenes.serving_array(16)
    grid = scenes.serving_grid(1024)
    Y = scenes.serving_frames(16, L=12)
    return mics, grid, fs, N, 343.0, 256, True, Y


@pytest.mark.parametrize("name", ["room_forced", "uca16_pn4232"])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_randomized_global_fit(native, name, dtype):
    mics, grid, fs, N, c, R, gf, Y = _case(name)
    print(f"[gpu-case] randomized global slri {name} R={R} {dtype}", flush=True)
    p = native.Plan(mics, grid, fs, N, "slri", R, dtype=dtype, c=c, global_fit=gf)
    info = p.info()
    PN = info["PN"]
    if name == "uca16_pn4232":
        assert PN > 4096, PN
    V = p.export("slri_v").reshape(PN, R)
    s_dev = p.export("slri_s")
    x = o.tdoa_samples(mics, grid, fs, c)
    Np = o.max_lags(mics, fs, c, 2)
    lam = np.concatenate([o.interp_matrix(x[q], Np[q]) for q in range(len(Np))], axis=1)
    sig = np.linalg.svd(lam, compute_uv=False)
    # orthonormal columns
    np.testing.assert_allclose(V.T @ V, np.eye(R), atol=1e-9)
    # Eckart-Young
    err = np.linalg.norm(lam - (lam @ V) @ V.T) ** 2
    opt = float(np.sum(sig[R:] ** 2))
    print(f"[fit] {name}: error {err:.6e}, optimum {opt:.6e}, ratio {err / opt:.6f}", flush=True)
    assert err <= 1.01 * opt + 1e-12 * float(np.sum(sig ** 2))
    # leading singular values
    rel = np.abs(s_dev[: R // 4] - sig[: R // 4]) / sig[: R // 4]
    print(f"[fit] {name}: leading singular values max rel error {rel.max():.2e}", flush=True)
    assert rel.max() <= 1e-4
    # maps against the oracle's rank-R map with the same V
    xi = o.gcc_samples_direct(o.phat(Y), Np, N // 2)
    ref = o.slri_global_map(xi, lam @ V, V.T)
    z = p.compute(torch.from_numpy(Y).cuda()).cpu().numpy()
    check_maps(z, ref, TOL[dtype], f"randomized global slri {name} {dtype}")
    p.close()
