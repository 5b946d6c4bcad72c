"""Precision sweep on the square4_plane1k frames (M = 4, J = 1024, 100
frames): conv. FD-SRP, SLRI (R = 8 per pair) and SSPI (Q = 4) with FP32,
BF16, FP16 and FP8 (E4M3) operands and FP32 accumulation, phases and fits in
FP64.  Each map is compared with (i) the FP64 oracle of the same variant
(the parity target: relative error <= 1e-5 in FP32, <= 1e-2 in BF16 and
FP16; FP8 is reported against 6e-2) and (ii) the FP64 oracle of conv.
FD-SRP; argmax agreement is counted against both, up to the error band of
the reference map."""

import numpy as np
import pytest

import oracle as o
from paper_2306_08514_amd import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "bf16": 1e-2, "f16": 1e-2, "fp8": 6e-2}


def _argmax_agree(z, ref):
    """fraction of frames whose pick lies within the reference's error band
    of the reference maximum"""
    band = 2 * np.abs(z - ref).max(axis=1)
    pick = z.argmax(axis=1)
    return float(np.mean(ref[np.arange(len(ref)), pick] >= ref.max(axis=1) - band))


def test_precision_sweep():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_08514_amd import native
    native.lib()
    cfg = scenes.workload("square4_plane1k")
    Y = scenes.make_frames(cfg)
    Yt = torch.from_numpy(Y).cuda()
    K = cfg["N"] // 2
    x = o.tdoa_samples(cfg["mics"], cfg["grid"], cfg["fs"], cfg["c"])
    Np = o.max_lags(cfg["mics"], cfg["fs"], cfg["c"], 2)
    psi = o.phat(Y)
    xi = o.gcc_samples_ifft(psi, Np, K)
    ref = {"fd": o.fd_map(psi, x, K),
           "slri": o.slri_map(xi, o.slri_factors(x, Np, 8)),
           "sspi": o.sspi_map(xi, [o.sspi_select(x[q], Np[q], 4) for q in range(len(Np))], Np)}
    rows = []
    for variant, rq in (("fd", 0), ("slri", 8), ("sspi", 4)):
        for dtype in ("f32", "bf16", "f16", "fp8"):
            print(f"[gpu-case] precision {variant} {dtype}", flush=True)
            p = native.Plan(cfg["mics"], cfg["grid"], cfg["fs"], cfg["N"], variant, rq, dtype=dtype)
            z = p.compute(Yt).cpu().numpy().astype(np.float64)
            own = ref[variant]
            e_own = np.linalg.norm(z - own, axis=1) / np.linalg.norm(own, axis=1)
            e_fd = np.linalg.norm(z - ref["fd"], axis=1) / np.linalg.norm(ref["fd"], axis=1)
            rows.append((variant, dtype, float(np.median(e_own)), float(e_own.max()), _argmax_agree(z, own),
                         float(np.median(e_fd)), _argmax_agree(z, ref["fd"])))
            assert e_own.max() <= TOL[dtype], (variant, dtype, e_own.max())
    print("\n| form | operands | median rel vs own FP64 | max rel vs own | argmax vs own | median rel vs FP64 FD "
          "| argmax vs FD |")
    print("|---|---|---|---|---|---|---|")
    for r in rows:
        print(f"| {r[0]} | {r[1]} | {r[2]:.2e} | {r[3]:.2e} | {r[4] * 100:.0f} % | {r[5]:.2e} | {r[6] * 100:.0f} % |")
