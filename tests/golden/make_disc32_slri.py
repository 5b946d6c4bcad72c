"""Writes tests/golden/disc32_slri_r8.npz: FP64 oracle SLRI maps (R = 8 per
pair) of the disc32_box200k workload (M = 32, J = 200,000, fs 48 kHz,
N = 2048) at 4 frames x 2000 sampled candidates.

The per-pair factors come from the oracle's Gram route (the right singular
vectors of each Lambda_p over all 200,000 candidates), the GCC samples from
the oracle's iFFT; nothing here calls the HIP library.  Run from the
repository root:

    python tests/golden/make_disc32_slri.py

(about 10 minutes on 8 cores; the frames are regenerated from their seed).
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as o  # noqa: E402
from paper_2306_08514_amd import scenes  # noqa: E402

R = 8
FRAMES = np.array([0, 77, 150, 255])
NCOLS = 2000


def main():
    t0 = time.time()
    cfg = scenes.workload("disc32_box200k")
    Y = scenes.make_frames(cfg)
    x = o.tdoa_samples(cfg["mics"], cfg["grid"], cfg["fs"], cfg["c"])
    Np = o.max_lags(cfg["mics"], cfg["fs"], cfg["c"], 2)
    rng = np.random.default_rng(20)
    cols = np.sort(rng.choice(x.shape[1], NCOLS, replace=False))
    print(f"frames and geometry in {time.time() - t0:.0f} s", flush=True)
    fac = o.slri_factors_gram(x, Np, R, cols)
    print(f"factors in {time.time() - t0:.0f} s", flush=True)
    xi = o.gcc_samples_ifft(o.phat(Y[FRAMES]), Np, cfg["N"] // 2)
    z = o.slri_map(xi, fac)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "disc32_slri_r8.npz")
    np.savez_compressed(out, z=z, frames=FRAMES, cols=cols, R=R,
                        note="oracle SLRI R=8 per pair, disc32_box200k, Gram route")
    print(f"wrote {out} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
