"""Map comparison used by every GPU parity test.

A GPU map z and the FP64 oracle's map z_ref (same frames, same candidates)
pass at tolerance tol when, for every map (row):

* every value is finite;
* the relative L2 error ||z - z_ref|| / ||z_ref|| is at most tol;
* every element is within tol * max_j |z_ref[j]| of the oracle, so an error
  confined to one candidate tile cannot hide in the norm of a large map;
* the argmax agrees, or the GPU's pick lies within the error band of the
  oracle's maximum (near ties).
"""

import numpy as np

import oracle as o


def map_errors(z, z_ref):
    """Per-map relative L2 error and per-map element error relative to the
    map's largest oracle magnitude."""
    z = np.asarray(z, dtype=np.float64)
    z_ref = np.asarray(z_ref, dtype=np.float64)
    rel = o.rel_error(z, z_ref)
    elem = np.abs(z - z_ref).max(axis=-1) / np.abs(z_ref).max(axis=-1)
    return rel, elem


def check_maps(z, z_ref, tol, label, argmax=True):
    """Asserts the bounds above; returns (max L2 error, max element error)."""
    z = np.asarray(z, dtype=np.float64)
    z_ref = np.asarray(z_ref, dtype=np.float64)
    assert z.shape == z_ref.shape, (label, z.shape, z_ref.shape)
    assert np.all(np.isfinite(z)), f"{label}: non-finite map values"
    rel, elem = map_errors(z, z_ref)
    worst, worst_e = float(rel.max()), float(elem.max())
    print(f"[maps] {label}: L2 {worst:.2e}  elem {worst_e:.2e}  (tol {tol:.0e})", flush=True)
    assert worst <= tol, f"{label}: max rel L2 error {worst:.3e} > {tol:.1e} (median {np.median(rel):.3e})"
    bad = np.nonzero(elem > tol)[0]
    if len(bad):
        f = int(bad[0])
        j = int(np.abs(z[f] - z_ref[f]).argmax())
        raise AssertionError(f"{label}: element error {elem[f]:.3e} of the map's max |z_ref| > {tol:.1e} "
                             f"on map {f} at candidate {j} (gpu {z[f, j]:.6g}, oracle {z_ref[f, j]:.6g}); "
                             f"{len(bad)} maps over")
    if argmax:
        a_gpu = o.argmax_map(z)
        a_ref = o.argmax_map(z_ref)
        err = np.abs(z - z_ref).max(axis=1)
        top = z_ref.max(axis=1)
        picked = z_ref[np.arange(len(z_ref)), a_gpu]
        off = (a_gpu != a_ref) & (picked < top - 2 * err - 1e-12 * np.abs(top))
        assert not off.any(), f"{label}: argmax disagrees beyond the error band on maps {np.nonzero(off)[0][:10]}"
    return worst, worst_e
