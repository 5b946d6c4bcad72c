"""Evaluation harness: map error and localisation accuracy against relative
complexity for every form the library computes (the measures of Sec. V-A),
on seeded synthetic scenes.

    python -m paper_2306_08514_amd.evaluate [--scene nf4|ff6|room|square|farfield]
        [--sources 16] [--frames 8] [--dtype f32] [--forms slri,sspi,...] [--out results.json]

For each form and setting (R or Q per pair, the global R_Lambda or Q_Lambda,
R_H of LR-SRP) a plan is built on the device and every frame mapped once.
Reported per setting:
  C_rel   the plan's run-time MAC count over conv. FD-SRP's 2 J P (K - 1);
  eps_z   10 log10 ||z_type - z||^2 / ||z||^2 per frame against conv. FD-SRP
          computed by the library in FP64 (median and 10th / 90th
          percentiles);
  eps_H   10 log10 ||H_type - H||_F^2 / ||H||_F^2 of (64), H the single-sided
          steering matrix (19).  For SI, TD, SLRI and SSPI, H_type = Lambda_type
          S with the sampling rows S_n[k] = exp(j pi k n / K), evaluated per
          (location, pair) from the plan's FP64 fit without forming H (see
          eps_h_db); for LR-SRP from the singular values: every entry of H
          has unit modulus, so ||H||_F^2 = J P (K - 1) and ||H - H_lr||_F^2 =
          ||H||_F^2 - sum_{r <= R_H} sigma_r^2;
  rho_s   the fraction of frames whose peak lies within eps_th of the true
          source (distance, near field) or direction (angle, far field),
          at 4, 8 and 16 cm or 3 degrees.
Peaks come from the device argmax.  Everything runs through the C ABI; the
harness itself only compares maps and positions.
"""

import argparse
import json
import sys
import time

import numpy as np

SWEEPS = {
    "fd": [dict(variant="fd")],
    "td": [dict(variant="td")],
    "si": [dict(variant="si")],
    "slri": [dict(variant="slri", rq=r) for r in (2, 4, 8, 16, 24, 31)],
    "slri_global": [dict(variant="slri", rq=r, global_fit=True) for r in (16, 32, 64, 128, 224, 448)],
    "sspi": [dict(variant="sspi", rq=q) for q in (1, 2, 4, 8)],
    "sspi_global": [dict(variant="sspi", rq=q, global_fit=True) for q in (1, 2, 4, 8)],
    "lr": [dict(variant="lr", rq=r) for r in (16, 64, 256, 1024)],
}
NF_THRESHOLDS = (0.04, 0.08, 0.16)   # metres
FF_THRESHOLDS = (3.0,)               # degrees


def localisation_error(grid, picks, truth, far_field):
    """eps_s of Sec. V-A: distance between the picked and the true position
    (near field) or the angle in degrees between directions (far field)."""
    q = grid[picks]
    if far_field:
        c = np.clip(np.sum(q * truth, axis=1), -1.0, 1.0)
        return np.degrees(np.arccos(c))
    return np.linalg.norm(q - truth, axis=1)


def accuracy(eps_s, thresholds):
    """rho_s of Sec. V-A averaged over frames, per threshold."""
    return {f"{t:g}": float(np.mean(eps_s <= t)) for t in thresholds}


def dirichlet_sum(t, K):
    """sum_{k=1}^{K-1} cos(pi k t / K) = sin((K - 1/2) pi t / K) /
    (2 sin(pi t / (2K))) - 1/2, and K - 1 at t = 0 (mod 2K)."""
    t = np.asarray(t, dtype=np.float64)
    th = np.pi * t / K
    sh = np.sin(th / 2.0)
    small = np.abs(sh) < 1e-12
    out = np.empty_like(t)
    out[~small] = np.sin((K - 0.5) * th[~small]) / (2.0 * sh[~small]) - 0.5
    out[small] = K - 1.0
    return out


def row_errors(lags, lam, x, K):
    """sum_{k=1}^{K-1} |sum_n lam_n exp(j pi k n / K) - exp(j pi k x / K)|^2 for
    rows of interpolation weights lam at integer lags (arrays [..., n], x
    [...]), in closed form: with G(d) = sum_k cos(pi k d / K) = K - 1 (d = 0),
    -1 (d even), 0 (d odd) for |d| < 2K, the weights' own energy is
    K sum lam^2 - (sum over even lags)^2 - (sum over odd lags)^2; the steering
    row has energy K - 1; the cross term is sum_n lam_n D(n - x)."""
    lags = np.asarray(lags)
    lam = np.asarray(lam, dtype=np.float64)
    even = (lags % 2) == 0
    e_sum = np.sum(np.where(even, lam, 0.0), axis=-1)
    o_sum = np.sum(np.where(even, 0.0, lam), axis=-1)
    own = K * np.sum(lam * lam, axis=-1) - e_sum ** 2 - o_sum ** 2
    cross = np.sum(lam * dirichlet_sum(lags - np.asarray(x)[..., None], K), axis=-1)
    return (K - 1.0) + own - 2.0 * cross


def eps_h_db(native, cfg, variant, rq, far_field=False, global_fit=False, chunk=8192):
    """eps_H of (64) for SI, TD, SLRI or SSPI from a host-only plan's FP64
    fit (the same fit the device plan uses), summed over (location, pair)
    blocks by row_errors."""
    p = native.Plan(cfg["mics"], cfg["grid"], cfg["fs"], cfg["N"], variant, rq, device=-1, c=cfg["c"],
                    far_field=far_field, global_fit=global_fit)
    info = p.info()
    P, K, J = info["P"], info["K"], info["J"]
    x = p.export("tdoa").reshape(P, J)
    Np = p.export("np").astype(np.int64)
    off = np.concatenate([[0], np.cumsum(2 * Np + 1)])
    num = 0.0
    if variant in ("slri", "si") and global_fit:
        U = p.export("slri_u").reshape(J, -1)
        V = p.export("slri_v").reshape(int(off[-1]), -1)
        for j0 in range(0, J, chunk):
            lam = U[j0:j0 + chunk] @ V.T                     # rows of the stacked fit
            for q in range(P):
                lags = np.arange(-Np[q], Np[q] + 1)
                num += np.sum(row_errors(lags, lam[:, off[q]:off[q + 1]], x[q, j0:j0 + chunk], K))
    elif variant in ("slri", "si"):
        U = p.export("slri_u").reshape(P, J, -1)
        R = U.shape[2]
        V = p.export("slri_v").reshape(P, -1, R)
        for q in range(P):
            lags = np.arange(-Np[q], Np[q] + 1)
            Vq = V[q, :2 * Np[q] + 1]
            for j0 in range(0, J, chunk):
                lam = U[q, j0:j0 + chunk] @ Vq.T
                num += np.sum(row_errors(lags, lam, x[q, j0:j0 + chunk], K))
    else:
        start = p.export("sspi_start").reshape(J, P)
        w = p.export("sspi_w").reshape(J, P, -1)
        lags = start[:, :, None] + np.arange(w.shape[2])[None, None, :]
        num = float(np.sum(row_errors(lags, w, x.T, K)))
    p.close()
    return 10.0 * np.log10(max(num, 1e-300) / (J * P * (K - 1.0)))


def map_error_db(z, z_ref):
    """eps_z of Sec. V-A per frame (rows), in dB; -inf where the maps agree."""
    num = np.sum((z - z_ref) ** 2, axis=1)
    den = np.sum(z_ref ** 2, axis=1)
    with np.errstate(divide="ignore"):
        return 10.0 * np.log10(num / den)


def run(scene="nf4", n_sources=16, frames=8, dtype="f32", forms=None, seed=0, log=None, **scene_kw):
    import torch
    from . import native, scenes
    native.lib()
    forms = forms or list(SWEEPS)
    t0 = time.time()
    cfg, Y, truth = scenes.evaluation_scene(scene, n_sources, frames, seed=seed, **scene_kw)
    far = cfg["far_field"]
    thresholds = FF_THRESHOLDS if far else NF_THRESHOLDS
    Yt = torch.from_numpy(Y).cuda()
    grid = cfg["grid"]
    J = grid.shape[0]

    def plan(variant, rq=0, dt="f32", **kw):
        return native.Plan(cfg["mics"], grid, cfg["fs"], cfg["N"], variant, rq, dtype=dt, c=cfg["c"],
                           far_field=far, **kw)

    ref_plan = plan("fd", dt="f64")
    z_ref = ref_plan.compute(Yt)
    info = ref_plan.info()
    C = 2.0 * J * info["P"] * (info["K"] - 1)
    z_ref_h = z_ref.cpu().numpy().astype(np.float64)
    ref_plan.close()
    if log:
        log(f"scene {scene}: J={J}, {len(Y)} frames, reference in {time.time() - t0:.1f} s")
    rows = []
    for form in forms:
        for setting in SWEEPS[form]:
            kw = dict(setting)
            variant = kw.pop("variant")
            rq = kw.pop("rq", 0)
            if variant == "lr" and min(J, info["P"] * (info["K"] - 1)) > 8192:
                rows.append({"form": form, "setting": rq, "skipped": "H's Gram matrix above 8192 (slow fit)"})
                continue
            t1 = time.time()
            try:
                p = plan(variant, rq, dtype if variant != "fd" else "f32", **kw)
            except native.SrpError as e:
                if variant != "si":
                    rows.append({"form": form, "setting": rq, "skipped": str(e)})
                    continue
                # SI (44) is also global SLRI at full rank R_Lambda = PN,
                # whose tall operand (J x PN) is smaller than the per-pair
                # form's (J x P max_p (2 N_p + 1)) when the lag counts differ
                p = plan("slri", info["PN"], dtype, global_fit=True)
                variant, rq, kw = "slri", info["PN"], {"global_fit": True}
            plan_s = time.time() - t1
            z = p.compute(Yt)
            idx, _ = native.argmax(z)
            torch.cuda.synchronize()
            zh = z.cpu().numpy().astype(np.float64)
            eps_z = map_error_db(zh, z_ref_h)
            eps_s = localisation_error(grid, idx.cpu().numpy(), truth, far)
            pi = p.info()
            row = {"form": form, "setting": pi["rank_or_q"] if variant != "fd" else 0, "requested": rq,
                   "C_rel": pi["macs_per_map"] / C, "plan_seconds": plan_s,
                   "eps_z_db": {"median": float(np.median(eps_z)), "p10": float(np.percentile(eps_z, 10)),
                                "p90": float(np.percentile(eps_z, 90))} if variant != "fd" else None,
                   "rho_s": accuracy(eps_s, thresholds),
                   "eps_s_median": float(np.median(eps_s))}
            if variant == "lr":
                sv = p.export("lr_s")
                frac = max(1.0 - float(np.sum(sv ** 2)) / C * 2.0, 1e-16)  # C / 2 = J P (K - 1) = ||H||_F^2
                row["eps_H_db"] = 10.0 * np.log10(frac)
            elif variant != "fd":
                row["eps_H_db"] = eps_h_db(native, cfg, variant, rq, far, kw.get("global_fit", False))
            rows.append(row)
            p.close()
            del z
            if log:
                log(f"{form} {rq}: C_rel {row['C_rel']:.2e}, eps_z {row['eps_z_db']}, rho_s {row['rho_s']}")
    return {"scene": scene, "J": J, "frames": int(len(Y)), "sources": n_sources, "dtype": dtype,
            "thresholds": list(thresholds), "far_field": far, "rows": rows}


def markdown(res):
    th = res["thresholds"]
    unit = "deg" if res["far_field"] else "m"
    lines = [f"scene {res['scene']}: J = {res['J']}, {res['frames']} frames from {res['sources']} sources, "
             f"{res['dtype']} operands", "",
             "| form | setting | C_rel | eps_H dB | median eps_z dB (p10, p90) | " +
             " | ".join(f"rho_s @ {t:g} {unit}" for t in th) + " |",
             "|---|---:|---:|---:|---|" + "---:|" * len(th)]
    for r in res["rows"]:
        if "skipped" in r:
            lines.append(f"| {r['form']} | {r['setting']} | — | — | skipped: {r['skipped'][:60]} |" + " |" * len(th))
            continue
        e = r["eps_z_db"]
        es = "reference" if e is None else f"{e['median']:.1f} ({e['p10']:.1f}, {e['p90']:.1f})"
        eh = f"{r['eps_H_db']:.1f}" if "eps_H_db" in r else "—"
        lines.append(f"| {r['form']} | {r['setting']} | {r['C_rel']:.2e} | {eh} | {es} | " +
                     " | ".join(f"{r['rho_s'][f'{t:g}']:.2f}" for t in th) + " |")
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--scene", default="nf4", choices=["nf4", "ff6", "room", "square", "farfield"])
    ap.add_argument("--sources", type=int, default=16)
    ap.add_argument("--frames", type=int, default=8)
    ap.add_argument("--dtype", default="f32")
    ap.add_argument("--forms", default=",".join(SWEEPS))
    ap.add_argument("--grid-stride", type=int, default=2)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)

    def log(msg):
        print(f"[eval] {msg}", file=sys.stderr, flush=True)

    kw = {"grid_stride": args.grid_stride} if args.scene == "room" else {}
    res = run(args.scene, args.sources, args.frames, args.dtype, args.forms.split(","), log=log, **kw)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)
    sys.stdout.write(markdown(res))


if __name__ == "__main__":
    main()
