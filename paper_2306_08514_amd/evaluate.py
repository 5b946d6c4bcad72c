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
          in FP32 (median and 10th / 90th percentiles);
  eps_H   for LR-SRP, 10 log10 of the discarded energy of H: since every
          entry of H has unit modulus, ||H||_F^2 = J P (K - 1) and
          ||H - H_lr||_F^2 = ||H||_F^2 - sum_{r <= R_H} sigma_r^2;
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

    ref_plan = plan("fd")
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
                # SI (44) is global SLRI at full rank R_Lambda = PN, which
                # has no per-pair lag limit
                p = plan("slri", info["PN"], dtype, global_fit=True)
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
             "| form | setting | C_rel | median eps_z dB (p10, p90) | " +
             " | ".join(f"rho_s @ {t:g} {unit}" for t in th) + " |",
             "|---|---:|---:|---|" + "---:|" * len(th)]
    for r in res["rows"]:
        if "skipped" in r:
            lines.append(f"| {r['form']} | {r['setting']} | — | skipped: {r['skipped'][:60]} |" + " |" * len(th))
            continue
        e = r["eps_z_db"]
        es = "reference" if e is None else f"{e['median']:.1f} ({e['p10']:.1f}, {e['p90']:.1f})"
        lines.append(f"| {r['form']} | {r['setting']} | {r['C_rel']:.2e} | {es} | " +
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
