"""Serving-mix benchmark on one GPU.

Plans for every array x grid of the serving mix are registered and stay
resident: M in {4, 8, 16, 32} microphones (0.2 m square, 0.3 m and 0.5 m
UCAs, 2 m disc), J in {1024, 16384, 125000, 200000} candidates, and for each
the forms conv. FD-SRP, SLRI with R = 4..16 per pair and SSPI with
Q = 2..8, all with BF16 operands (4 x 4 x 21 = 336 plans).  Requests then
arrive as a seeded Poisson process; each picks M, J and the form uniformly
(R or Q uniformly in its range) and 1..64 frames from that array's pool of
synthetic frames.  The continuous-batching server coalesces and overlaps
them; per rate the benchmark reports the offered and achieved load, p50/p99
latency from submission to maps ready, and batching statistics.

Before the runs every plan is timed alone (32- and 256-frame batches): the
cost model gives the offered load of each rate in device-seconds per
second and the rate at which the mix would fill the device; past it the
queue grows without bound and p99 with the run's length.

    python -m paper_2306_08514_amd.serve_bench [--rates 500,1000,2000] [--duration 10]
"""

import argparse
import json
import sys
import time

import numpy as np


def build_catalogue(srv, pools, log):
    from . import scenes
    keys, t_kind = [], {"fd": 0.0, "slri": 0.0, "sspi": 0.0}
    for M in scenes.SERVING_M:
        mics, fs, N = scenes.serving_array(M)
        for J in scenes.SERVING_J:
            grid = scenes.serving_grid(J)
            for variant, params in (("fd", [0]), ("slri", range(4, 17)), ("sspi", range(2, 9))):
                for rq in params:
                    key = (M, J, variant, rq)
                    t0 = time.perf_counter()
                    srv.register(key, mics=mics, grid=grid, fs=fs, N=N, variant=variant, rank_or_q=rq,
                                 dtype="bf16")
                    t_kind[variant] += time.perf_counter() - t0
                    keys.append(key)
            log(f"registered M={M} J={J}: {len(keys)} plans, resident {srv.resident_bytes() / 2**30:.1f} GiB")
    return keys, t_kind


def cost_model(ex, keys, pools, log, frames=(32, 256)):
    """Device milliseconds per map of every plan, each alone on the device,
    for batches of 32 frames (about the mean request, 32.5 frames) and of
    256 frames (the largest coalesced batch); from HIP events around
    three calls after one warm-up call."""
    import torch
    out = {}
    for key in keys:
        p = ex.plan(key)
        row = {}
        for n in frames:
            fr = pools[key[0]][:n].contiguous()
            z = p.empty_maps(n)
            ws = torch.empty(max(1, p.workspace_size(n)), dtype=torch.uint8, device="cuda")
            p.compute(fr, maps=z, workspace=ws)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(3):
                p.compute(fr, maps=z, workspace=ws)
            e1.record()
            torch.cuda.synchronize()
            row[n] = e0.elapsed_time(e1) / 3 / n
            del z, ws
        out[key] = row
    torch.cuda.empty_cache()
    log(f"cost model: {len(out)} plans timed")
    return out


def offered_load(costs, rate, frames_mean=32.5, batch=32):
    """Device seconds per second that requests at `rate` per second bring, in
    the mix's proportions (M, J and the form uniform, R or Q uniform in
    their ranges), each map at its plan's cost for `batch`-frame batches."""
    from . import scenes
    tot = 0.0
    nM, nJ = len(scenes.SERVING_M), len(scenes.SERVING_J)
    for M in scenes.SERVING_M:
        for J in scenes.SERVING_J:
            for variant, params in (("fd", [0]), ("slri", range(4, 17)), ("sspi", range(2, 9))):
                c = np.mean([costs[(M, J, variant, rq)][batch] for rq in params])
                tot += c / (nM * nJ * 3)
    return rate * frames_mean * tot / 1e3


def run_rate(srv, pools, rate, duration, rng, log):
    from . import scenes
    import torch
    srv.reset_stats()
    n = int(rate * duration)
    gaps = rng.exponential(1.0 / rate, n)
    arrivals = np.cumsum(gaps)
    forms = ["fd", "slri", "sspi"]
    frames_total = 0
    # results are dropped as they complete (a request's maps are not kept):
    # only completions and errors are counted
    counts = {"done": 0, "failed": 0, "rejected": 0}

    def on_done(f):
        e = f.exception()
        if e is None:
            counts["done"] += 1
        elif "queue full" in str(e):
            counts["rejected"] += 1
        else:
            counts["failed"] += 1
    t0 = time.perf_counter()
    for i in range(n):
        M = scenes.SERVING_M[rng.integers(4)]
        J = scenes.SERVING_J[rng.integers(4)]
        variant = forms[rng.integers(3)]
        rq = 0 if variant == "fd" else int(rng.integers(4, 17) if variant == "slri" else rng.integers(2, 9))
        nf = int(rng.integers(1, 65))
        l0 = int(rng.integers(0, pools[M].shape[0] - nf + 1))
        # pace by sleeping (a spin would hold the GIL and starve the
        # scheduler thread)
        dt = arrivals[i] - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        srv.submit((M, J, variant, rq), pools[M][l0:l0 + nf]).add_done_callback(on_done)
        frames_total += nf
    t_sub = time.perf_counter() - t0
    ok = srv.drain(timeout=600)
    t_all = time.perf_counter() - t0
    st = srv.stats()
    res = {"offered_req_per_s": n / arrivals[-1], "offered_maps_per_s": frames_total / arrivals[-1],
           "requests": n, "maps": frames_total, "submit_seconds": t_sub, "total_seconds": t_all,
           "drained": bool(ok), "completed_requests": counts["done"], "failed": counts["failed"],
           "rejected": counts["rejected"],
           "achieved_maps_per_s": st["maps"] / t_all, **st}
    log(f"rate {rate}/s: offered {res['offered_maps_per_s']:.0f} maps/s, achieved {res['achieved_maps_per_s']:.0f} "
        f"maps/s, p50 {st['p50_ms']:.1f} ms, p99 {st['p99_ms']:.1f} ms, {st['requests_per_batch']:.2f} req/batch, "
        f"{st['rejected_requests']} rejected")
    torch.cuda.synchronize()
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--rates", default="500,1000,2000")
    ap.add_argument("--duration", type=float, default=10.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--max-batch-frames", type=int, default=256)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--max-queue", type=int, default=1024)
    args = ap.parse_args(argv)

    def log(msg):
        print(f"[serve] {msg}", file=sys.stderr, flush=True)

    import torch
    from . import native, scenes
    from .serving import Server, TorchExecutor
    native.lib()
    t0 = time.perf_counter()
    pools = {M: torch.from_numpy(scenes.serving_frames(M, 256)).cuda() for M in scenes.SERVING_M}
    log(f"frame pools in {time.perf_counter() - t0:.1f} s")
    ex = TorchExecutor(device=0, n_slots=args.slots, timing=True)
    srv = Server(ex, n_slots=args.slots, max_batch_frames=args.max_batch_frames, max_queue=args.max_queue).start()
    t1 = time.perf_counter()
    keys, t_kind = build_catalogue(srv, pools, log)
    t_reg = time.perf_counter() - t1
    # warm-up: every plan once
    for k in keys:
        srv.submit(k, pools[k[0]][:4])
    srv.drain(timeout=600)
    costs = cost_model(ex, keys, pools, log)
    # the rate at which the mix would occupy the device fully (offered load
    # 1 device-second per second) with 32-frame and with 256-frame batches
    cap32 = 1.0 / offered_load(costs, 1.0, batch=32)
    cap256 = 1.0 / offered_load(costs, 1.0, batch=256)
    log(f"cost model: the mix fills the device at {cap32:.0f} req/s (32-frame batches), "
        f"{cap256:.0f} req/s (256-frame batches)")
    by_class = {}
    for (M, J, variant, rq), c in costs.items():
        by_class.setdefault(f"{variant} M={M} J={J}", []).append(c[32])
    rng = np.random.default_rng(2306085144 + args.seed)
    results = {}
    for rate in [float(r) for r in args.rates.split(",")]:
        ex.busy = {}
        results[f"{rate:g}"] = run_rate(srv, pools, rate, args.duration, rng, log)
        results[f"{rate:g}"]["offered_load_cost_model"] = {"batch32": offered_load(costs, rate, batch=32),
                                                           "batch256": offered_load(costs, rate, batch=256)}
        # batch spans (start to done on the slot's stream, overlapping other
        # slots) by plan class, largest first
        spans = sorted(ex.busy.items(), key=lambda kv: -kv[1][0])
        results[f"{rate:g}"]["batch_span_ms_by_class"] = [
            {"variant": k[0], "M": k[1], "J": k[2], "span_ms": v[0], "batches": v[1], "frames": v[2]}
            for k, v in spans[:16]]
    srv.stop()
    out = {"workload": "serving mix: Poisson arrivals; M in {4,8,16,32}, J in {1k,16k,125k,200k}, "
                       "FD / SLRI R=4..16 / SSPI Q=2..8 uniform, 1-64 frames, BF16 operands",
           "plans": len(keys), "resident_gib": srv.resident_bytes() / 2 ** 30,
           "registration_seconds": t_reg, "registration_seconds_by_form": t_kind,
           "slots": args.slots, "max_batch_frames": args.max_batch_frames, "duration_s": args.duration,
           "cost_model": {"capacity_req_per_s_batch32": cap32, "capacity_req_per_s_batch256": cap256,
                          "ms_per_map_batch32_by_class": {k: float(np.mean(v)) for k, v in
                                                          sorted(by_class.items(), key=lambda kv: -np.mean(kv[1]))}},
           "rates": results}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
