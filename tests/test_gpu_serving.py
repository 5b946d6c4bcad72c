"""GPU test of the continuous-batching server: a Poisson mix of requests over
several resident plans (arrays and grids of different sizes, FD/SLRI/SSPI,
BF16 operands) is served with overlapping streams, and every request's maps
are bitwise identical to the same request computed alone.  A second mix
holds the large classes of the serving workload: the 32-microphone 2 m disc
array (496 pairs, 48 kHz, N = 2048; FD with generated steering) and the
125k and 200k grids, next to small plans."""

import time

import numpy as np
import pytest

from paper_2306_08514_amd import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_08514_amd import native
    from paper_2306_08514_amd.serving import Server, TorchExecutor
    native.lib()
    ex = TorchExecutor(device=0, n_slots=4)
    srv = Server(ex, n_slots=4, max_batch_frames=256).start()
    pools, plans = {}, []
    for M in (4, 8, 16):
        mics, fs, N = scenes.serving_array(M)
        pools[M] = torch.from_numpy(scenes.serving_frames(M, L=96)).cuda()
        for J in (1024, 16384):
            grid = scenes.serving_grid(J)
            for variant, rq in (("fd", 0), ("slri", 8), ("sspi", 4), ("slri", 13), ("sspi", 7)):
                key = (M, J, variant, rq)
                srv.register(key, mics=mics, grid=grid, fs=fs, N=N, variant=variant, rank_or_q=rq,
                             dtype="bf16")
                plans.append(key)
    yield srv, ex, pools, plans
    srv.stop()


@pytest.mark.parametrize("M", [4, 8, 16, 32])
@pytest.mark.parametrize("variant,rq", [("fd", 0), ("fdgen", 0), ("slri", 8), ("sspi", 4), ("sspi", 7)])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_maps_do_not_depend_on_the_frame_slot(M, variant, rq, dtype):
    """A frame's map is bitwise the same whatever its position in the batch
    (tile slot, tile index, chunk): the property continuous batching needs.
    fdgen: conv. FD-SRP with generated steering, whose contraction is split
    over pairs on this small grid."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_08514_amd import native
    print(f"[gpu-case] slot invariance M={M} {variant} {rq} {dtype}", flush=True)
    mics, fs, N = scenes.serving_array(M)
    pool = torch.from_numpy(scenes.serving_frames(M, L=96)).cuda()
    kw = {"fd_steering": "generated"} if variant == "fdgen" else {}
    p = native.Plan(mics, scenes.serving_grid(1024), fs, N, "fd" if variant == "fdgen" else variant, rq,
                    dtype=dtype, frame_tile=64, **kw)
    ref = p.compute(pool[10:30].contiguous())
    for lo, hi in ((0, 10), (3, 10), (17, 10), (46, 5), (0, 57)):
        # 20 frames at offset `lo` (+ `hi` more after them) in one call
        batch = torch.cat([pool[50:50 + lo], pool[10:30], pool[30:30 + hi]], 0)
        z = p.compute(batch)[lo:lo + 20]
        torch.cuda.synchronize()
        assert torch.equal(z, ref), (lo, hi)
    p.close()


def test_mix_results_equal_alone(setup):
    srv, ex, pools, plans = setup
    print("[gpu-case] serving mix", flush=True)
    rng = np.random.default_rng(3)
    reqs = []
    t = 0.0
    t0 = time.perf_counter()
    for i in range(240):
        t += rng.exponential(1.0 / 4000.0)
        key = plans[rng.integers(len(plans))]
        n = int(rng.integers(1, 65))
        l0 = int(rng.integers(0, 96 - n + 1))
        fr = pools[key[0]][l0:l0 + n]
        while time.perf_counter() - t0 < t:
            pass
        reqs.append((key, fr, srv.submit(key, fr)))
    # a burst: every slot busy at once
    for i in range(60):
        key = plans[i % len(plans)]
        n = int(rng.integers(1, 65))
        fr = pools[key[0]][:n]
        reqs.append((key, fr, srv.submit(key, fr)))
    assert srv.drain(timeout=120)
    st = srv.stats()
    print("serving stats", st, flush=True)
    for key, fr, fut in reqs:
        z = fut.result()
        alone = ex.plan(key).compute(fr.contiguous())
        torch.cuda.synchronize()
        assert torch.equal(z, alone), key
    assert st["requests"] == 300
    assert st["failed_requests"] == 0
    assert st["max_inflight"] >= 2


@pytest.fixture(scope="module")
def large_setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_08514_amd import native
    from paper_2306_08514_amd.serving import Server, TorchExecutor
    native.lib()
    ex = TorchExecutor(device=0, n_slots=4)
    srv = Server(ex, n_slots=4, max_batch_frames=256).start()
    pools, plans = {}, []
    specs = [(32, 200000, "fd", 0), (32, 200000, "slri", 8), (32, 200000, "sspi", 4),
             (32, 125000, "slri", 12), (32, 125000, "sspi", 6), (32, 125000, "fd", 0),
             (8, 125000, "fd", 0), (8, 125000, "slri", 8), (8, 125000, "sspi", 4),
             (16, 200000, "sspi", 5), (4, 1024, "fd", 0), (16, 16384, "slri", 16)]
    for M, J, variant, rq in specs:
        mics, fs, N = scenes.serving_array(M)
        if M not in pools:
            pools[M] = torch.from_numpy(scenes.serving_frames(M, L=96)).cuda()
        key = (M, J, variant, rq)
        print(f"[gpu-case] register {key}", flush=True)
        srv.register(key, mics=mics, grid=scenes.serving_grid(J), fs=fs, N=N, variant=variant,
                     rank_or_q=rq, dtype="bf16")
        plans.append(key)
    yield srv, ex, pools, plans
    srv.stop()
    for key in plans:
        ex.drop(key)
    torch.cuda.empty_cache()


def test_large_classes_mix_results_equal_alone(large_setup):
    """M = 32 and J in {125k, 200k} requests (1-64 frames) arriving while
    others run, coalesced per plan up to 256 frames, against each request
    computed alone."""
    srv, ex, pools, plans = large_setup
    print("[gpu-case] serving mix, large classes", flush=True)
    rng = np.random.default_rng(5)
    reqs = []
    t = 0.0
    t0 = time.perf_counter()
    for i in range(48):
        t += rng.exponential(1.0 / 400.0)
        key = plans[rng.integers(len(plans))]
        n = int(rng.integers(1, 65))
        l0 = int(rng.integers(0, 96 - n + 1))
        fr = pools[key[0]][l0:l0 + n]
        while time.perf_counter() - t0 < t:
            pass
        reqs.append((key, fr, srv.submit(key, fr)))
    # a burst over every plan, two requests each, so same-plan requests
    # coalesce and several plans run at once
    for i in range(2 * len(plans)):
        key = plans[i % len(plans)]
        n = int(rng.integers(1, 65))
        fr = pools[key[0]][96 - n:]
        reqs.append((key, fr, srv.submit(key, fr)))
    assert srv.drain(timeout=120)
    st = srv.stats()
    print("serving stats (large classes)", st, flush=True)
    for key, fr, fut in reqs:
        z = fut.result()
        alone = ex.plan(key).compute(fr.contiguous())
        torch.cuda.synchronize()
        assert torch.equal(z, alone), key
    assert st["failed_requests"] == 0
    assert st["max_inflight"] >= 2
    assert st["requests"] == len(reqs)
    assert st["requests_per_batch"] > 1.0
