"""GPU test of the continuous-batching server: a Poisson mix of requests over
several resident plans (arrays and grids of different sizes, FD/SLRI/SSPI,
BF16 operands) is served with overlapping streams, and every request's maps
are bitwise identical to the same request computed alone."""

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


@pytest.mark.parametrize("M", [4, 8, 16])
@pytest.mark.parametrize("variant,rq", [("fd", 0), ("slri", 8), ("sspi", 4), ("sspi", 7)])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_maps_do_not_depend_on_the_frame_slot(M, variant, rq, dtype):
    """A frame's map is bitwise the same whatever its position in the batch
    (tile slot, tile index, chunk): the property continuous batching needs."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_08514_amd import native
    print(f"[gpu-case] slot invariance M={M} {variant} {rq} {dtype}", flush=True)
    mics, fs, N = scenes.serving_array(M)
    pool = torch.from_numpy(scenes.serving_frames(M, L=96)).cuda()
    p = native.Plan(mics, scenes.serving_grid(1024), fs, N, variant, rq, dtype=dtype, frame_tile=64)
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
