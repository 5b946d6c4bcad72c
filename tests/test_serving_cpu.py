"""CPU tests of the continuous-batching scheduler with a fake executor.

The fake executor computes maps with the FP64 oracle (conv. FD-SRP of the
request's frames) and completes a batch after a simulated device time, so
admission, coalescing, slot reuse, budget limits, cancellation and error
propagation are all exercised without a GPU."""

import threading
import time

import numpy as np
import pytest

import oracle as o
from paper_2306_08514_amd import scenes
from paper_2306_08514_amd.serving import AdmissionError, Server


class FakeExecutor:
    def __init__(self, per_frame_s=1e-3, fixed_s=2e-3, plan_bytes=1000, frame_bytes=10,
                 fail_on=None):
        self.per_frame_s, self.fixed_s = per_frame_s, fixed_s
        self.plan_bytes, self.frame_bytes = plan_bytes, frame_bytes
        self.plans = {}
        self.launched = []          # (key, n_requests, frames)
        self.fail_on = fail_on
        self.concurrent = 0
        self.max_concurrent = 0
        self.lock = threading.Lock()

    def default_budget(self):
        return 10 ** 9

    def build(self, key, spec, budget_left):
        cfg = spec["cfg"]
        x = o.tdoa_samples(cfg["mics"], cfg["grid"], cfg["fs"], cfg["c"])
        self.plans[key] = (x, cfg["N"] // 2)
        return self.plan_bytes

    def drop(self, key):
        self.plans.pop(key, None)

    def frames_len(self, frames):
        return frames.shape[0]

    def footprint(self, key, n):
        return n * self.frame_bytes

    def mark_ready(self, frames):
        return None

    def launch(self, key, frames_list, ready, slot):
        if self.fail_on is not None and key == self.fail_on:
            raise RuntimeError("device failure (simulated)")
        x, K = self.plans[key]
        fr = np.concatenate(frames_list, 0)
        z = o.fd_map(o.phat(fr), x, K)
        n = fr.shape[0]
        with self.lock:
            self.launched.append((key, len(frames_list), n))
            self.concurrent += 1
            self.max_concurrent = max(self.max_concurrent, self.concurrent)
        sizes = [f.shape[0] for f in frames_list]
        return {"t": time.perf_counter() + self.fixed_s + self.per_frame_s * n, "z": z, "sizes": sizes,
                "open": True}

    def poll(self, h):
        return time.perf_counter() >= h["t"]

    def results(self, h):
        out, o0 = [], 0
        for n in h["sizes"]:
            out.append(h["z"][o0:o0 + n])
            o0 += n
        return out

    def release(self, h):
        with self.lock:
            self.concurrent -= 1


def _cfg(stride=8):
    return scenes.workload("square4_plane1k", L=40, grid_stride=stride)


@pytest.fixture(scope="module")
def frames():
    cfg = _cfg()
    return cfg, scenes.make_frames(cfg)


def test_results_equal_the_alone_computation_and_requests_coalesce(frames):
    cfg, Y = frames
    ex = FakeExecutor(per_frame_s=2e-3, fixed_s=5e-3)
    srv = Server(ex, n_slots=1, max_batch_frames=64).start()
    srv.register("a", cfg=cfg)
    rng = np.random.default_rng(0)
    reqs = []
    for _ in range(12):
        n = int(rng.integers(1, 5))
        l0 = int(rng.integers(0, Y.shape[0] - n))
        reqs.append((Y[l0:l0 + n], srv.submit("a", Y[l0:l0 + n])))
    srv.drain(timeout=30)
    x = o.tdoa_samples(cfg["mics"], cfg["grid"], cfg["fs"], cfg["c"])
    for fr, fut in reqs:
        # numpy's blocked products are not bitwise batch-invariant; the HIP
        # path is, and the GPU serving test checks it bit for bit
        np.testing.assert_allclose(fut.result(), o.fd_map(o.phat(fr), x, cfg["N"] // 2), rtol=1e-12, atol=1e-9)
    st = srv.stats()
    srv.stop()
    assert st["requests"] == 12
    assert st["batches"] < 12             # later arrivals were coalesced
    assert st["requests_per_batch"] > 1
    assert st["p99_ms"] >= st["p50_ms"] > 0


def test_admission_is_capped_by_memory_not_only_slots(frames):
    cfg, Y = frames
    # 4 slots, but the budget holds the plan plus one 8-frame batch only
    ex = FakeExecutor(per_frame_s=5e-3, fixed_s=5e-3, plan_bytes=1000, frame_bytes=10)
    srv = Server(ex, n_slots=4, hbm_budget=1000 + 80, max_batch_frames=8).start()
    srv.register("a", cfg=cfg)
    futs = [srv.submit("a", Y[i * 8:(i + 1) * 8]) for i in range(4)]
    srv.drain(timeout=30)
    assert all(f.result().shape == (8, cfg["grid"].shape[0]) for f in futs)
    assert ex.max_concurrent == 1
    srv.stop()


def test_slots_overlap_when_memory_allows(frames):
    cfg, Y = frames
    ex = FakeExecutor(per_frame_s=5e-3, fixed_s=10e-3)
    srv = Server(ex, n_slots=3, max_batch_frames=4).start()
    srv.register("a", cfg=cfg)
    srv.register("b", cfg=_cfg(stride=16))
    futs = [srv.submit("a" if i % 2 else "b", Y[i:i + 4]) for i in range(0, 24, 4)]
    srv.drain(timeout=30)
    assert all(f.done() for f in futs)
    assert ex.max_concurrent >= 2
    srv.stop()


def test_over_budget_request_and_plan_are_rejected(frames):
    cfg, Y = frames
    ex = FakeExecutor(plan_bytes=1000, frame_bytes=10)
    srv = Server(ex, n_slots=2, hbm_budget=1050).start()
    srv.register("a", cfg=cfg)
    fut = srv.submit("a", Y[:10])            # needs 100 bytes > 50 left
    with pytest.raises(AdmissionError):
        fut.result(timeout=5)
    with pytest.raises(AdmissionError):
        srv.register("b", cfg=cfg)           # a second 1000-byte plan
    with pytest.raises(KeyError):
        srv.submit("nope", Y[:1]).result(timeout=5)
    ok = srv.submit("a", Y[:5])              # 50 bytes fits
    assert ok.result(timeout=10).shape[0] == 5
    srv.stop()


def test_cancelled_requests_are_skipped(frames):
    cfg, Y = frames
    ex = FakeExecutor(per_frame_s=20e-3, fixed_s=20e-3)
    srv = Server(ex, n_slots=1, max_batch_frames=2).start()
    srv.register("a", cfg=cfg)
    first = srv.submit("a", Y[:2])
    time.sleep(0.005)                        # the first batch is on the device
    queued = [srv.submit("a", Y[2 + 2 * i:4 + 2 * i]) for i in range(3)]
    assert queued[1].cancel()
    srv.drain(timeout=30)
    assert first.done() and queued[0].done() and queued[2].done()
    assert queued[1].cancelled()
    assert sum(n for _, _, n in ex.launched) == 6
    srv.stop()


def test_executor_failure_fails_its_batch_and_the_server_keeps_serving(frames):
    cfg, Y = frames
    ex = FakeExecutor(fail_on="bad")
    srv = Server(ex, n_slots=2).start()
    srv.register("bad", cfg=cfg)
    srv.register("good", cfg=cfg)
    fut = srv.submit("bad", Y[:2])
    with pytest.raises(RuntimeError):
        fut.result(timeout=10)
    ok = srv.submit("good", Y[:3])
    assert ok.result(timeout=10).shape[0] == 3
    assert srv.drain(timeout=10)
    assert srv.stats()["failed_requests"] == 1
    srv.stop()


def test_queue_bound_rejects_fast_and_recovers(frames):
    """Backpressure: with the device busy and the queue at its bound, a new
    request fails at once with AdmissionError; once the queue drains, new
    requests are served again."""
    cfg, Y = frames
    ex = FakeExecutor(per_frame_s=5e-3, fixed_s=200e-3)
    srv = Server(ex, n_slots=1, max_batch_frames=1, max_queue=3).start()
    srv.register("a", cfg=cfg)
    first = srv.submit("a", Y[:1])
    t0 = time.monotonic()
    while not ex.launched and time.monotonic() - t0 < 10:
        time.sleep(0.001)                    # until the first batch is on the device
    assert ex.launched
    queued = [srv.submit("a", Y[i:i + 1]) for i in range(1, 4)]
    over = srv.submit("a", Y[5:6])
    with pytest.raises(AdmissionError):
        over.result(timeout=1)
    assert srv.drain(timeout=30)
    assert first.result().shape[0] == 1 and all(f.result().shape[0] == 1 for f in queued)
    assert srv.stats()["rejected_requests"] == 1
    assert srv.submit("a", Y[:2]).result(timeout=10).shape[0] == 2
    srv.stop()
