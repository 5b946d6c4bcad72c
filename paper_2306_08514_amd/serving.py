"""Continuous-batching SRP-map server.

Requests are (plan key, frames) pairs.  Plans are registered once and stay
resident in HBM; their bytes are charged against the device budget for as
long as they live.  A scheduler thread

* admits queued requests whenever a stream slot is free and the request's
  workspace, output and staging bytes fit the remaining budget,
* coalesces the queued requests of one plan along the frame axis into one
  library call (every map depends only on its own frame and the plan, so a
  request's maps are bitwise the same alone or inside a batch),
* runs the batches of different slots concurrently on separate streams, and
* completes a request when its batch's event has fired, recording the
  latency from submission to completion.

The executor performs the device work; `TorchExecutor` drives the HIP
library through torch streams.  Any object with the same methods can stand
in for it (the tests use a CPU one).
"""

import collections
import concurrent.futures
import threading
import time

import numpy as np


class AdmissionError(RuntimeError):
    """A request can never fit the memory budget."""


class _Request:
    __slots__ = ("key", "frames", "n", "t_submit", "future", "ready")

    def __init__(self, key, frames, n, future, ready):
        self.key, self.frames, self.n = key, frames, n
        self.future, self.ready = future, ready
        self.t_submit = time.perf_counter()


class _Batch:
    __slots__ = ("key", "requests", "frames", "bytes", "handle", "slot", "t_launch")


class Server:
    """Continuous-batching scheduler over an executor.

    executor       object with build/footprint/launch/poll/results/release
    n_slots        batches that may be in flight at once (one stream each)
    hbm_budget     bytes available to plans plus in-flight work (None: the
                   executor's default)
    max_batch_frames  cap on the frames coalesced into one batch
    max_queue      requests that may wait; beyond it submit() fails fast with
                   AdmissionError (backpressure: every waiting request holds
                   device resources such as its ready event)
    """

    def __init__(self, executor, n_slots=4, hbm_budget=None, max_batch_frames=1024,
                 poll_interval=20e-6, max_queue=1024):
        self.ex = executor
        self.n_slots = int(n_slots)
        self.max_queue = int(max_queue)
        self.budget = int(hbm_budget if hbm_budget is not None else executor.default_budget())
        self.max_batch_frames = int(max_batch_frames)
        self.poll_interval = poll_interval
        self._plans = {}                     # key -> resident bytes
        self._queue = collections.deque()    # FIFO of _Request
        self._inflight = []                  # _Batch
        self._free_slots = list(range(self.n_slots))
        self._lock = threading.Condition()
        self._thread = None
        self._stop = False
        self._lat = []                       # seconds per completed request
        self._maps_done = 0
        self._t0 = None
        self._t_last = None
        self._batches = 0
        self._coalesced = 0
        self._max_inflight = 0
        self._failed = 0
        self._rejected = 0
        self.error = None

    # --------------------------------------------------------------- plans --
    def register(self, key, **spec):
        """Builds the plan `key` and keeps it resident; raises AdmissionError if
        its bytes do not fit the budget next to the plans already resident."""
        with self._lock:
            if key in self._plans:
                return self._plans[key]
            used = sum(self._plans.values())
        nbytes = self.ex.build(key, spec, self.budget - used)
        with self._lock:
            if sum(self._plans.values()) + nbytes > self.budget:
                self.ex.drop(key)
                raise AdmissionError(f"plan {key!r} needs {nbytes} bytes; budget {self.budget} "
                                     f"with {sum(self._plans.values())} already resident")
            self._plans[key] = nbytes
        return nbytes

    def resident_bytes(self):
        with self._lock:
            return sum(self._plans.values())

    # ------------------------------------------------------------- requests --
    def submit(self, key, frames):
        """Queues one request; returns a Future resolving to its maps."""
        fut = concurrent.futures.Future()
        if key not in self._plans:
            fut.set_exception(KeyError(f"unknown plan {key!r}"))
            return fut
        with self._lock:
            full = len(self._queue) >= self.max_queue
        if full:
            with self._lock:
                self._rejected += 1
            fut.set_exception(AdmissionError(f"queue full ({self.max_queue} requests waiting)"))
            return fut
        n = self.ex.frames_len(frames)
        need = self.ex.footprint(key, n)
        if sum(self._plans.values()) + need > self.budget:
            fut.set_exception(AdmissionError(
                f"request of {n} frames needs {need} bytes beyond the resident plans; budget "
                f"{self.budget}"))
            return fut
        req = _Request(key, frames, n, fut, self.ex.mark_ready(frames))
        with self._lock:
            if self._t0 is None:
                self._t0 = req.t_submit
            self._queue.append(req)
            self._lock.notify()
        return fut

    # ------------------------------------------------------------ scheduler --
    def start(self):
        if self._thread is None:
            self._stop = False
            self._thread = threading.Thread(target=self._run, name="srp-scheduler", daemon=True)
            self._thread.start()
        return self

    def stop(self, drain=True):
        if drain:
            self.drain()
        with self._lock:
            self._stop = True
            self._lock.notify()
        if self._thread is not None:
            self._thread.join()
            self._thread = None
        with self._lock:
            pending = list(self._queue)
            self._queue.clear()
        for r in pending:
            r.future.cancel()

    def drain(self, timeout=None):
        t_end = None if timeout is None else time.perf_counter() + timeout
        while True:
            with self._lock:
                if not self._queue and not self._inflight:
                    return True
                if self.error is not None:
                    raise self.error
            if t_end is not None and time.perf_counter() > t_end:
                return False
            time.sleep(self.poll_interval * 10)

    def _inflight_bytes(self):
        return sum(b.bytes for b in self._inflight)

    def _take_batch(self):
        """Pops the head request's plan's queued requests (FIFO) that fit the
        frame cap and the free memory; None if the head does not fit now."""
        head = self._queue[0]
        free = self.budget - sum(self._plans.values()) - self._inflight_bytes()
        take, frames = [], 0
        for r in list(self._queue):
            if r.key != head.key:
                continue
            if take and frames + r.n > self.max_batch_frames:
                break
            if self.ex.footprint(r.key, frames + r.n) > free:
                break
            take.append(r)
            frames += r.n
        if not take:
            return None
        for r in take:
            self._queue.remove(r)
        b = _Batch()
        b.key, b.requests, b.frames = head.key, take, frames
        b.bytes = self.ex.footprint(head.key, frames)
        return b

    def _complete(self, b):
        outs = self.ex.results(b.handle)
        t = time.perf_counter()
        for r, z in zip(b.requests, outs):
            if not r.future.cancelled():
                r.future.set_result(z)
            self._lat.append(t - r.t_submit)
        self._maps_done += b.frames
        self._t_last = t
        self.ex.release(b.handle)
        self._free_slots.append(b.slot)

    def _run(self):
        try:
            while True:
                with self._lock:
                    if self._stop:
                        return
                    # completions
                    still = []
                    for b in self._inflight:
                        if self.ex.poll(b.handle):
                            self._complete(b)
                        else:
                            still.append(b)
                    self._inflight = still
                    # admissions: continuous batching
                    while self._queue and self._free_slots:
                        # drop cancelled requests at the head
                        while self._queue and self._queue[0].future.cancelled():
                            self._queue.popleft()
                        if not self._queue:
                            break
                        b = self._take_batch()
                        if b is None:
                            break
                        b.slot = self._free_slots.pop()
                        b.t_launch = time.perf_counter()
                        try:
                            b.handle = self.ex.launch(b.key, [r.frames for r in b.requests],
                                                      [r.ready for r in b.requests], b.slot)
                        except Exception as e:  # this batch fails; the server keeps serving
                            for r in b.requests:
                                if not r.future.done():
                                    r.future.set_exception(e)
                            self._free_slots.append(b.slot)
                            self._failed += len(b.requests)
                            continue
                        self._inflight.append(b)
                        self._batches += 1
                        self._coalesced += len(b.requests)
                        self._max_inflight = max(self._max_inflight, len(self._inflight))
                    idle = not self._inflight and not self._queue
                    if idle:
                        self._lock.wait(timeout=0.01)
                if not idle:
                    time.sleep(self.poll_interval)
        except BaseException as e:  # surfaced by drain()
            self.error = e
            with self._lock:
                for b in self._inflight:
                    for r in b.requests:
                        if not r.future.done():
                            r.future.set_exception(e)
                for r in self._queue:
                    if not r.future.done():
                        r.future.set_exception(e)

    # ---------------------------------------------------------------- stats --
    def reset_stats(self):
        """Starts a new measurement window (in-flight work is not affected)."""
        with self._lock:
            self._lat = []
            self._maps_done = 0
            self._t0 = None
            self._t_last = None
            self._batches = 0
            self._coalesced = 0
            self._max_inflight = len(self._inflight)
            self._failed = 0
            self._rejected = 0

    def stats(self):
        lat = np.array(self._lat) * 1e3
        span = (self._t_last - self._t0) if self._t0 is not None and self._t_last is not None else 0.0
        return {
            "requests": int(lat.size),
            "maps": int(self._maps_done),
            "batches": int(self._batches),
            "requests_per_batch": self._coalesced / max(1, self._batches),
            "max_inflight": int(self._max_inflight),
            "failed_requests": int(self._failed),
            "rejected_requests": int(self._rejected),
            "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_ms": float(lat.mean()) if lat.size else None,
            "maps_per_s": self._maps_done / span if span > 0 else None,
            "resident_bytes": self.resident_bytes(),
        }


class TorchExecutor:
    """Runs batches through the HIP library on a pool of torch streams.

    Plans are native.Plan objects built on `device`.  A batch's frames are
    concatenated on its slot's stream (after waiting for each request's
    ready event), the library computes into a fresh output, and an event on
    the slot's stream marks completion."""

    def __init__(self, device=0, n_slots=4, timing=False):
        import torch
        from . import native
        self.torch, self.native = torch, native
        self.timing = bool(timing)
        self.busy = {}  # (variant, M, J) -> (device ms, batches, frames) when timing
        self.device = torch.device("cuda", device)
        self.dev_index = device
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_slots)]
        self.plans = {}

    def default_budget(self):
        free, _ = self.torch.cuda.mem_get_info(self.device)
        return int(free * 0.8)

    def build(self, key, spec, budget_left):
        p = self.native.Plan(device=self.dev_index, hbm_budget=max(1, int(budget_left)), **spec)
        self.plans[key] = p
        return p.info()["device_bytes"]

    def drop(self, key):
        p = self.plans.pop(key, None)
        if p is not None:
            p.close()

    def plan(self, key):
        return self.plans[key]

    def frames_len(self, frames):
        return int(frames.shape[0])

    def footprint(self, key, n):
        p = self.plans[key]
        esz = 8 if p.dtype == "f64" else 4
        frames_bytes = n * p.M * (p.K + 1) * 8
        return p.workspace_size(n) + n * p.map_pitch * esz + frames_bytes

    def mark_ready(self, frames):
        ev = self.torch.cuda.Event()
        ev.record(self.torch.cuda.current_stream(self.device))
        return ev

    def launch(self, key, frames_list, ready, slot):
        torch = self.torch
        p = self.plans[key]
        s = self.streams[slot]
        t0 = None
        with torch.cuda.stream(s):
            for ev in ready:
                s.wait_event(ev)
            for f in frames_list:
                f.record_stream(s)
            fr = frames_list[0] if len(frames_list) == 1 else torch.cat(frames_list, 0)
            L = fr.shape[0]
            ws = torch.empty(max(1, p.workspace_size(L)), dtype=torch.uint8, device=self.device)
            out = p.empty_maps(L, self.device)
            if self.timing:
                t0 = torch.cuda.Event(enable_timing=True)
                t0.record(s)
            p.compute(fr, maps=out, workspace=ws, stream=s)
            done = torch.cuda.Event(enable_timing=self.timing)
            done.record(s)
        sizes = [f.shape[0] for f in frames_list]
        return (done, out, sizes, fr, ws, t0, key)

    def poll(self, handle):
        return handle[0].query()

    def results(self, handle):
        out, sizes = handle[1], handle[2]
        res, o = [], 0
        for n in sizes:
            res.append(out[o:o + n])
            o += n
        return res

    def release(self, handle):
        # the caching allocator reclaims ws / frames once unreferenced
        if self.timing and handle[5] is not None:
            key = handle[6]
            cls = (key[2], key[0], key[1]) if isinstance(key, tuple) and len(key) >= 3 else key
            ms = handle[5].elapsed_time(handle[0])
            tot, n, frames = self.busy.get(cls, (0.0, 0, 0))
            self.busy[cls] = (tot + ms, n + 1, frames + sum(handle[2]))
