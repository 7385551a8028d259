"""Continuous-batching render server for the SAR rasterizer.

Scenes stay resident on the device. Requests (render, or render + L1
gradient against a target) arrive at any time. Planner threads count each
request's pairs exactly (one device query on a stream of their own, off the
scheduler thread) and price it in bytes. The scheduler admits planned
requests into fused launches as launch slots and device memory free up,
checking each candidate batch's exact workspace bytes against the budget. A
fused launch's pair counts are the sums of its requests', so its plan is
built on the host (sdgr_plan_host) without another device query. Requests
that arrive while others run are picked up without waiting for a queue to
drain, and two launches overlap on the device. Each request is its own
scene entry in the fused launch (aliasing the resident tensors), so its
gradient is never mixed with another request's.

The GPU executor calls the library through ``api.Renderer``; a fake executor
with simulated memory and latency drives the same scheduler on the CPU for
tests.
"""
from __future__ import annotations

import collections
import ctypes
import gc
import itertools
import queue
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

__all__ = ["Request", "Result", "Server", "GpuExecutor", "FakeExecutor", "percentile"]


@dataclass
class Request:
    scene_id: str
    views: Sequence            # View-like objects (their `scene` is ignored)
    want_grad: bool = False
    target: object = None      # flat target images (device tensor) for the L1 gradient
    deadline_s: Optional[float] = None   # fail if not admitted within this time
    id: int = -1
    arrival: float = 0.0
    cost: int = 0              # exact workspace bytes alone (set by the planner)
    plan_info: object = None   # executor's planning result (e.g. pair counts)

    @property
    def nviews(self) -> int:
        return len(self.views)

    @property
    def pixels(self) -> int:
        return sum(int(v.img_w) * int(v.img_h) for v in self.views)


@dataclass
class Result:
    request_id: int
    images: list                 # per view, (H, W)
    grads: Optional[dict] = None  # per parameter, same shapes as the scene tensors
    latency_s: float = 0.0
    batch_id: int = -1
    batch_requests: int = 1


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * p / 100.0
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


class _Launch:
    """Handle of one launched batch (executor-specific payload)."""

    def __init__(self, batch_id, requests, bytes_, payload):
        self.batch_id = batch_id
        self.requests = requests
        self.bytes = bytes_
        self.payload = payload


def _plan_bytes(plan, want_grad: bool) -> int:
    return int(plan.state_bytes + plan.fwd_scratch_bytes +
               (plan.bwd_scratch_bytes if want_grad else 0)) + 3 * 256


class GpuExecutor:
    """Fused launches on the device; one HIP stream per launch slot and one
    per planner thread."""

    def __init__(self, scenes: Dict[str, object], device="cuda", options=None, slots=2):
        import torch
        from . import api
        from . import _capi
        self.torch = torch
        self.api = api
        self.C = _capi
        self.lib = _capi.lib()
        self.device = torch.device(device)
        self.scenes = dict(scenes)
        self.options = options or api.RenderOptions()
        self.opts_c = self.options.to_c()
        self.streams = [torch.cuda.Stream(self.device) for _ in range(slots)]
        self.free_streams = list(range(slots))
        self._plan_streams = threading.local()
        # one scene struct per resident scene, reused by every plan
        self._scene_c = {k: api._scene_struct(g) for k, g in self.scenes.items()}

    # -- planning (planner threads) -----------------------------------------
    def prepare(self, req: Request) -> None:
        """Exact pair counts and workspace bytes of the request alone: one
        device query on this thread's own stream."""
        torch = self.torch
        st = getattr(self._plan_streams, "s", None)
        if st is None:
            st = self._plan_streams.s = torch.cuda.Stream(self.device)
        with torch.cuda.stream(st):
            rend = self.api.Renderer([self.scenes[req.scene_id]], list(req.views), self.options)
            plan = rend.plan()
        views_c, _, _ = self.api._view_structs(list(req.views), [0] * req.nviews)
        req.plan_info = (int(plan.pairs_c), int(plan.pairs_i), views_c)
        req.cost = _plan_bytes(plan, req.want_grad)

    def _fused_plan(self, reqs: List[Request]):
        """Plan of a fused launch from the parts' counts (host only)."""
        C = self.C
        nv = sum(r.nviews for r in reqs)
        scenes = (C.Scene * len(reqs))(*[self._scene_c[r.scene_id] for r in reqs])
        views = (C.View * nv)()
        k, off = 0, 0
        for i, r in enumerate(reqs):
            for j in range(r.nviews):
                views[k] = r.plan_info[2][j]
                views[k].scene = i
                views[k].img_offset = off
                off += views[k].img_w * views[k].img_h
                k += 1
        pc = sum(r.plan_info[0] for r in reqs)
        pi = sum(r.plan_info[1] for r in reqs)
        plan = C.Plan()
        C.check(self.lib.sdgr_plan_host(scenes, len(reqs), views, nv, ctypes.byref(self.opts_c),
                                        pc, pi, ctypes.byref(plan)))
        return plan

    def batch_bytes(self, reqs: List[Request]) -> int:
        """Exact workspace bytes of the fused launch of `reqs`."""
        if len(reqs) == 1:
            return reqs[0].cost
        return _plan_bytes(self._fused_plan(reqs), any(r.want_grad for r in reqs))

    # -- launches (scheduler thread) ----------------------------------------
    def launch(self, batch_id: int, reqs: List[Request]) -> _Launch:
        torch = self.torch
        k = self.free_streams.pop()
        stream = self.streams[k]
        try:
            # inputs (resident scenes, targets) were made on the default stream
            stream.wait_stream(torch.cuda.default_stream(self.device))
            with torch.cuda.stream(stream):
                scenes = [self.scenes[r.scene_id] for r in reqs]
                views, ids = [], []
                for i, r in enumerate(reqs):
                    views.extend(r.views)
                    ids.extend([i] * r.nviews)
                rend = self.api.Renderer(scenes, views, self.options, scene_ids=ids)
                plan = rend.plan_for(sum(r.plan_info[0] for r in reqs),
                                     sum(r.plan_info[1] for r in reqs))
                res = rend.forward(plan)
                grads = None
                if any(r.want_grad for r in reqs):
                    G = torch.zeros_like(res.images)
                    v0 = 0
                    for r in reqs:
                        off0 = res.shapes[v0][0]
                        npx = r.pixels
                        if r.want_grad:
                            s = res.images[off0:off0 + npx]
                            G[off0:off0 + npx] = torch.sign(s - r.target.reshape(-1)) / npx
                        v0 += r.nviews
                    grads = rend.backward(res, G)
                done = torch.cuda.Event()
                done.record(stream)
            return _Launch(batch_id, reqs, _plan_bytes(plan, grads is not None),
                           (k, rend, res, grads, done))
        except Exception:
            self.free_streams.append(k)
            raise

    def done(self, launch: _Launch) -> bool:
        return launch.payload[4].query()

    def finish(self, launch: _Launch) -> List[Result]:
        k, rend, res, grads, done = launch.payload
        done.synchronize()
        self.free_streams.append(k)
        rend.status(res)     # a pair overflow would mean the counts were not additive
        out, v0 = [], 0
        for i, r in enumerate(launch.requests):
            imgs = [res.image(v0 + j) for j in range(r.nviews)]
            out.append(Result(r.id, imgs, grads[i] if (grads is not None and r.want_grad)
                              else None))
            v0 += r.nviews
        return out

    def abandon(self, launch: _Launch):
        k = launch.payload[0]
        launch.payload[4].synchronize()
        self.free_streams.append(k)


class FakeExecutor:
    """CPU stand-in: simulated memory, planning time and latency,
    deterministic results.

    cost(req) = bytes_per_view * views; a fused launch costs the sum plus
    batch_overhead per extra request; planning takes plan_s(req) seconds;
    latency_s(batch) = base_s + per_view_s * views; `fail_on(req)` may raise
    to simulate a failing launch."""

    def __init__(self, bytes_per_view=1 << 20, base_s=0.002, per_view_s=0.0005,
                 fail_on=None, slots=2, plan_s=None, batch_overhead=0):
        self.bytes_per_view = bytes_per_view
        self.base_s = base_s
        self.per_view_s = per_view_s
        self.fail_on = fail_on
        self.slots = slots
        self.free = slots
        self.plan_s = plan_s
        self.batch_overhead = batch_overhead
        self.launched: List[List[int]] = []
        self.planned: List[int] = []

    def prepare(self, req: Request) -> None:
        if self.plan_s is not None:
            time.sleep(self.plan_s(req))
        req.cost = req.nviews * self.bytes_per_view
        self.planned.append(req.id)

    def batch_bytes(self, reqs) -> int:
        return sum(r.cost for r in reqs) + self.batch_overhead * (len(reqs) - 1)

    def launch(self, batch_id, reqs):
        if self.fail_on is not None:
            for r in reqs:
                if self.fail_on(r):
                    raise RuntimeError(f"simulated launch failure (request {r.id})")
        self.free -= 1
        self.launched.append([r.id for r in reqs])
        views = sum(r.nviews for r in reqs)
        t_done = time.perf_counter() + self.base_s + self.per_view_s * views
        return _Launch(batch_id, reqs, self.batch_bytes(reqs), t_done)

    def done(self, launch):
        return time.perf_counter() >= launch.payload

    def finish(self, launch):
        while not self.done(launch):
            time.sleep(1e-4)
        self.free += 1
        return [Result(r.id, [("image", r.scene_id, j) for j in range(r.nviews)],
                       {"grad": r.id} if r.want_grad else None)
                for r in launch.requests]

    def abandon(self, launch):
        self.free += 1


class Server:
    """Scheduler loop around an executor.

    hbm_budget: bytes that in-flight launches may use together.
    max_views: views per fused launch. slots: launches in flight at once.
    batching=False gives the plain form: one request per launch, FIFO, one
    launch in flight.

    gc_freeze: move every object alive at construction (imported modules,
    resident scenes, whatever the caller built before) to the collector's
    permanent generation (``gc.freeze``). The collector's full passes run on
    whichever thread happens to allocate and hold the interpreter lock
    meanwhile; over the few hundred thousand objects a process with torch
    holds, one pass stalls the scheduler (and the planners) for 40-60 ms,
    which alone makes the latency tail. Frozen objects are never collected;
    the setting is process-wide and is not undone by close()."""

    def __init__(self, executor, hbm_budget: int, max_views: int = 64, slots: int = 2,
                 batching: bool = True, planners: int = 2, gc_freeze: bool = True):
        if gc_freeze:
            gc.collect()
            gc.freeze()
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_views = max_views if batching else 1 << 30
        self.slots = slots if batching else 1
        self.batching = batching
        self._pending = collections.deque()
        self._inflight: List[_Launch] = []
        self._used = 0
        self._ids = itertools.count()
        self._batches = itertools.count()
        self._futures: Dict[int, Future] = {}
        self._cv = threading.Condition()
        self._stop = False
        self.latencies: List[float] = []
        self.completed = 0
        self.failed = 0
        self.images_done = 0
        self.batch_sizes: List[int] = []
        self._plan_q: queue.Queue = queue.Queue()
        self._planning = 0
        self._planners = [threading.Thread(target=self._plan_loop, name=f"sdgr-planner-{k}",
                                           daemon=True) for k in range(max(1, planners))]
        for t in self._planners:
            t.start()
        self._thread = threading.Thread(target=self._loop, name="sdgr-server", daemon=True)
        self._thread.start()

    # ------------------------------------------------------------ client side
    def submit(self, req: Request) -> Future:
        """Queue a request; it is planned off the scheduler thread, then
        admitted. Returns a future of its Result."""
        fut: Future = Future()
        with self._cv:
            req.id = next(self._ids)
            req.arrival = time.perf_counter()
            self._futures[req.id] = fut
            self._planning += 1
        self._plan_q.put(req)
        return fut

    def close(self, wait=True):
        with self._cv:
            self._stop = True
            self._cv.notify()
        for _ in self._planners:
            self._plan_q.put(None)
        if wait:
            for t in self._planners:
                t.join()
            self._thread.join()

    # ------------------------------------------------------------- planners
    def _plan_loop(self):
        while True:
            req = self._plan_q.get()
            if req is None:
                return
            fut = self._futures.get(req.id)
            err = None
            if fut is not None and not fut.cancelled():
                try:
                    self.ex.prepare(req)
                    if req.cost > self.budget:
                        err = MemoryError(f"request {req.id} needs {req.cost} bytes, more "
                                          f"than the HBM budget of {self.budget}")
                except Exception as exc:   # a request that cannot be planned fails alone
                    err = exc
            with self._cv:
                self._planning -= 1
                if fut is None or fut.cancelled():
                    self._futures.pop(req.id, None)
                elif err is not None:
                    self._fail([req], err)
                else:
                    self._pending.append(req)
                self._cv.notify()

    def stats(self) -> dict:
        return {"completed": self.completed, "failed": self.failed,
                "p50_ms": percentile(self.latencies, 50) * 1e3,
                "p99_ms": percentile(self.latencies, 99) * 1e3,
                "images": self.images_done,
                "mean_batch_requests": (sum(self.batch_sizes) / len(self.batch_sizes)
                                        if self.batch_sizes else 0.0)}

    # ------------------------------------------------------------ scheduler
    def _admit(self) -> List[Request]:
        """Requests for the next launch (called with the lock held)."""
        batch, views, nbytes = [], 0, 0
        now = time.perf_counter()
        while self._pending:
            r = self._pending[0]
            fut = self._futures.get(r.id)
            if fut is None or fut.cancelled():
                self._pending.popleft()
                self._futures.pop(r.id, None)
                continue
            if r.deadline_s is not None and now - r.arrival > r.deadline_s:
                self._pending.popleft()
                self._fail([r], TimeoutError(f"request {r.id} not admitted within "
                                             f"{r.deadline_s} s"))
                continue
            if batch and views + r.nviews > self.max_views:
                break
            # the candidate batch's exact workspace bytes (a fused launch's
            # parameter-gradient parts grow with all of its Gaussians)
            need = self.ex.batch_bytes(batch + [r]) if batch else r.cost
            if self._used + need > self.budget:
                break                      # wait for memory to free up
            batch.append(self._pending.popleft())
            views += r.nviews
            if not self.batching:
                break
        return batch

    def _fail(self, reqs, exc):
        for r in reqs:
            fut = self._futures.pop(r.id, None)
            if fut is not None and not fut.done():
                fut.set_exception(exc)
                self.failed += 1

    def _launch(self, batch: List[Request]):
        bid = next(self._batches)
        try:
            launch = self.ex.launch(bid, batch)
        except Exception as exc:   # isolate the failing request(s)
            if len(batch) == 1:
                self._fail(batch, exc)
                return
            for r in batch:
                self._launch([r])
            return
        self._inflight.append(launch)
        self._used += launch.bytes
        self.batch_sizes.append(len(batch))

    def _retire(self, launch: _Launch):
        try:
            results = self.ex.finish(launch)
        except Exception as exc:
            self._fail(launch.requests, exc)
            results = []
        t = time.perf_counter()
        with self._cv:
            self._used -= launch.bytes
            for res, r in zip(results, launch.requests):
                res.latency_s = t - r.arrival
                res.batch_id = launch.batch_id
                res.batch_requests = len(launch.requests)
                self.latencies.append(res.latency_s)
                self.completed += 1
                self.images_done += r.nviews
                fut = self._futures.pop(r.id, None)
                if fut is not None and not fut.cancelled():
                    fut.set_result(res)

    def _loop(self):
        while True:
            # retire finished launches (oldest first)
            for launch in list(self._inflight):
                if self.ex.done(launch):
                    self._inflight.remove(launch)
                    self._retire(launch)
            with self._cv:
                if self._stop and not self._pending and not self._inflight and \
                        not self._planning:
                    return
                batch = []
                if len(self._inflight) < self.slots and self._pending:
                    batch = self._admit()
                if not batch:
                    if self._inflight:
                        pass
                    elif not self._stop:
                        self._cv.wait(timeout=0.01)
                        continue
            if batch:
                self._launch(batch)
            elif self._inflight:
                time.sleep(5e-5)
