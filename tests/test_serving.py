"""Scheduler tests of the continuous-batching server on the CPU (fake
executor with simulated memory and latency), and on the GPU: every request's
result is the same alone and in a fused mix."""
import math
import time
from types import SimpleNamespace

import numpy as np
import pytest

from paper_2506_21633_amd import scenes
from paper_2506_21633_amd.serve import FakeExecutor, Request, Server, percentile


def views(k, size=64):
    return [scenes.View.from_degrees(10.0 * i, 30.0, size, 0.1) for i in range(k)]


def test_requests_arriving_during_a_launch_are_batched_when_a_slot_frees():
    ex = FakeExecutor(base_s=0.05, per_view_s=0.0)
    srv = Server(ex, hbm_budget=1 << 40, max_views=64, slots=1)
    first = srv.submit(Request("a", views(1)))
    time.sleep(0.01)                       # the first launch is now running
    later = [srv.submit(Request("b", views(2))) for _ in range(5)]
    results = [f.result(timeout=5) for f in [first] + later]
    srv.close()
    assert ex.launched[0] == [0]
    assert ex.launched[1] == [1, 2, 3, 4, 5]          # admitted together
    assert {r.batch_requests for r in results[1:]} == {5}


def test_two_slots_overlap_launches():
    ex = FakeExecutor(base_s=0.05, per_view_s=0.0)
    srv = Server(ex, hbm_budget=1 << 40, slots=2)
    t0 = time.perf_counter()
    f1 = srv.submit(Request("a", views(1)))
    time.sleep(0.005)
    f2 = srv.submit(Request("b", views(1)))
    f1.result(5), f2.result(5)
    srv.close()
    assert time.perf_counter() - t0 < 0.095           # not serialised
    assert len(ex.launched) == 2


def test_gc_freeze_moves_existing_objects_out_of_the_collectors_passes():
    import gc
    before = gc.get_freeze_count()
    srv = Server(FakeExecutor(base_s=0.0), hbm_budget=1 << 40, gc_freeze=False)
    srv.close()
    assert gc.get_freeze_count() == before
    keep = [[i] for i in range(1000)]                 # tracked containers alive now
    srv = Server(FakeExecutor(base_s=0.0), hbm_budget=1 << 40)
    assert gc.get_freeze_count() >= before + len(keep)
    assert srv.submit(Request("a", views(1))).result(5).images
    srv.close()


def test_hbm_budget_limits_batches():
    ex = FakeExecutor(bytes_per_view=100, base_s=0.02, per_view_s=0.0)
    srv = Server(ex, hbm_budget=350, max_views=64, slots=1)
    futs = [srv.submit(Request("a", views(1))) for _ in range(7)]
    for f in futs:
        f.result(5)
    srv.close()
    assert max(len(b) for b in ex.launched) <= 3
    assert sum(len(b) for b in ex.launched) == 7


def test_view_cap_limits_batches():
    ex = FakeExecutor(base_s=0.02)
    srv = Server(ex, hbm_budget=1 << 40, max_views=8, slots=1)
    futs = [srv.submit(Request("a", views(3))) for _ in range(6)]
    for f in futs:
        f.result(5)
    srv.close()
    assert all(sum(3 for _ in b) <= 8 for b in ex.launched[1:])


def test_request_larger_than_budget_is_rejected():
    ex = FakeExecutor(bytes_per_view=1000)
    srv = Server(ex, hbm_budget=500)
    f = srv.submit(Request("a", views(1)))
    with pytest.raises(MemoryError):
        f.result(1)
    ok = Server(FakeExecutor(bytes_per_view=1), hbm_budget=500)
    assert ok.submit(Request("a", views(1))).result(5).images
    srv.close()
    ok.close()


def test_failing_request_is_isolated_and_serving_continues():
    ex = FakeExecutor(base_s=0.02, fail_on=lambda r: r.id == 3)
    srv = Server(ex, hbm_budget=1 << 40, slots=1)
    futs = [srv.submit(Request("a", views(1))) for _ in range(6)]
    outcomes = []
    for f in futs:
        try:
            f.result(5)
            outcomes.append("ok")
        except RuntimeError:
            outcomes.append("fail")
    later = srv.submit(Request("a", views(1))).result(5)
    srv.close()
    assert outcomes == ["ok", "ok", "ok", "fail", "ok", "ok"]
    assert later.images and srv.stats()["failed"] == 1


def test_cancel_and_deadline():
    ex = FakeExecutor(base_s=0.1, per_view_s=0.0)
    srv = Server(ex, hbm_budget=1 << 40, slots=1)
    busy = srv.submit(Request("a", views(1)))
    time.sleep(0.01)
    cancelled = srv.submit(Request("b", views(1)))
    assert cancelled.cancel()
    late = srv.submit(Request("c", views(1), deadline_s=0.01))
    busy.result(5)
    with pytest.raises(TimeoutError):
        late.result(5)
    srv.close()
    assert all(0 not in b or b == [0] for b in ex.launched)
    assert not any(1 in b for b in ex.launched)


def test_slow_planning_does_not_hold_up_planned_requests():
    """Requests are planned on planner threads: a request whose plan takes
    long is overtaken by later ones, and launches keep flowing meanwhile."""
    ex = FakeExecutor(base_s=0.005, per_view_s=0.0,
                      plan_s=lambda r: 0.3 if r.scene_id == "slow" else 0.0)
    srv = Server(ex, hbm_budget=1 << 40, slots=1, planners=2)
    slow = srv.submit(Request("slow", views(1)))
    time.sleep(0.01)
    fast = [srv.submit(Request("fast", views(1))) for _ in range(3)]
    t_fast = []
    for f in fast:
        f.result(5)
        t_fast.append(time.perf_counter())
    slow.result(5)
    t_slow = time.perf_counter()
    srv.close()
    assert max(t_fast) < t_slow
    assert ex.launched[-1] == [0]          # the slow request launched last


def test_admission_uses_the_batch_bytes():
    """The fused launch may cost more than the sum of its parts (here 100
    bytes per extra request): admission checks the batch's own bytes."""
    ex = FakeExecutor(bytes_per_view=100, base_s=0.05, per_view_s=0.0, batch_overhead=100)
    srv = Server(ex, hbm_budget=500, max_views=64, slots=1)
    blocker = srv.submit(Request("a", views(1)))
    time.sleep(0.01)                       # the blocker runs; the rest queue up
    futs = [srv.submit(Request("b", views(1))) for _ in range(6)]
    for f in [blocker] + futs:
        f.result(5)
    srv.close()
    # 3 requests cost 300 + 200 = 500 (fits), 4 would cost 400 + 300 = 700
    assert max(len(b) for b in ex.launched) == 3


def test_poisson_stream_served_vs_plain():
    """Under load, batching amortises the per-launch cost: fewer launches and
    lower tail latency than one request per launch."""
    rng = np.random.default_rng(0)
    arrivals = np.cumsum(rng.exponential(1 / 400.0, 80))
    sizes = rng.integers(1, 5, 80)

    def run(batching):
        ex = FakeExecutor(base_s=0.004, per_view_s=0.0002)
        srv = Server(ex, hbm_budget=1 << 40, max_views=64, slots=2, batching=batching)
        t0 = time.perf_counter()
        futs = []
        for a, k in zip(arrivals, sizes):
            while time.perf_counter() - t0 < a:
                time.sleep(1e-4)
            futs.append(srv.submit(Request("s", views(int(k)))))
        lat = [f.result(30).latency_s for f in futs]
        srv.close()
        return lat, len(ex.launched)

    lat_b, n_b = run(True)
    lat_p, n_p = run(False)
    assert n_p == 80 and n_b < n_p
    assert percentile(lat_b, 99) < percentile(lat_p, 99)
    assert percentile(lat_b, 50) <= percentile(lat_b, 99)


# -------------------------------------------------------------------- GPU

@pytest.mark.gpu
def test_served_results_equal_plain_results(cuda):
    import torch
    from paper_2506_21633_amd import api
    from paper_2506_21633_amd.serve import GpuExecutor
    res_scenes = {"v0": scenes.vehicle(11, 20_000), "v1": scenes.vehicle(12, 60_000),
                  "v2": scenes.vehicle(13, 5_000)}
    dev_scenes = {k: api.GaussianTensors.from_numpy(s, cuda) for k, s in res_scenes.items()}
    rng = np.random.default_rng(3)
    reqs = []
    for i in range(9):
        sid = f"v{i % 3}"
        size = [64, 128, 96][i % 3]
        vs = [scenes.View.from_degrees(float(rng.uniform(0, 360)), [30.0, 45.0][j % 2], size, 0.1)
              for j in range(1 + i % 4)]
        want = i % 2 == 1
        tgt = torch.rand(sum(v.img_w * v.img_h for v in vs), device=cuda) if want else None
        reqs.append((sid, vs, want, tgt))
    ex = GpuExecutor(dev_scenes, cuda)
    # a fused launch's plan built on the host from its parts' exact counts
    # equals the plan the device query gives for the fused problem
    parts = [Request(sid, vs, want, tgt) for sid, vs, want, tgt in reqs[:5]]
    for r in parts:
        ex.prepare(r)
    fused = api.Renderer([dev_scenes[r.scene_id] for r in parts],
                         [v for r in parts for v in r.views],
                         scene_ids=[i for i, r in enumerate(parts) for _ in r.views])
    queried, host = fused.plan(), ex._fused_plan(parts)
    for name, _ in type(host)._fields_:
        assert getattr(host, name) == getattr(queried, name), name
    srv = Server(ex, hbm_budget=8 << 30, max_views=64, slots=2)
    futs = [srv.submit(Request(sid, vs, want, tgt)) for sid, vs, want, tgt in reqs]
    served = [f.result(120) for f in futs]
    srv.close()
    assert max(r.batch_requests for r in served) > 1           # really mixed
    for (sid, vs, want, tgt), got in zip(reqs, served):
        r = api.Renderer([dev_scenes[sid]], vs)
        res = r.forward()
        for v in range(len(vs)):
            ref = res.image(v)
            err = float((got.images[v] - ref).abs().max() / ref.abs().max().clamp_min(1e-30))
            assert err <= 1e-5, (sid, v, err)
        if want:
            npx = sum(v.img_w * v.img_h for v in vs)
            G = torch.sign(res.images[:npx] - tgt) / npx
            full = torch.zeros_like(res.images)
            full[:npx] = G
            ref_g = r.backward(res, full)[0]
            for k, t in ref_g.items():
                a, b = got.grads[k].double().flatten(), t.double().flatten()
                cos = float(a @ b / (a.norm() * b.norm()).clamp_min(1e-300))
                assert cos >= 0.9999, (sid, k, cos)
        else:
            assert got.grads is None
