"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances (FP32 kernels against the FP64 oracle):
  images      max |S_gpu - S_ref| / max |S_ref| <= 1e-4
  A (shares)  relative L2 <= 1e-4
  gradients   per parameter group cosine >= 0.9999, relative L2 <= 1e-3
The FP32 error budget behind them: every footprint and attenuation term is
evaluated in FP32 with the hardware exp2 (relative error ~1e-7 per term),
sums over up to ~1e3 terms per pixel, and the early ray termination at
optical depth 16 drops terms below exp(-16) ~ 1.1e-7 of the incident
intensity.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2506_21633_amd import scenes

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-4
A_TOL = 1e-4
GRAD_COS = 0.9999
GRAD_L2 = 1e-3
GROUPS = ("means", "scales", "quats", "amp", "ext")


def api():
    from paper_2506_21633_amd import api as _api
    return _api


def img_err(a, ref):
    return float(np.abs(a - ref).max() / max(np.abs(ref).max(), 1e-30))


def rel_l2(a, ref):
    return float(np.linalg.norm((a - ref).ravel()) / max(np.linalg.norm(ref.ravel()), 1e-30))


def cosine(a, b):
    a, b = a.ravel().astype(np.float64), b.ravel().astype(np.float64)
    return float(a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-300))


def gpu_run(scene, views, options=None, G=None, cuda="cuda"):
    A_ = api()
    g = A_.GaussianTensors.from_numpy(scene, cuda)
    r = A_.Renderer([g], views, options or A_.RenderOptions())
    res = r.forward()
    out = dict(images=[res.image(v).cpu().numpy() for v in range(len(views))],
               A=r.intensity_shares(res).cpu().numpy().reshape(len(views), scene.n),
               tau=r.optical_depth(res).cpu().numpy(), plan=res.plan)
    if G is not None:
        flat = np.concatenate([np.asarray(x, np.float32).ravel() for x in G])
        d = r.backward(res, torch.as_tensor(flat, device=cuda))[0]
        out["grads"] = {k: v.cpu().numpy() for k, v in d.items()}
    torch.cuda.synchronize()
    r.status(res)
    return out


def check_forward(scene, views, out, shadowing=True):
    A_ref, _, S_ref = oracle.forward(scene, views, shadowing=shadowing)
    for v in range(len(views)):
        e = img_err(out["images"][v], S_ref[v])
        assert e <= IMG_TOL, (v, e)
    assert rel_l2(out["A"], A_ref) <= A_TOL
    return A_ref, S_ref


def check_grads(scene, views, G, out, shadowing=True):
    ref, _ = oracle.backward(scene, views, G, shadowing=shadowing)
    for k in GROUPS:
        c, l2 = cosine(out["grads"][k], ref[k]), rel_l2(out["grads"][k], ref[k])
        assert c >= GRAD_COS and l2 <= GRAD_L2, (k, c, l2)


# ------------------------------------------------------------------ forward

def test_fwd_1k_forward_parity(cuda):
    sc, views = scenes.fwd_1k()
    out = gpu_run(sc, views)
    check_forward(sc, views, out)
    assert out["plan"].pairs_c > 0 and out["plan"].pairs_i > 0


def test_fwd_1k_no_shadowing_and_full_optical_depth(cuda):
    sc, views = scenes.fwd_1k()
    A_ = api()
    out = gpu_run(sc, views, A_.RenderOptions(shadowing=False))
    check_forward(sc, views, out, shadowing=False)
    out = gpu_run(sc, views, A_.RenderOptions(tau_max=0.0))
    _, tau_ref, _ = oracle.forward(sc, views)
    assert rel_l2(out["tau"], tau_ref[0].ravel()) <= 1e-5


def _small_scene(seed, n=300, half=1.5, smin=0.04, smax=0.2):
    rng = scenes.make_rng(seed)
    return scenes.Scene(rng.uniform(-half, half, (n, 3)).astype(np.float32),
                        np.exp(rng.uniform(np.log(smin), np.log(smax), (n, 3))).astype(np.float32),
                        scenes.random_quats(rng, n),
                        rng.uniform(0.2, 1.0, n).astype(np.float32),
                        rng.uniform(1.0, 4.0, n).astype(np.float32))


def test_ragged_sizes_and_custom_computation_grid(cuda):
    sc = _small_scene(7)
    views = [scenes.View(azimuth=0.3, grazing=math.radians(50), img_w=37, img_h=29,
                         d_az=0.11, d_rg=0.12, comp_w=41, comp_h=23, comp_d_az=0.09,
                         comp_d_el=0.2),
             scenes.View.from_degrees(123.0, 30.0, 64, 0.1),
             scenes.View(azimuth=-2.0, grazing=math.radians(20), img_w=16, img_h=80,
                         d_az=0.2, d_rg=0.05)]
    out = gpu_run(sc, views)
    check_forward(sc, views, out)


@pytest.mark.parametrize("deterministic", [False, True])
@pytest.mark.parametrize("plane", ["computation", "imaging"])
def test_pair_overflow_is_reported_and_recovered(cuda, plane, deterministic):
    """A plan with too few pairs on one plane: the kernels clamp to empty
    lists, sdgr_status reports SDGR_EOVERFLOW and the asynchronous check sets
    its device flag; the exact plan then renders as the oracle does and
    leaves a fresh flag clear."""
    import ctypes
    A_ = api()
    from paper_2506_21633_amd import _capi as C
    sc = _small_scene(31)
    views = [scenes.View.from_degrees(20.0, 45.0, 64, 0.06),
             scenes.View.from_degrees(200.0, 30.0, 48, 0.06)]
    r = A_.Renderer([A_.GaussianTensors.from_numpy(sc, cuda)], views,
                    A_.RenderOptions(deterministic=deterministic))
    exact = r.plan()
    small = C.Plan()
    ctypes.pointer(small)[0] = exact
    pc, pi = (exact.pairs_c // 2, exact.pairs_i) if plane == "computation" else \
        (exact.pairs_c, exact.pairs_i // 2)
    C.check(C.lib().sdgr_plan_resize(ctypes.byref(small), pc, pi))
    flags = torch.zeros(1, dtype=torch.int32, device=cuda)
    res = r.forward(small)
    r.backward(res, torch.ones_like(res.images))
    r.status_into(res, flags)
    torch.cuda.synchronize()
    assert int(flags.item()) != 0
    with pytest.raises(C.SDGRError) as err:
        r.status(res)
    assert err.value.code == C.SDGR_EOVERFLOW
    ok = r.forward(exact)
    clear = torch.zeros(1, dtype=torch.int32, device=cuda)
    r.status_into(ok, clear)
    torch.cuda.synchronize()
    assert int(clear.item()) == 0
    r.status(ok)
    _, _, S_ref = oracle.forward(sc, views)
    for v in range(len(views)):
        assert img_err(ok.image(v).cpu().numpy(), S_ref[v]) <= IMG_TOL


def test_tiny_and_one_pixel_images(cuda):
    sc = _small_scene(8, n=50, half=0.2)
    views = [scenes.View(azimuth=0.0, grazing=0.7, img_w=1, img_h=1, d_az=0.1, d_rg=0.1),
             scenes.View(azimuth=1.0, grazing=0.7, img_w=3, img_h=9, d_az=0.1, d_rg=0.1)]
    out = gpu_run(sc, views)
    check_forward(sc, views, out)


def test_empty_outside_and_degenerate_gaussians(cuda):
    v = [scenes.View.from_degrees(10.0, 40.0, 32, 0.1)]
    empty = scenes.Scene(*(np.zeros((0,) + s, np.float32) for s in ((3,), (3,), (4,), (), ())))
    out = gpu_run(empty, v)
    assert np.all(out["images"][0] == 0)
    far = _small_scene(9, n=40)
    far.means[:, 0] += 500.0
    out = gpu_run(far, v)
    assert np.all(out["images"][0] == 0) and np.all(out["A"] == 0)
    sc = _small_scene(10, n=100, half=0.8)
    bad = sc.subset(slice(0, 3))
    bad.quats[0] = 0.0
    bad.scales[1, 2] = -0.1
    bad.means[2, 1] = np.nan
    both = sc.concat(bad)
    out_a = gpu_run(sc, v)
    out_b = gpu_run(both, v)
    assert img_err(out_b["images"][0], out_a["images"][0]) <= 1e-6
    assert np.all(out_b["A"][0, -3:] == 0)


def test_more_views_than_view_major_keys(cuda):
    """Above 256 views the imaging-plane bucket keys are global tile ids
    (two sort passes) instead of (tile within the view, view)."""
    sc = _small_scene(18, n=60, half=0.6)
    views = [scenes.View.from_degrees(1.5 * k, 30.0 + (k % 7), 16 + (k % 3) * 4, 0.1)
             for k in range(260)]
    rng = scenes.make_rng(19)
    G = [rng.standard_normal((v.img_h, v.img_w)) for v in views]
    out = gpu_run(sc, views, G=G)
    check_forward(sc, views, out)
    check_grads(sc, views, G, out)


def test_views_of_an_empty_scene_between_others(cuda):
    """Several scenes in one launch, with views of an empty scene between
    views of non-empty ones: the per-view segments of the depth and pair
    sorts include empty ones."""
    A_ = api()
    sc = [_small_scene(20, n=200),
          scenes.Scene(*(np.zeros((0,) + s, np.float32) for s in ((3,), (3,), (4,), (), ()))),
          _small_scene(21, n=150, half=1.0)]
    which = [0, 1, 1, 2, 1, 0, 2]
    views = [scenes.View.from_degrees(25.0 * k, 35.0 + 2 * k, 32 + 4 * (k % 2), 0.1, scene=s)
             for k, s in enumerate(which)]
    rng = scenes.make_rng(22)
    G = [rng.standard_normal((v.img_h, v.img_w)) for v in views]
    r = A_.Renderer([A_.GaussianTensors.from_numpy(x, cuda) for x in sc], views)
    res = r.forward()
    flat = np.concatenate([g.astype(np.float32).ravel() for g in G])
    grads = r.backward(res, torch.as_tensor(flat, device=cuda))
    torch.cuda.synchronize()
    r.status(res)
    for k, v in enumerate(views):
        img = res.image(k).cpu().numpy()
        if which[k] == 1:
            assert np.all(img == 0)
            continue
        S_ref = oracle.forward_view(sc[which[k]], v)[2]
        assert img_err(img, S_ref) <= IMG_TOL, k
    for s in (0, 2):
        vs = [v for v in views if v.scene == s]
        gs = [G[k] for k, v in enumerate(views) if v.scene == s]
        ref, _ = oracle.backward(sc[s], vs, gs)
        for k in GROUPS:
            g = grads[s][k].cpu().numpy()
            assert cosine(g, ref[k]) >= GRAD_COS and rel_l2(g, ref[k]) <= GRAD_L2, (s, k)


def test_permutation_invariance(cuda):
    sc = _small_scene(11, n=400)
    views = scenes.vehicle_views(48, 0.1, count=3, step=40.0)
    out = gpu_run(sc, views)
    perm = scenes.make_rng(1).permutation(sc.n)
    out_p = gpu_run(sc.subset(perm), views)
    for v in range(3):
        assert img_err(out_p["images"][v], out["images"][v]) <= 1e-5
    assert rel_l2(out_p["A"], out["A"][:, perm]) <= 1e-5


def test_repeat_runs_agree(cuda):
    sc = _small_scene(12, n=500)
    views = scenes.vehicle_views(48, 0.1, count=4, step=30.0)
    a, b = gpu_run(sc, views), gpu_run(sc, views)
    for v in range(4):
        assert img_err(a["images"][v], b["images"][v]) <= 1e-6


# ------------------------------------------------------------------ backward

@pytest.mark.parametrize("shadowing", [True, False])
def test_gradient_parity_small(cuda, shadowing):
    sc = _small_scene(13, n=300)
    views = [scenes.View.from_degrees(20.0, 40.0, 40, 0.1),
             scenes.View(azimuth=2.0, grazing=0.5, img_w=33, img_h=27, d_az=0.12, d_rg=0.1)]
    rng = scenes.make_rng(14)
    G = [rng.standard_normal((v.img_h, v.img_w)) for v in views]
    A_ = api()
    out = gpu_run(sc, views, A_.RenderOptions(shadowing=shadowing), G=G)
    check_forward(sc, views, out, shadowing=shadowing)
    check_grads(sc, views, G, out, shadowing=shadowing)


def test_building_subset_forward_backward(cuda):
    sc = scenes.building(202, n=6000)
    views = scenes.building_views(64, 0.3, step=120.0)
    target = scenes.jitter(sc, 203)
    S_t = [s for s in oracle.forward(target, views)[2]]
    _, _, S = oracle.forward(sc, views)
    G = [np.sign(S[v] - S_t[v]) / (len(views) * 64 * 64) for v in range(len(views))]
    out = gpu_run(sc, views, G=G)
    check_forward(sc, views, out)
    check_grads(sc, views, G, out)


def test_recompute_mode_matches(cuda):
    sc = _small_scene(15, n=300)
    views = scenes.vehicle_views(40, 0.1, count=3, step=50.0)
    rng = scenes.make_rng(16)
    G = [rng.standard_normal((40, 40)) for _ in views]
    A_ = api()
    a = gpu_run(sc, views, A_.RenderOptions(recompute=False), G=G)
    b = gpu_run(sc, views, A_.RenderOptions(recompute=True), G=G)
    assert b["plan"].state_bytes < a["plan"].state_bytes
    for v in range(3):
        assert img_err(b["images"][v], a["images"][v]) <= 1e-6
    for k in GROUPS:
        assert rel_l2(b["grads"][k], a["grads"][k]) <= 1e-5, k


def test_autograd_function_matches_renderer(cuda):
    A_ = api()
    sc = _small_scene(17, n=200)
    views = scenes.vehicle_views(32, 0.1, count=2, step=90.0)
    t = {k: torch.tensor(getattr(sc, k), device=cuda, requires_grad=True) for k in GROUPS}
    imgs = A_.render(t["means"], t["scales"], t["quats"], t["amp"], t["ext"], views)
    assert imgs.shape == (2, 32, 32)
    w = torch.randn(imgs.shape, device=cuda, generator=torch.Generator(cuda).manual_seed(0))
    (imgs * w).sum().backward()
    G = [w[k].cpu().numpy() for k in range(2)]
    ref, _ = oracle.backward(sc, views, G)
    for k in GROUPS:
        g = t[k].grad.cpu().numpy()
        assert cosine(g, ref[k]) >= GRAD_COS and rel_l2(g, ref[k]) <= GRAD_L2, k


# ------------------------------------------------- full size, sampled outputs

@pytest.fixture(scope="module")
def vehicle_full():
    return scenes.vehicle(303, 200_000), scenes.vehicle_views()


def test_vehicle_200k_72_views_sampled_parity(cuda, vehicle_full):
    """The benchmark's launch (200k Gaussians, 72 views of 256x256 in one
    call), checked at sampled pixels and Gaussians of two views against the
    oracle's sampled mode."""
    sc, views = vehicle_full
    out = gpu_run(sc, views)
    rng = scenes.make_rng(304)
    for v in (0, 37):
        img = out["images"][v]
        hot = np.flatnonzero(img.ravel() > 0.05 * img.max())
        pix = np.concatenate([rng.choice(hot, 24, replace=False),
                              rng.choice(img.size, 8, replace=False)])
        gids = rng.choice(sc.n, 32, replace=False)
        S_ref, A_ref = oracle.sparse_forward(sc, views[v], pix, gids)
        assert np.abs(img.ravel()[pix] - S_ref).max() <= IMG_TOL * img.max()
        a = out["A"][v, gids]
        assert np.abs(a - A_ref).max() <= A_TOL * max(out["A"][v].max(), 1e-30)


def test_vehicle_200k_gradient_properties(cuda, vehicle_full):
    """At full size: L = <W, S> is linear in the amplitudes P (A does not
    depend on P), so dL/dP must predict L(P + d) - L(P) to FP32 accuracy."""
    A_ = api()
    sc, views = vehicle_full
    views = views[:8]
    rng = scenes.make_rng(305)
    W = [rng.standard_normal((256, 256)).astype(np.float32) for _ in views]
    base = gpu_run(sc, views, G=W)
    L0 = sum(float((base["images"][v] * W[v]).sum(dtype=np.float64)) for v in range(8))
    d = rng.uniform(0.0, 0.05, sc.n).astype(np.float32)
    sp = sc.copy()
    sp.amp = sc.amp + d
    L1 = sum(float((x * W[v]).sum(dtype=np.float64))
             for v, x in enumerate(gpu_run(sp, views)["images"]))
    pred = float(base["grads"]["amp"].astype(np.float64) @ d)
    assert abs((L1 - L0) - pred) <= 1e-3 * abs(pred)
