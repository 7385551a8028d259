"""The reconstruction loop's kernels against the reference steps of
oracle.training (element by element), and a short end-to-end
reconstruction of a synthetic vehicle.

Bars: Adam parameters and moments within 1e-6 relative (FP32 against FP64
over five steps: each step's FP32 rounding ~6e-8 relative); densify and
prune decisions and output order exact (both sides decide in FP32), moments
copied or zeroed exactly, displaced centres within 1e-6 of the scene size;
nearest squared distances within 1e-5 relative (FP32 differences of
coordinates of size ~10); SSIM and PSNR within 1e-5 (FP32 window sums of
121 taps, accumulated in FP64 over positions)."""
import ctypes
import math

import numpy as np
import pytest
import torch

from oracle import training as T
from paper_2506_21633_amd import scenes

pytestmark = pytest.mark.gpu


def C():
    from paper_2506_21633_amd import _capi
    return _capi


def dev(a, cuda):
    return torch.as_tensor(np.ascontiguousarray(a, np.float32), device=cuda)


@pytest.mark.parametrize("log_space", [0, 1])
def test_adam_matches_reference(cuda, log_space):
    L = C().lib()
    rng = np.random.default_rng(700 + log_space)
    sizes = [1, 300, 4097]
    xs = [rng.uniform(0.1, 2.0, n) if log_space else rng.standard_normal(n) for n in sizes]
    lrs = [0.01, 0.003, 0.05]
    xd = [dev(x, cuda) for x in xs]
    md = [torch.zeros_like(t) for t in xd]
    vd = [torch.zeros_like(t) for t in xd]
    cfg = C().AdamConfig(0.9, 0.999, 1e-15, 0)
    # the reference takes the decay rates the kernel receives (FP32 values)
    rcfg = T.AdamConfig(beta1=float(np.float32(0.9)), beta2=float(np.float32(0.999)), eps=1e-15)
    host = lambda t: t.cpu().numpy().astype(np.float64)
    for t in range(1, 6):
        # the reference steps from the GPU's own FP32 state: each step is
        # compared on its own, the errors do not compound
        state = [(host(xd[k]), host(md[k]), host(vd[k])) for k in range(3)]
        gs = [rng.standard_normal(n).astype(np.float32) for n in sizes]
        gd = [dev(g, cuda) for g in gs]
        # the last group clamped: to [0.5, 1.5] in log space, [-1, 1] else
        lo, hi = (0.5, 1.5) if log_space else (-1.0, 1.0)
        bnd = [(0.0, 0.0), (0.0, 0.0), (lo, hi)]
        arr = (C().ParamGroup * 3)(*[
            C().ParamGroup(xd[k].data_ptr(), gd[k].data_ptr(), md[k].data_ptr(),
                           vd[k].data_ptr(), sizes[k], lrs[k], log_space, *bnd[k], 0)
            for k in range(3)])
        C().check(L.sdgr_adam_step(arr, 3, t, ctypes.byref(cfg), None))
        torch.cuda.synchronize()
        ref = [T.adam_step(*state[k][:1], gs[k], *state[k][1:], t, lrs[k], bool(log_space),
                           rcfg, *bnd[k]) for k in range(3)]
        for k in range(3):
            x, m, v = ref[k]
            # moments: FP32 rounding of terms of size |g| ~ 1 (cancellation in m)
            assert np.allclose(xd[k].cpu().numpy(), x, rtol=1e-6, atol=1e-6 * lrs[k]), (t, k)
            assert np.allclose(md[k].cpu().numpy(), m, rtol=1e-6, atol=1e-7), (t, k)
            assert np.allclose(vd[k].cpu().numpy(), v, rtol=1e-6, atol=1e-9), (t, k)


def _random_set(rng, n, shc=16, amp=True):
    p = dict(means=rng.uniform(-3, 3, (n, 3)),
             scales=np.exp(rng.uniform(np.log(0.01), np.log(0.6), (n, 3))),
             quats=rng.standard_normal((n, 4)),
             ext=np.exp(rng.uniform(np.log(1e-3), np.log(3.0), n)),
             sh=rng.standard_normal((n, shc)))
    if amp:
        p["amp"] = rng.uniform(0.1, 2.0, n)
    p = {k: v.astype(np.float32) for k, v in p.items()}
    mom = {k: (rng.standard_normal(v.shape).astype(np.float32),
               rng.uniform(0, 1, v.shape).astype(np.float32)) for k, v in p.items()}
    return p, mom


def _gpu_set(p, m, v):
    s = C().GaussianSet()
    for g in C().SET_GROUPS:
        if g in p:
            setattr(s, g, p[g].data_ptr())
            setattr(s, "m_" + g, m[g].data_ptr())
            setattr(s, "v_" + g, v[g].data_ptr())
    s.sh_coeffs = int(p["sh"].shape[1]) if "sh" in p else 0
    return s


@pytest.mark.parametrize("amp", [True, False])
def test_densify_matches_reference(cuda, amp):
    L = C().lib()
    rng = np.random.default_rng(710)
    n = 3000
    p, mom = _random_set(rng, n, amp=amp)
    cnt = rng.integers(0, 4, n).astype(np.float32)
    acc = (cnt * rng.uniform(0.0, 0.006, n)).astype(np.float32)
    gdir = rng.standard_normal((n, 3)).astype(np.float32)
    gdir[rng.random(n) < 0.05] = 0.0          # no direction: no displacement
    cfg = T.DensifyConfig(grad_threshold=0.003, split_scale=0.1, max_radius=1.2,
                          kappa_min=0.005, split_factor=1.6)
    ref, rmom, act = T.densify(p, mom, acc, cnt, gdir, cfg)
    assert len(set(act)) == 4   # every path taken
    pin = {k: dev(v, cuda) for k, v in p.items()}
    min_ = {k: dev(mom[k][0], cuda) for k in p}
    vin = {k: dev(mom[k][1], cuda) for k in p}
    cap = 2 * n
    pout = {k: torch.full((cap,) + v.shape[1:], float("nan"), device=cuda) for k, v in p.items()}
    mout = {k: torch.full_like(t, float("nan")) for k, t in pout.items()}
    vout = {k: torch.full_like(t, float("nan")) for k, t in pout.items()}
    wsb = L.sdgr_densify_workspace_bytes(n)
    ws = torch.empty(wsb, dtype=torch.uint8, device=cuda)
    n_out = torch.zeros(1, dtype=torch.int64, device=cuda)
    c = C().DensifyConfig(cfg.grad_threshold, cfg.split_scale, cfg.max_radius, cfg.kappa_min,
                          cfg.split_factor, 0)
    sin, sout = _gpu_set(pin, min_, vin), _gpu_set(pout, mout, vout)
    # the statistics stay referenced until the kernels have run
    acc_d, cnt_d, dir_d = dev(acc, cuda), dev(cnt, cuda), dev(gdir, cuda)
    C().check(L.sdgr_densify(ctypes.byref(sin), n, acc_d.data_ptr(), cnt_d.data_ptr(),
                             dir_d.data_ptr(), ctypes.byref(c), ctypes.byref(sout), cap,
                             n_out.data_ptr(), ws.data_ptr(), wsb, None))
    k = int(n_out.item())
    assert k == len(ref["means"])
    for name in p:
        got = pout[name][:k].cpu().numpy()
        if name == "means":
            assert np.allclose(got, ref[name], rtol=0, atol=1e-6 * 3.0), name
        elif name == "scales":
            assert np.allclose(got, ref[name], rtol=1e-6, atol=0), name
        else:   # copied
            assert np.array_equal(got, ref[name].astype(np.float32)), name
        assert np.array_equal(mout[name][:k].cpu().numpy(), rmom[name][0].astype(np.float32))
        assert np.array_equal(vout[name][:k].cpu().numpy(), rmom[name][1].astype(np.float32))


def test_densify_statistics(cuda):
    L = C().lib()
    rng = np.random.default_rng(720)
    n = 5000
    acc = torch.zeros(n, device=cuda)
    cnt = torch.zeros(n, device=cuda)
    dr = torch.zeros((n, 3), device=cuda)
    want_acc, want_cnt, want_dir = np.zeros(n), np.zeros(n), np.zeros((n, 3))
    for _ in range(4):
        g = rng.standard_normal((n, 3)).astype(np.float32)
        g[rng.random(n) < 0.3] = 0.0
        g_d = dev(g, cuda)
        C().check(L.sdgr_densify_stats(g_d.data_ptr(), n, acc.data_ptr(), cnt.data_ptr(),
                                       dr.data_ptr(), None))
        nz = np.linalg.norm(g.astype(np.float64), axis=1)
        want_acc += nz
        want_cnt += nz > 0
        want_dir += g
    assert np.allclose(acc.cpu().numpy(), want_acc, rtol=1e-6)
    assert np.array_equal(cnt.cpu().numpy(), want_cnt)
    assert np.allclose(dr.cpu().numpy(), want_dir, rtol=1e-6, atol=1e-6)


def test_point_metrics_match_reference(cuda):
    from paper_2506_21633_amd import train
    rng = np.random.default_rng(730)
    truth = rng.uniform(-3, 3, (5000, 3)).astype(np.float32)
    recon = (truth[:3500] + rng.normal(0, 0.1, (3500, 3))).astype(np.float32)
    recon = np.concatenate([recon, rng.uniform(-3, 3, (700, 3)).astype(np.float32)])
    got = train.point_metrics(dev(recon, cuda), dev(truth, cuda), tau=0.15)
    want = T.chamfer_f1(recon, truth, tau=0.15)
    for k in ("r2g", "g2r", "cd"):
        assert math.isclose(got[k], want[k], rel_tol=1e-5), k
    # a match decided within FP32 rounding of tau may differ
    for k in ("precision", "recall", "f1"):
        assert abs(got[k] - want[k]) <= 2.0 / 3500, k
    d2 = train.nearest_sq(dev(recon, cuda), dev(truth, cuda)).cpu().numpy()
    assert np.allclose(d2, T.nearest_sq(recon, truth), rtol=1e-5, atol=1e-6)


def test_image_metrics_match_reference(cuda):
    from paper_2506_21633_amd import train
    rng = np.random.default_rng(740)
    ref = rng.gamma(2.0, 1.0, (3, 24, 19)).astype(np.float32)
    img = (ref + rng.normal(0, 0.4, ref.shape)).astype(np.float32)
    img[2] = ref[2]                                    # identical: SSIM 1, PSNR inf
    L = float(ref.max())
    got = train.image_metrics(dev(img, cuda), dev(ref, cuda), L)
    for k in range(3):
        assert abs(got["ssim_per"][k] - T.ssim(img[k], ref[k], L)) <= 1e-5, k
    for k in range(2):
        assert abs(got["psnr_per"][k] - T.psnr(img[k], ref[k])) <= 1e-4, k
    assert got["psnr_per"][2] == np.inf


def test_short_reconstruction_improves(cuda):
    """A compressed schedule (600 iterations, SH degree + 1 every 150,
    densify every 50 from 150 to 450) on the synthetic vehicle: the loss,
    the Chamfer distance and F1 improve on the hemispherical start, and
    densification changes the Gaussian count."""
    from paper_2506_21633_amd import api, train
    gt = scenes.vehicle(909, 6000)
    gt_sh = gt.copy()
    gt_sh.sh = (gt.amp / (0.5 / math.sqrt(math.pi)))[:, None].astype(np.float32)
    views = scenes.reconstruction_views(48, 0.25)
    r = api.Renderer([api.GaussianTensors.from_numpy(gt, cuda)], views)
    targets = r.forward().stacked().clone()
    init = scenes.hemisphere_init(3000, 3.5, seed=910, center=(0.0, 0.0, -1.25))
    cfg = train.TrainConfig(iterations=600, sh_every=150, densify_from=150,
                            densify_until=450, densify_every=50)
    rec = train.Reconstruction(init, views, targets, cfg, device=cuda)
    truth = torch.as_tensor(gt.means, device=cuda)
    before = train.point_metrics(rec.p["means"], truth, tau=0.25)
    l0 = rec.loss()
    rec.run()
    l1 = rec.loss()
    after = train.point_metrics(rec.p["means"], truth, tau=0.25)
    print(f"\nloss {l0:.4g} -> {l1:.4g}, n {init.n} -> {rec.n}, densify calls "
          f"{rec.densify_calls}, cd {before['cd']:.4g} -> {after['cd']:.4g}, "
          f"f1 {before['f1']:.3f} -> {after['f1']:.3f}")
    assert rec.densify_calls == 6 and rec.n != init.n
    assert torch.isfinite(rec.p["means"]).all() and (rec.p["scales"] > 0).all()
    assert l1 < 0.6 * l0
    assert after["cd"] < 0.5 * before["cd"] and after["f1"] > before["f1"]
