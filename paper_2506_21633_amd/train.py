"""Reconstruction of a Gaussian scene from SAR images (Sec. III-B) on the
library: each iteration renders a batch of training views forward and
backward (sdgr_forward / sdgr_backward), takes the L1 loss's cotangent, and
steps every parameter array with one fused Adam launch (sdgr_adam_step);
between densify_from and densify_until it accumulates the position-gradient
statistics (sdgr_densify_stats) and every densify_every iterations densifies
and prunes (sdgr_densify, Sec. II-B). The SH degree of the phase function
rises by one every sh_every iterations up to sh_max. Evaluation renders
held-out views and compares them with the ground truth's (sdgr_image_metrics:
SSIM, PSNR) and the Gaussians' centres with the ground-truth point cloud
(sdgr_nearest_sq: Chamfer distance, precision, recall, F1).

PyTorch supplies device memory, the stream and the loss's elementwise sign;
every other step is a library kernel.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

from . import _capi as C
from . import api

__all__ = ["TrainConfig", "Reconstruction", "image_metrics", "point_metrics"]


@dataclass
class TrainConfig:
    iterations: int = 30_000
    batch_views: int = 8
    # learning rates; the means' decays exponentially from lr_means to
    # lr_means_final (both times the scene extent). The paper gives none; on
    # the synthetic SAR set a step 25x the usual camera-scene default moves
    # the initial shell onto the target within the schedule
    lr_means: float = 4e-3
    lr_means_final: float = 4e-5
    lr_scales: float = 5e-3          # log space
    lr_quats: float = 1e-3
    lr_ext: float = 5e-2             # log space
    lr_sh: float = 2.5e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-15
    sh_every: int = 2_500            # SH degree + 1 every sh_every iterations
    sh_max: int = 3
    densify_from: int = 10_000
    densify_until: int = 25_000
    densify_every: int = 100
    grad_threshold: float = 0.003
    max_radius_frac: float = 0.3     # of the illumination range
    split_frac: float = 0.01         # of the extent: larger std splits
    kappa_min: float = 0.005
    split_factor: float = 1.6
    # bounds after each step of the positive parameters (stepped in log
    # space, which bounds neither): an extinction of 50 is opaque already
    ext_bounds: tuple = (1e-6, 50.0)
    scale_bounds: tuple = (1e-5, 1e3)
    seed: int = 0


def _ptr(t: Optional[torch.Tensor]) -> int:
    return 0 if t is None else t.data_ptr()


def _stream(dev) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


GROUPS = ("means", "scales", "quats", "ext", "sh")
LOG_SPACE = {"scales": 1, "ext": 1}


class Reconstruction:
    """Fits Gaussians (means, scales, quats, ext, sh [n, 16]) to target
    images of `views` (torch [V, H, W] on the device, one image size)."""

    def __init__(self, init, views, targets: torch.Tensor, cfg: TrainConfig = TrainConfig(),
                 options: Optional[api.RenderOptions] = None, device="cuda"):
        self.cfg = cfg
        self.dev = torch.device(device)
        self.lib = C.lib()
        self.views = list(views)
        self.options = options or api.RenderOptions()
        V, H, W = targets.shape
        if V != len(self.views) or any(v.img_w != W or v.img_h != H for v in self.views):
            raise ValueError("targets must be [V, H, W] matching the views")
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=self.dev)
        sh = getattr(init, "sh", None)
        if sh is None or sh.shape[1] != 16:
            raise ValueError("the initial scene needs sh with 16 coefficients")
        self.p = {"means": f(init.means), "scales": f(init.scales), "quats": f(init.quats),
                  "ext": f(init.ext), "sh": f(sh)}
        self.m = {k: torch.zeros_like(t) for k, t in self.p.items()}
        self.v = {k: torch.zeros_like(t) for k, t in self.p.items()}
        self._reset_stats()
        # the scene's extent and the radar's illumination range (image side)
        self.illum = max(max(v.img_w * v.d_az, v.img_h * v.d_rg) for v in self.views)
        self.extent = 0.5 * self.illum
        # fixed batches of views, visited in a seeded order each epoch
        rng = np.random.default_rng(cfg.seed)
        order = rng.permutation(len(self.views))
        B = min(cfg.batch_views, len(self.views))
        self.batches = [order[k:k + B] for k in range(0, len(order), B)]
        self.targets = [targets[b].reshape(-1).contiguous() for b in self.batches]
        self.renderers = [None] * len(self.batches)
        self.rng = rng
        self.epoch_order = []
        self.it = 0
        self.sh_active = 0
        self.history = []
        self.adam_cfg = C.AdamConfig(cfg.beta1, cfg.beta2, cfg.eps, 0)
        self.densify_calls = 0

    # ------------------------------------------------------------ state
    @property
    def n(self) -> int:
        return int(self.p["means"].shape[0])

    def _reset_stats(self):
        n = self.p["means"].shape[0]
        self.acc = torch.zeros(n, dtype=torch.float32, device=self.dev)
        self.cnt = torch.zeros(n, dtype=torch.float32, device=self.dev)
        self.dir = torch.zeros((n, 3), dtype=torch.float32, device=self.dev)

    def gaussians(self) -> api.GaussianTensors:
        p = self.p
        return api.GaussianTensors(p["means"], p["scales"], p["quats"], None, p["ext"],
                                   sh=p["sh"], sh_active=self.sh_active)

    def _renderer(self, b: int) -> api.Renderer:
        r = self.renderers[b]
        if r is None:
            r = api.Renderer([self.gaussians()], [self.views[k] for k in self.batches[b]],
                             self.options)
            r.bound = (self.n, self.sh_active, self.p["means"].data_ptr())
            self.renderers[b] = r
        else:
            key = (self.n, self.sh_active, self.p["means"].data_ptr())
            if r.bound != key:
                if r.bound[:2] != key[:2]:
                    # pair counts change with the Gaussians, the plan's
                    # coefficient count with the SH degree
                    r.replan()
                r.scenes = [self.gaussians()]
                r._rebind()
                r.bound = key
        return r

    # ------------------------------------------------------------ steps
    def _lr_means(self) -> float:
        c = self.cfg
        t = min(self.it / max(c.iterations, 1), 1.0)
        return self.extent * math.exp((1 - t) * math.log(c.lr_means) +
                                      t * math.log(c.lr_means_final))

    def _adam(self, grads: dict):
        c = self.cfg
        lrs = {"means": self._lr_means(), "scales": c.lr_scales, "quats": c.lr_quats,
               "ext": c.lr_ext, "sh": c.lr_sh}
        bounds = {"ext": c.ext_bounds, "scales": c.scale_bounds}
        arr = (C.ParamGroup * len(GROUPS))()
        for k, name in enumerate(GROUPS):
            lo, hi = bounds.get(name, (0.0, 0.0))
            arr[k] = C.ParamGroup(self.p[name].data_ptr(), grads[name].data_ptr(),
                                  self.m[name].data_ptr(), self.v[name].data_ptr(),
                                  self.p[name].numel(), lrs[name], LOG_SPACE.get(name, 0),
                                  lo, hi, 0)
        C.check(self.lib.sdgr_adam_step(arr, len(GROUPS), self.it, ctypes.byref(self.adam_cfg),
                                        _stream(self.dev)))

    def _set(self, p, m, v) -> C.GaussianSet:
        s = C.GaussianSet()
        for g in ("means", "scales", "quats", "ext", "sh"):
            setattr(s, g, _ptr(p[g]))
            setattr(s, "m_" + g, _ptr(m[g]))
            setattr(s, "v_" + g, _ptr(v[g]))
        s.sh_coeffs = int(p["sh"].shape[1])
        s.reserved = 0
        return s

    def densify(self) -> int:
        """Densify and prune now; returns the new Gaussian count."""
        c = self.cfg
        n = self.n
        cap = 2 * n
        newp = {k: torch.empty((cap,) + tuple(t.shape[1:]), dtype=torch.float32, device=self.dev)
                for k, t in self.p.items()}
        newm = {k: torch.empty_like(t) for k, t in newp.items()}
        newv = {k: torch.empty_like(t) for k, t in newp.items()}
        wsb = self.lib.sdgr_densify_workspace_bytes(n)
        ws = torch.empty(max(int(wsb), 256), dtype=torch.uint8, device=self.dev)
        n_out = torch.zeros(1, dtype=torch.int64, device=self.dev)
        cfg = C.DensifyConfig(c.grad_threshold, c.split_frac * self.extent,
                              c.max_radius_frac * self.illum, c.kappa_min, c.split_factor, 0)
        sin, sout = self._set(self.p, self.m, self.v), self._set(newp, newm, newv)
        C.check(self.lib.sdgr_densify(ctypes.byref(sin), n, self.acc.data_ptr(),
                                      self.cnt.data_ptr(), self.dir.data_ptr(),
                                      ctypes.byref(cfg), ctypes.byref(sout), cap,
                                      n_out.data_ptr(), ws.data_ptr(), ws.numel(),
                                      _stream(self.dev)))
        k = int(n_out.item())   # synchronises
        self.p = {name: t[:k] for name, t in newp.items()}
        self.m = {name: t[:k] for name, t in newm.items()}
        self.v = {name: t[:k] for name, t in newv.items()}
        self._reset_stats()
        self.densify_calls += 1
        return k

    def step(self) -> None:
        """One iteration: forward and backward of the next batch of views,
        the statistics, one Adam step, and densify/prune on schedule."""
        c = self.cfg
        self.it += 1
        self.sh_active = min(c.sh_max, (self.it - 1) // c.sh_every)
        if not self.epoch_order:
            self.epoch_order = list(self.rng.permutation(len(self.batches)))
        b = int(self.epoch_order.pop())
        r = self._renderer(b)
        target = self.targets[b]
        while True:
            res = r.forward(r.planned(0.1))
            G = torch.sign(res.images[:target.numel()] - target) / float(target.numel())
            full = torch.zeros_like(res.images)
            full[:target.numel()] = G
            grads = r.backward(res, full)[0]
            try:
                r.status(res)
                break
            except C.SDGRError as exc:
                if exc.code != C.SDGR_EOVERFLOW:
                    raise
                r.replan()
        in_window = c.densify_from <= self.it < c.densify_until
        if in_window:
            C.check(self.lib.sdgr_densify_stats(grads["means"].data_ptr(), self.n,
                                                self.acc.data_ptr(), self.cnt.data_ptr(),
                                                self.dir.data_ptr(), _stream(self.dev)))
        self._adam(grads)
        if in_window and self.it % c.densify_every == 0:
            self.densify()

    def loss(self, b: int = 0) -> float:
        """Mean L1 of one batch at the current parameters (synchronises)."""
        r = self._renderer(b)
        res = r.forward()
        t = self.targets[b]
        return float((res.images[:t.numel()] - t).abs().mean())

    def run(self, iterations: Optional[int] = None, log_every: int = 0):
        for _ in range(iterations or self.cfg.iterations):
            self.step()
            if log_every and self.it % log_every == 0:
                self.history.append((self.it, self.n, self.loss()))
        return self


# ------------------------------------------------------------------ metrics

def image_metrics(images: torch.Tensor, refs: torch.Tensor, data_range: Optional[float] = None):
    """Mean SSIM and PSNR of images [N, H, W] against refs (library kernel);
    data_range defaults to the largest reference value."""
    images = images.contiguous().float()
    refs = refs.contiguous().float()
    N, H, W = refs.shape
    L = float(refs.max()) if data_range is None else float(data_range)
    ss = torch.empty(N, dtype=torch.float32, device=refs.device)
    mse = torch.empty_like(ss)
    mx = torch.empty_like(ss)
    C.check(C.lib().sdgr_image_metrics(images.data_ptr(), refs.data_ptr(), N, H, W, L,
                                       ss.data_ptr(), mse.data_ptr(), mx.data_ptr(),
                                       _stream(refs.device)))
    ss, mse, mx = ss.cpu().numpy(), mse.cpu().numpy(), mx.cpu().numpy()
    psnr = np.where(mse > 0, 10.0 * np.log10(np.maximum(mx, 1e-30) ** 2 / np.maximum(mse, 1e-300)),
                    np.inf)
    return dict(ssim=float(ss.mean()), psnr=float(psnr.mean()), ssim_per=ss, psnr_per=psnr)


def nearest_sq(q: torch.Tensor, ref: torch.Tensor) -> torch.Tensor:
    q, ref = q.contiguous().float(), ref.contiguous().float()
    out = torch.empty(q.shape[0], dtype=torch.float32, device=q.device)
    C.check(C.lib().sdgr_nearest_sq(q.data_ptr(), q.shape[0], ref.data_ptr(), ref.shape[0],
                                    out.data_ptr(), _stream(q.device)))
    return out


def point_metrics(recon: torch.Tensor, truth: torch.Tensor, tau: float):
    """Chamfer distance (half the sum of the mean nearest squared distances
    both ways), precision, recall and F1 at distance tau."""
    r2g = nearest_sq(truth, recon).double()
    g2r = nearest_sq(recon, truth).double()
    p = float((g2r.sqrt() < tau).double().mean())
    r = float((r2g.sqrt() < tau).double().mean())
    f1 = 2 * p * r / (p + r) if p + r > 0 else 0.0
    return dict(r2g=float(r2g.mean()), g2r=float(g2r.mean()),
                cd=0.5 * float(r2g.mean() + g2r.mean()), precision=p, recall=r, f1=f1)
