"""Python binding of the SDGR library: argument marshalling around the C ABI.

Every step of the forward and backward runs in the HIP kernels behind
``libsdgr.so``; PyTorch supplies device memory (all workspaces are torch
tensors) and the stream (the current stream of the tensors' device).

    scene = GaussianTensors.from_numpy(scenes.vehicle(), device="cuda")
    images = render(scene.means, scene.scales, scene.quats, scene.amp,
                    scene.ext, views)            # [V, H, W], differentiable

Optional per-Gaussian inputs: ``ext_back`` (the backward extinction; only
ext + ext_back enters the model) and ``sh`` ([n, (deg + 1)^2] coefficients
of a real spherical-harmonics phase function evaluated at the direction to
the radar, replacing amp; a view's ``radar_range`` places the radar, 0 is a
plane wave). ``RenderOptions.cell_area`` scales intensities by the
computation-plane cell area.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _capi as C

__all__ = ["RenderOptions", "GaussianTensors", "Renderer", "ForwardResult",
           "render", "SDGRFunction", "count_work", "WORK_NAMES"]


@dataclass(frozen=True)
class RenderOptions:
    shadowing: bool = True
    recompute: bool = False
    q_max: float = 9.0
    tau_max: float = 16.0
    dilation: float = 0.0
    deterministic: bool = False
    cell_area: bool = False

    def to_c(self) -> C.Options:
        o = C.Options()
        o.shadowing = int(bool(self.shadowing))
        o.recompute = int(bool(self.recompute))
        o.q_max = float(self.q_max)
        o.tau_max = float(self.tau_max)
        o.dilation = float(self.dilation)
        o.deterministic = int(bool(self.deterministic))
        o.tile = 0
        o.cell_area = int(bool(self.cell_area))
        o.reserved = 0
        return o


@dataclass
class GaussianTensors:
    means: torch.Tensor
    scales: torch.Tensor
    quats: torch.Tensor
    amp: Optional[torch.Tensor]            # None only with sh
    ext: torch.Tensor
    ext_back: Optional[torch.Tensor] = None
    sh: Optional[torch.Tensor] = None      # [n, (deg + 1)^2]
    sh_active: Optional[int] = None        # degree in use (<= the array's); None: all

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def sh_degree(self) -> int:
        """Degree the renderer evaluates (-1 without sh)."""
        if self.sh is None:
            return -1
        deg = int(round(math.sqrt(self.sh.shape[1]))) - 1
        if deg < 0 or deg > 3 or (deg + 1) ** 2 != self.sh.shape[1]:
            raise ValueError("sh must have 1, 4, 9 or 16 coefficients per Gaussian")
        if self.sh_active is not None:
            if not 0 <= self.sh_active <= deg:
                raise ValueError("sh_active outside 0..the array's degree")
            return int(self.sh_active)
        return deg

    @staticmethod
    def from_numpy(scene, device="cuda") -> "GaussianTensors":
        f = lambda a: None if a is None else torch.as_tensor(
            np.ascontiguousarray(a, dtype=np.float32), device=device)
        return GaussianTensors(f(scene.means), f(scene.scales), f(scene.quats),
                               f(scene.amp), f(scene.ext), f(getattr(scene, "ext_back", None)),
                               f(getattr(scene, "sh", None)))

    def named(self) -> dict:
        """The parameter tensors that are present, by gradient name."""
        d = {"means": self.means, "scales": self.scales, "quats": self.quats,
             "amp": self.amp, "ext": self.ext, "ext_back": self.ext_back, "sh": self.sh}
        return {k: v for k, v in d.items() if v is not None}


def _dev_f32(t: torch.Tensor, shape, name) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32:
        raise ValueError(f"{name} must be float32")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.contiguous()


def _scene_struct(g: GaussianTensors) -> C.Scene:
    n = g.n
    m = _dev_f32(g.means, (n, 3), "means")
    s = _dev_f32(g.scales, (n, 3), "scales")
    q = _dev_f32(g.quats, (n, 4), "quats")
    e = _dev_f32(g.ext, (n,), "ext")
    if g.amp is None and g.sh is None:
        raise ValueError("a scene needs amp or sh")
    a = None if g.amp is None else _dev_f32(g.amp, (n,), "amp")
    eb = None if g.ext_back is None else _dev_f32(g.ext_back, (n,), "ext_back")
    deg = g.sh_degree
    sh = None if g.sh is None else _dev_f32(g.sh, (n, g.sh.shape[1]), "sh")
    ptr = lambda t: 0 if t is None else t.data_ptr()
    st = C.Scene(n, m.data_ptr(), s.data_ptr(), q.data_ptr(), ptr(a), e.data_ptr(), ptr(eb),
                 ptr(sh), max(deg, 0), 0 if sh is None else int(sh.shape[1]))
    st._keep = (m, s, q, a, e, eb, sh)
    return st


def _view_structs(views, scene_ids=None):
    arr = (C.View * len(views))()
    off = 0
    shapes = []
    for k, v in enumerate(views):
        c = arr[k]
        c.azimuth = float(v.azimuth)
        c.grazing = float(v.grazing)
        c.d_az = float(v.d_az)
        c.d_rg = float(v.d_rg)
        c.comp_d_az = float(getattr(v, "comp_d_az", 0.0))
        c.comp_d_el = float(getattr(v, "comp_d_el", 0.0))
        c.img_offset = off
        c.img_w = int(v.img_w)
        c.img_h = int(v.img_h)
        c.comp_w = int(getattr(v, "comp_w", 0))
        c.comp_h = int(getattr(v, "comp_h", 0))
        c.scene = int(scene_ids[k] if scene_ids is not None else getattr(v, "scene", 0))
        c.reserved = 0
        c.radar_range = float(getattr(v, "radar_range", 0.0))
        shapes.append((off, int(v.img_h), int(v.img_w)))
        off += int(v.img_h) * int(v.img_w)
    return arr, shapes, off


def _stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _buf(nbytes: int, device) -> torch.Tensor:
    t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    if t.data_ptr() % 256:
        raise RuntimeError("workspace allocation not 256-byte aligned")
    return t


@dataclass
class ForwardResult:
    images: torch.Tensor          # flat float32 [image_floats]
    shapes: list                  # per view (offset, H, W)
    plan: C.Plan
    state: torch.Tensor

    def image(self, v: int) -> torch.Tensor:
        off, h, w = self.shapes[v]
        return self.images[off:off + h * w].view(h, w)

    def stacked(self) -> torch.Tensor:
        hs = {(h, w) for _, h, w in self.shapes}
        if len(hs) != 1:
            raise ValueError("views have different image sizes")
        h, w = hs.pop()
        return self.images[:len(self.shapes) * h * w].view(len(self.shapes), h, w)


class Renderer:
    """One (scenes, views, options) problem bound to the C ABI.

    Views refer to scenes through their ``scene`` attribute (or
    ``scene_ids``); several scenes and image sizes may share one launch."""

    def __init__(self, scenes: Sequence[GaussianTensors], views, options=None,
                 scene_ids=None):
        if isinstance(scenes, GaussianTensors):
            scenes = [scenes]
        self.scenes = list(scenes)
        self.device = self.scenes[0].means.device
        self.options = options or RenderOptions()
        self.lib = C.lib()
        self.views_c, self.shapes, self.image_floats = _view_structs(views, scene_ids)
        self.nv = len(views)
        self.opts_c = self.options.to_c()
        self._rebind()

    def _rebind(self):
        structs = [_scene_struct(g) for g in self.scenes]
        self._keep = [s._keep for s in structs]   # contiguous tensors behind the pointers
        self.scenes_c = (C.Scene * len(structs))(*structs)

    def plan(self) -> C.Plan:
        """Exact plan: counts the pairs on the device (synchronises)."""
        p = C.Plan()
        qb = self.lib.sdgr_query_bytes(len(self.scenes), self.nv)
        q = _buf(qb, self.device)
        C.check(self.lib.sdgr_plan_query(self.scenes_c, len(self.scenes), self.views_c,
                                         self.nv, ctypes.byref(self.opts_c), q.data_ptr(),
                                         qb, _stream_ptr(self.device), ctypes.byref(p)))
        self._last_exact = p
        return p

    def planned(self, headroom: float = 0.1) -> C.Plan:
        """A plan sized from this renderer's last exact query plus
        `headroom` (querying once if there is none). Pair counts move little
        while Gaussians are optimised, so most steps need no query; a forward
        that outgrows it reports SDGR_EOVERFLOW through status()."""
        if getattr(self, "_last_exact", None) is None:
            self._last_exact = self.plan()
        base = self._last_exact
        p = C.Plan()
        ctypes.pointer(p)[0] = base
        C.check(self.lib.sdgr_plan_resize(ctypes.byref(p),
                                          int(math.ceil(base.pairs_c * (1 + headroom))) + 64,
                                          int(math.ceil(base.pairs_i * (1 + headroom))) + 64))
        return p

    def plan_for(self, pairs_c: int, pairs_i: int) -> C.Plan:
        """The plan at given pair capacities, from host data only (no
        device work): e.g. the summed exact counts of the problems a fused
        launch joins."""
        p = C.Plan()
        C.check(self.lib.sdgr_plan_host(self.scenes_c, len(self.scenes), self.views_c, self.nv,
                                        ctypes.byref(self.opts_c), int(pairs_c), int(pairs_i),
                                        ctypes.byref(p)))
        return p

    def replan(self):
        """Forget the cached pair counts (after an overflow)."""
        self._last_exact = None

    def forward(self, plan: Optional[C.Plan] = None) -> ForwardResult:
        plan = plan or self.plan()
        state = _buf(plan.state_bytes, self.device)
        scratch = _buf(plan.fwd_scratch_bytes, self.device)
        images = torch.zeros(max(int(plan.image_floats), 1), dtype=torch.float32,
                             device=self.device)
        C.check(self.lib.sdgr_forward(self.scenes_c, len(self.scenes), self.views_c, self.nv,
                                      ctypes.byref(self.opts_c), ctypes.byref(plan),
                                      state.data_ptr(), scratch.data_ptr(),
                                      images.data_ptr(), _stream_ptr(self.device)))
        return ForwardResult(images, self.shapes, plan, state)

    def backward(self, fwd: ForwardResult, grad_images: torch.Tensor):
        """Gradients for every scene: list of dicts of tensors, one entry per
        parameter tensor the scene has (amp's is zero with sh)."""
        g = grad_images.contiguous().view(-1)
        if g.dtype != torch.float32 or g.numel() < fwd.plan.image_floats:
            raise ValueError("grad_images must be float32 and cover every image")
        scratch = _buf(fwd.plan.bwd_scratch_bytes, self.device)
        outs = []
        grads_c = (C.SceneGrad * len(self.scenes))()
        # every scene's gradient tensors are views of one allocation (a fused
        # launch of many requests would otherwise make ~100 allocator calls);
        # each view starts on a 64-float boundary
        named = [sc.named() for sc in self.scenes]
        total = sum((t.numel() + 63) // 64 * 64 for d in named for t in d.values())
        flat = torch.empty(max(total, 1), dtype=torch.float32, device=self.device)
        off = 0
        for k, sc in enumerate(self.scenes):
            d = {}
            for name, t in named[k].items():
                d[name] = flat[off:off + t.numel()].view(t.shape)
                off += (t.numel() + 63) // 64 * 64
            if "sh" in d and sc.sh_degree + 1 < round(math.sqrt(sc.sh.shape[1])):
                d["sh"].zero_()   # the coefficients above the active degree get none
            ptr = lambda name: d[name].data_ptr() if name in d else 0
            grads_c[k] = C.SceneGrad(ptr("means"), ptr("scales"), ptr("quats"), ptr("amp"),
                                     ptr("ext"), ptr("ext_back"), ptr("sh"))
            outs.append(d)
        C.check(self.lib.sdgr_backward(self.scenes_c, len(self.scenes), self.views_c, self.nv,
                                       ctypes.byref(self.opts_c), ctypes.byref(fwd.plan),
                                       fwd.state.data_ptr(), scratch.data_ptr(), g.data_ptr(),
                                       grads_c, _stream_ptr(self.device)))
        return outs

    def status(self, fwd: ForwardResult):
        C.check(self.lib.sdgr_status(ctypes.byref(fwd.plan), fwd.state.data_ptr(),
                                     _stream_ptr(self.device)))

    def status_into(self, fwd: ForwardResult, flags: torch.Tensor):
        """The overflow check without a host sync: ORs the flag into the
        device int32 tensor `flags` (one element, starting at 0), so a loop
        can read it once for many steps."""
        if flags.dtype != torch.int32 or flags.numel() < 1 or not flags.is_cuda:
            raise ValueError("flags must be a CUDA int32 tensor")
        C.check(self.lib.sdgr_status_accumulate(ctypes.byref(fwd.plan), fwd.state.data_ptr(),
                                                flags.data_ptr(), _stream_ptr(self.device)))

    def intensity_shares(self, fwd: ForwardResult) -> torch.Tensor:
        """A per record, view-major (flat)."""
        out = torch.empty(max(int(fwd.plan.records), 1), dtype=torch.float32,
                          device=self.device)
        C.check(self.lib.sdgr_read_intensity(ctypes.byref(fwd.plan), fwd.state.data_ptr(),
                                             out.data_ptr(), _stream_ptr(self.device)))
        return out[:fwd.plan.records]

    def work_counters(self, fwd: ForwardResult) -> dict:
        """Work counters of the last forward (and backward) on `fwd`'s state;
        filled only for calls made while count_work(True) was in effect."""
        wk = (ctypes.c_uint64 * len(WORK_NAMES))()
        C.check(self.lib.sdgr_read_work(ctypes.byref(fwd.plan), fwd.state.data_ptr(), wk,
                                        len(WORK_NAMES),
                                        _stream_ptr(self.device)))
        return dict(zip(WORK_NAMES, list(wk)))

    def optical_depth(self, fwd: ForwardResult) -> torch.Tensor:
        out = torch.empty(max(int(fwd.plan.rays), 1), dtype=torch.float32, device=self.device)
        C.check(self.lib.sdgr_read_optical_depth(ctypes.byref(fwd.plan), fwd.state.data_ptr(),
                                                 out.data_ptr(), _stream_ptr(self.device)))
        return out[:fwd.plan.rays]


WORK_NAMES = ("hits_a_fwd", "hits_a_bwd", "hits_b_fwd", "hits_b_bwd", "rounds_a_fwd",
              "rounds_a_bwd", "rounds_b_fwd", "list_prefix_a", "max_batches_a_fwd",
              "max_batches_a_bwd", "extra_hit_groups_a_fwd", "extra_hit_groups_a_bwd",
              "rays_stopped_tau_max", "max_list_prefix_a", "tiles_a_bwd_long", "tiles_a_bwd_short",
              "tiles_a_bwd_stored", "tiles_a_bwd_rederived")


def count_work(on: bool) -> None:
    """Turn the library's work counters on or off for later calls."""
    C.check(C.lib().sdgr_profile_count(int(bool(on))))


class SDGRFunction(torch.autograd.Function):
    """Differentiable SAR rendering of one scene over a batch of views of
    equal image size; the backward is the library's hand-written one.
    ext_back and sh may be None (and amp None when sh is given)."""

    @staticmethod
    def forward(ctx, views, options, means, scales, quats, amp, ext, ext_back=None, sh=None):
        det = lambda t: None if t is None else t.detach()
        g = GaussianTensors(det(means), det(scales), det(quats), det(amp), det(ext),
                            det(ext_back), det(sh))
        r = Renderer([g], views, options)
        res = r.forward()
        ctx.renderer = r
        ctx.result = res
        return res.stacked()

    @staticmethod
    def backward(ctx, grad_images):
        r, res = ctx.renderer, ctx.result
        full = torch.zeros_like(res.images)
        n = grad_images.numel()
        full[:n] = grad_images.reshape(-1)
        d = r.backward(res, full)[0]
        ctx.renderer = ctx.result = None
        return (None, None, d["means"], d["scales"], d["quats"], d.get("amp"), d["ext"],
                d.get("ext_back"), d.get("sh"))


def render(means, scales, quats, amp, ext, views, options: Optional[RenderOptions] = None,
           ext_back=None, sh=None):
    """SAR images [V, H, W] of one scene; differentiable w.r.t. every
    parameter tensor given (amp may be None when sh is given)."""
    return SDGRFunction.apply(list(views), options or RenderOptions(), means, scales, quats,
                              amp, ext, ext_back, sh)
