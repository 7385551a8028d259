"""Seeded synthetic inputs: Gaussian scenes and radar views.

This module only *draws inputs*. It holds none of the rasterizer's arithmetic
(no projection, footprint, attenuation or image formation), so both the CPU
oracle and the HIP path consume exactly the arrays produced here.

Every generator is driven by ``numpy.random.Generator(PCG64(seed))`` and
returns float32 arrays, the precision the renderer takes at its boundary.

Scene shapes stand in for the paper's targets (simplified buildings of the
forward-rendering experiment, Sec. III-A; vehicles of the rendered and MSTAR
sets, Sec. III-B/C), whose models and datasets are not available: boxes,
cylinders and ground planes covered by surface-aligned Gaussians.

Angle convention: ``grazing`` is the depression angle theta of the radar
rotation matrix (Sec. II-A, Eq. for R_r); the workloads quote *incidence*
measured from the vertical, so grazing = 90 deg - incidence.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

__all__ = [
    "Scene", "View", "make_rng", "random_quats", "fwd_1k", "building",
    "vehicle", "large_block", "serving_scenes", "vehicle_views",
    "building_views", "large_views", "jitter", "WORKLOADS",
    "reconstruction_views", "reconstruction_test_views", "hemisphere_init",
]


@dataclass
class Scene:
    """N anisotropic Gaussians, structure-of-arrays, float32.

    means  (N,3) world position [m]
    scales (N,3) per-axis standard deviation [m], > 0 (not log)
    quats  (N,4) rotation quaternion (w, x, y, z), any nonzero norm
    amp    (N,)  scattering amplitude P >= 0 (phase function, scalar form)
    ext    (N,)  extinction kappa = k_e+ + k_e- >= 0, or k_e+ alone when
                 ext_back is given
    ext_back (N,) optional backward extinction k_e- (kappa = ext + ext_back)
    sh     (N,(d+1)^2) optional spherical-harmonics coefficients of the phase
                 function, degree d <= 3 (then amp is not used)
    """
    means: np.ndarray
    scales: np.ndarray
    quats: np.ndarray
    amp: np.ndarray
    ext: np.ndarray
    ext_back: Optional[np.ndarray] = None
    sh: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def sh_degree(self) -> int:
        return -1 if self.sh is None else int(round(math.sqrt(self.sh.shape[1]))) - 1

    def subset(self, idx) -> "Scene":
        opt = lambda a: None if a is None else a[idx].copy()
        return Scene(self.means[idx].copy(), self.scales[idx].copy(),
                     self.quats[idx].copy(), self.amp[idx].copy(),
                     self.ext[idx].copy(), opt(self.ext_back), opt(self.sh))

    def copy(self) -> "Scene":
        return self.subset(slice(None))

    def concat(self, other: "Scene") -> "Scene":
        if (self.ext_back is None) != (other.ext_back is None) or \
                (self.sh is None) != (other.sh is None):
            raise ValueError("scenes differ in their optional inputs")
        opt = lambda a, b: None if a is None else np.concatenate([a, b])
        return Scene(*(np.concatenate([a, b]) for a, b in zip(
            (self.means, self.scales, self.quats, self.amp, self.ext),
            (other.means, other.scales, other.quats, other.amp, other.ext))),
            ext_back=opt(self.ext_back, other.ext_back), sh=opt(self.sh, other.sh))


@dataclass
class View:
    """One radar view. Angles in radians (float64).

    Image: img_h range rows x img_w azimuth columns, spacings d_rg, d_az [m].
    Computation plane: comp_h x comp_w cells with spacings comp_d_el,
    comp_d_az; a zero means "use the paper's default" (same grid as the
    image, elevation spacing d_rg * tan(grazing)), which each consumer
    resolves itself.
    """
    azimuth: float
    grazing: float
    img_w: int
    img_h: int
    d_az: float
    d_rg: float
    comp_w: int = 0
    comp_h: int = 0
    comp_d_az: float = 0.0
    comp_d_el: float = 0.0
    scene: int = 0
    radar_range: float = 0.0   # slant distance of the radar from the origin [m]; 0: plane wave

    @staticmethod
    def from_degrees(azimuth_deg: float, incidence_deg: float, size: int,
                     spacing: float, **kw) -> "View":
        return View(azimuth=math.radians(azimuth_deg),
                    grazing=math.radians(90.0 - incidence_deg),
                    img_w=size, img_h=size, d_az=spacing, d_rg=spacing, **kw)


def make_rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_quats(rng, n) -> np.ndarray:
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.astype(np.float32)


def _log_uniform(rng, lo, hi, size):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size))


def _qmul(a, b):
    """Hamilton product of quaternion arrays (w, x, y, z)."""
    w1, x1, y1, z1 = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    w2, x2, y2, z2 = b[..., 0], b[..., 1], b[..., 2], b[..., 3]
    return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], axis=-1)


def _surface_quats(rng, normals):
    """Quaternions whose local z axis maps onto `normals`, spun about it by
    a uniform in-plane angle (so flattened Gaussians lie in the surface)."""
    n = normals.shape[0]
    nx, ny, nz = normals[:, 0], normals[:, 1], normals[:, 2]
    align = np.stack([1.0 + nz, -ny, nx, np.zeros(n)], axis=-1)
    flip = nz < -1.0 + 1e-9
    align[flip] = np.array([0.0, 1.0, 0.0, 0.0])
    align /= np.linalg.norm(align, axis=1, keepdims=True)
    a = rng.uniform(0.0, 2.0 * math.pi, n)
    spin = np.stack([np.cos(a / 2), np.zeros(n), np.zeros(n), np.sin(a / 2)],
                    axis=-1)
    q = _qmul(align, spin)
    return (q / np.linalg.norm(q, axis=1, keepdims=True)).astype(np.float32)


# ---------------------------------------------------------------- surfaces
# A surface patch list is [(area, sampler)] where sampler(rng, k) returns
# (points (k,3), normals (k,3)).

def _rect_patch(origin, u, v, normal):
    origin, u, v, normal = map(np.asarray, (origin, u, v, normal))
    area = float(np.linalg.norm(u) * np.linalg.norm(v))

    def sample(rng, k):
        a = rng.uniform(0, 1, (k, 1))
        b = rng.uniform(0, 1, (k, 1))
        return origin + a * u + b * v, np.tile(normal, (k, 1))
    return area, sample


def _box_patches(center, dims, bottom=True, top=True):
    cx, cy, cz = center
    dx, dy, dz = dims
    x0, y0, z0 = cx - dx / 2, cy - dy / 2, cz - dz / 2
    p = [
        _rect_patch((x0, y0, z0), (0, dy, 0), (0, 0, dz), (-1, 0, 0)),
        _rect_patch((x0 + dx, y0, z0), (0, dy, 0), (0, 0, dz), (1, 0, 0)),
        _rect_patch((x0, y0, z0), (dx, 0, 0), (0, 0, dz), (0, -1, 0)),
        _rect_patch((x0, y0 + dy, z0), (dx, 0, 0), (0, 0, dz), (0, 1, 0)),
    ]
    if top:
        p.append(_rect_patch((x0, y0, z0 + dz), (dx, 0, 0), (0, dy, 0),
                             (0, 0, 1)))
    if bottom:
        p.append(_rect_patch((x0, y0, z0), (dx, 0, 0), (0, dy, 0),
                             (0, 0, -1)))
    return p


def _cylinder_patches(center, radius, length, axis):
    """Closed cylinder with its axis along world x (axis=0) or z (axis=2)."""
    c = np.asarray(center, float)
    if axis == 2:
        e_ax, e_a, e_b = np.eye(3)[2], np.eye(3)[0], np.eye(3)[1]
    else:
        e_ax, e_a, e_b = np.eye(3)[0], np.eye(3)[1], np.eye(3)[2]

    def lateral(rng, k):
        t = rng.uniform(0, 2 * math.pi, (k, 1))
        h = rng.uniform(-length / 2, length / 2, (k, 1))
        nrm = np.cos(t) * e_a + np.sin(t) * e_b
        return c + h * e_ax + radius * nrm, nrm

    def cap(sign):
        def s(rng, k):
            t = rng.uniform(0, 2 * math.pi, (k, 1))
            r = radius * np.sqrt(rng.uniform(0, 1, (k, 1)))
            pts = c + sign * (length / 2) * e_ax + r * (np.cos(t) * e_a +
                                                          np.sin(t) * e_b)
            return pts, np.tile(sign * e_ax, (k, 1))
        return s
    return [(2 * math.pi * radius * length, lateral),
            (math.pi * radius ** 2, cap(1.0)),
            (math.pi * radius ** 2, cap(-1.0))]


def _ground_patch(half, holes):
    """Square [-half, half]^2 at z = 0 minus axis-aligned rectangular holes
    given as (x0, x1, y0, y1); sampled by rejection."""
    area = (2 * half) ** 2 - sum((h[1] - h[0]) * (h[3] - h[2]) for h in holes)

    def sample(rng, k):
        out = np.empty((0, 3))
        while out.shape[0] < k:
            m = max(2 * (k - out.shape[0]), 64)
            xy = rng.uniform(-half, half, (m, 2))
            keep = np.ones(m, bool)
            for x0, x1, y0, y1 in holes:
                keep &= ~((xy[:, 0] > x0) & (xy[:, 0] < x1) &
                          (xy[:, 1] > y0) & (xy[:, 1] < y1))
            xy = xy[keep]
            out = np.concatenate([out, np.column_stack(
                [xy, np.zeros(xy.shape[0])])])
        return out[:k], np.tile([0.0, 0.0, 1.0], (k, 1))
    return area, sample


def _sample_patches(rng, patches, n):
    areas = np.array([a for a, _ in patches], float)
    counts = rng.multinomial(n, areas / areas.sum())
    pts, nrm = [], []
    for (area, sampler), k in zip(patches, counts):
        if k:
            p, q = sampler(rng, int(k))
            pts.append(p)
            nrm.append(q)
    return np.concatenate(pts), np.concatenate(nrm)


def _extinction(rng, n):
    return rng.uniform(1.0, 4.0, n).astype(np.float32)


# ---------------------------------------------------------------- workloads

def fwd_1k(seed: int = 101, n: int = 1000):
    """1,000 Gaussians uniform in a 10 m cube; one view at 45 deg incidence,
    azimuth 0; 64x64 image at 0.15 m."""
    rng = make_rng(seed)
    means = rng.uniform(-5.0, 5.0, (n, 3)).astype(np.float32)
    scales = _log_uniform(rng, 0.05, 0.5, (n, 3)).astype(np.float32)
    quats = random_quats(rng, n)
    amp = rng.uniform(0.0, 1.0, n).astype(np.float32)
    ext = _extinction(rng, n)
    views = [View.from_degrees(0.0, 45.0, 64, 0.15)]
    return Scene(means, scales, quats, amp, ext), views


def building(seed: int = 202, n: int = 50_000):
    """One 10 x 8 x 6 m box on a ground square [-9.6, 9.6]^2; Gaussians
    flattened along the surface normal (normal std 0.01 m)."""
    rng = make_rng(seed)
    patches = _box_patches((0.0, 0.0, 3.0), (10.0, 8.0, 6.0), bottom=False)
    patches.append(_ground_patch(9.6, [(-5.0, 5.0, -4.0, 4.0)]))
    pts, nrm = _sample_patches(rng, patches, n)
    tang = _log_uniform(rng, 0.05, 0.2, (n, 2))
    scales = np.column_stack([tang, np.full(n, 0.01)]).astype(np.float32)
    quats = _surface_quats(rng, nrm)
    amp = rng.uniform(0.2, 1.0, n).astype(np.float32)
    ext = _extinction(rng, n)
    return Scene(pts.astype(np.float32), scales, quats, amp, ext)


def building_views(size: int = 128, spacing: float = 0.15,
                   incidence: float = 40.0, step: float = 10.0):
    return [View.from_degrees(k * step, incidence, size, spacing)
            for k in range(int(round(360.0 / step)))]


def _vehicle_primitives(rng):
    env = np.array([6.0, 3.0, 2.5])
    prims = []
    for _ in range(int(rng.integers(3, 7))):
        dims = rng.uniform(0.2, 1.0, 3) * env
        lo = np.array([-env[0] / 2, -env[1] / 2, 0.0]) + dims / 2
        hi = np.array([env[0] / 2, env[1] / 2, env[2]]) - dims / 2
        c = rng.uniform(lo, hi)
        c[2] -= env[2] / 2
        if rng.uniform() < 0.5:
            prims.extend(_box_patches(c, dims))
        else:
            axis = 2 if rng.uniform() < 0.5 else 0
            if axis == 2:
                radius, length = min(dims[0], dims[1]) / 2, dims[2]
            else:
                radius, length = min(dims[1], dims[2]) / 2, dims[0]
            prims.extend(_cylinder_patches(c, radius, length, axis))
    return prims


def vehicle(seed: int = 303, n: int = 200_000):
    """Composite of 3-6 axis-aligned boxes/cylinders inside a 6 x 3 x 2.5 m
    envelope (z-centred at 0), no ground; random Gaussian orientations."""
    rng = make_rng(seed)
    pts, _ = _sample_patches(rng, _vehicle_primitives(rng), n)
    scales = _log_uniform(rng, 0.02, 0.15, (n, 3)).astype(np.float32)
    quats = random_quats(rng, n)
    amp = rng.lognormal(0.0, 0.5, n).astype(np.float32)
    ext = _extinction(rng, n)
    return Scene(pts.astype(np.float32), scales, quats, amp, ext)


def vehicle_views(size: int = 256, spacing: float = 0.1, count: int = 72,
                  step: float = 5.0):
    """Azimuth k*step deg; incidence 30 deg for even k, 45 deg for odd k."""
    return [View.from_degrees(k * step, 30.0 if k % 2 == 0 else 45.0, size,
                              spacing) for k in range(count)]


def reconstruction_views(size: int = 64, spacing: float = 0.2):
    """Training views of the synthetic reconstruction (Sec. III-B): incidence
    15, 45 and 75 deg, azimuth every 15 deg (72 views)."""
    return [View.from_degrees(15.0 * k, inc, size, spacing)
            for inc in (15.0, 45.0, 75.0) for k in range(24)]


def reconstruction_test_views(size: int = 64, spacing: float = 0.2):
    """Held-out views between the training ones: azimuth 7.5 + 15 k deg,
    incidence 30 and 60 deg alternating (24 views)."""
    return [View.from_degrees(7.5 + 15.0 * k, 30.0 if k % 2 == 0 else 60.0, size, spacing)
            for k in range(24)]


def hemisphere_init(n: int, radius: float, seed: int = 404, sh_coeffs: int = 16,
                    p0: float = 0.5, kappa0: float = 0.5, center=(0.0, 0.0, 0.0)):
    """Initial point cloud of the reconstruction: n Gaussians on the upper
    hemispherical shell of the given radius about `center` (uniform in
    area), isotropic with the shell's mean point spacing as standard
    deviation, identity rotations, extinction kappa0, and a constant phase
    function p0 (degree-0 SH coefficient p0 / Y00, higher ones zero)."""
    rng = make_rng(seed)
    z = rng.uniform(0.0, 1.0, n)             # uniform in area on the hemisphere
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    rxy = np.sqrt(1.0 - z * z)
    pts = radius * np.stack([rxy * np.cos(phi), rxy * np.sin(phi), z], axis=1) + \
        np.asarray(center, np.float64)
    spacing = math.sqrt(2.0 * math.pi * radius * radius / max(n, 1))
    scales = np.full((n, 3), 0.5 * spacing, np.float32)
    quats = np.tile(np.array([1.0, 0.0, 0.0, 0.0], np.float32), (n, 1))
    sh = np.zeros((n, sh_coeffs), np.float32)
    sh[:, 0] = p0 / (0.5 / math.sqrt(math.pi))
    sc = Scene(pts.astype(np.float32), scales, quats, np.full(n, p0, np.float32),
               np.full(n, kappa0, np.float32))
    sc.sh = sh
    return sc


def large_block(seed: int = 505, n: int = 2_000_000):
    """Ground [-50, 50]^2 with 20-40 non-overlapping boxes (footprint sides
    U[4, 15] m, heights U[3, 30] m)."""
    rng = make_rng(seed)
    boxes = []
    target = int(rng.integers(20, 41))
    tries = 0
    while len(boxes) < target and tries < 10_000:
        tries += 1
        w, d = rng.uniform(4.0, 15.0, 2)
        h = rng.uniform(3.0, 30.0)
        cx, cy = rng.uniform(-45.0 + w / 2, 45.0 - w / 2), \
            rng.uniform(-45.0 + d / 2, 45.0 - d / 2)
        r = (cx - w / 2, cx + w / 2, cy - d / 2, cy + d / 2)
        if any(not (r[1] + 1 < b[0] or b[1] + 1 < r[0] or r[3] + 1 < b[2]
                    or b[3] + 1 < r[2]) for b, _ in boxes):
            continue
        boxes.append((r, h))
    patches = [_ground_patch(50.0, [b for b, _ in boxes])]
    for (x0, x1, y0, y1), h in boxes:
        patches.extend(_box_patches(((x0 + x1) / 2, (y0 + y1) / 2, h / 2),
                                    (x1 - x0, y1 - y0, h), bottom=False))
    pts, _ = _sample_patches(rng, patches, n)
    scales = _log_uniform(rng, 0.05, 0.5, (n, 3)).astype(np.float32)
    quats = random_quats(rng, n)
    amp = rng.lognormal(0.0, 0.7, n).astype(np.float32)
    ext = _extinction(rng, n)
    return Scene(pts.astype(np.float32), scales, quats, amp, ext)


def large_views(size: int = 1024, spacing: float = 0.1, count: int = 16,
                incidence: float = 35.0):
    return [View.from_degrees(k * 360.0 / count, incidence, size, spacing)
            for k in range(count)]


def serving_scenes(seed: int = 404, count: int = 8, n_lo: int = 10_000,
                   n_hi: int = 500_000):
    """Resident scenes for the serving stream: vehicle-like, with Gaussian
    counts log-uniform in [n_lo, n_hi]."""
    rng = make_rng(seed)
    ns = np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), count)).astype(int)
    seeds = rng.integers(0, 2 ** 31 - 1, count)
    return [vehicle(int(s), int(k)) for s, k in zip(seeds, ns)]


def jitter(scene: Scene, seed: int, sigma: float = 0.1) -> Scene:
    """Copy of `scene` with means displaced by N(0, sigma^2) per axis (the
    target of the L1 reconstruction loss)."""
    rng = make_rng(seed)
    out = scene.copy()
    out.means = (scene.means + rng.normal(0.0, sigma, scene.means.shape)
                 ).astype(np.float32)
    return out


WORKLOADS = {
    "fwd_1k": "1,000 Gaussians in a 10 m cube, 1 view, 64x64 @ 0.15 m, "
              "forward only",
    "building_50k": "50,000 Gaussians on a 10x8x6 m box + ground, 36 views, "
                    "128x128 @ 0.15 m, forward+backward, L1 loss",
    "vehicle_200k": "200,000 Gaussians on a vehicle-scale composite, 72 "
                    "views, 256x256 @ 0.1 m, forward+backward, L1 loss",
    "serving": "8 resident vehicle scenes of 1e4-5e5 Gaussians, Poisson "
               "requests of 1-16 views at 64-512 px",
    "large_2m": "2,000,000 Gaussians on a 100x100 m block, 16 views, "
                "1024x1024 @ 0.1 m, forward+backward with recomputation",
}
