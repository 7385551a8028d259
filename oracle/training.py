"""FP64 reference of the reconstruction loop's non-rendering steps and of the
evaluation metrics.

TEST INFRASTRUCTURE ONLY, like the rest of this package: the product path
never imports it, and it imports nothing from the product.

What it computes, each function citing the passage it follows:
  adam_step      -- the optimiser of the reconstruction (Sec. III-B: the
                    Gaussians' parameters are fitted by gradient descent;
                    Adam as published by Kingma and Ba, with bias correction).
                    Positive parameters may be stepped in log space.
  densify        -- densification and pruning (Sec. II-B, "Densification and
                    Pruning Operation"; thresholds from the ablation study:
                    gradient threshold 0.003, largest radius 0.3 times the
                    illumination range).
  psnr, ssim     -- image metrics (Sec. III-B, "Evaluation Metrics", the PSNR
                    and SSIM equations).
  chamfer_f1     -- point-cloud metrics (same passage: Chamfer distance and
                    precision, recall and F1 at a distance threshold).

Readings where the paper leaves the details open (each listed in the design
notes): the densification statistic is the mean, over the iterations in
which a Gaussian received a position gradient, of that gradient's norm; a
clone is displaced against the accumulated position gradient by its largest
standard deviation; a split makes two children with standard deviations
divided by 1.6, one standard deviation either side of the centre along the
largest axis, both displaced against the gradient by the children's largest
standard deviation; a Gaussian whose extinction is below kappa_min (the
paper's "excessively small" coefficient) or whose footprint radius (three
largest standard deviations) exceeds the largest radius is pruned. SSIM uses
the usual 11 x 11 Gaussian window (sigma 1.5) over the positions where the
window fits, C1 = (0.01 L)^2, C2 = (0.03 L)^2. Decisions that turn floating
point into a choice (the thresholds) are taken in FP32, as the kernels do.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# parameter groups of one scene, in the order the loop steps them
GROUPS = ("means", "scales", "quats", "amp", "ext", "sh")


# ---------------------------------------------------------------- optimiser

@dataclass
class AdamConfig:
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-15


def adam_step(x, g, m, v, t, lr, log_space=False, cfg=AdamConfig(), lo=0.0, hi=0.0):
    """One Adam step at iteration t (1-based) on a parameter array x with
    gradient g and moments m, v (all float64 copies are returned).

    log_space: x > 0 is stepped as u = log x, whose gradient is g x, and
    updated as x exp(-step). lo < hi: the result is clamped to [lo, hi]."""
    x = np.asarray(x, np.float64)
    g = np.asarray(g, np.float64)
    m = np.asarray(m, np.float64)
    v = np.asarray(v, np.float64)
    if log_space:
        g = g * x
    m = cfg.beta1 * m + (1.0 - cfg.beta1) * g
    v = cfg.beta2 * v + (1.0 - cfg.beta2) * g * g
    mhat = m / (1.0 - cfg.beta1 ** t)
    vhat = v / (1.0 - cfg.beta2 ** t)
    step = lr * mhat / (np.sqrt(vhat) + cfg.eps)
    x = x * np.exp(-step) if log_space else x - step
    if lo < hi:
        x = np.clip(x, lo, hi)
    return x, m, v


# ----------------------------------------------------- densify and prune

@dataclass
class DensifyConfig:
    grad_threshold: float = 0.003   # mean position-gradient norm
    split_scale: float = 0.1        # largest std above this: split, else clone
    max_radius: float = 1.0         # 3 x largest std above this: pruned
    kappa_min: float = 0.005        # extinction below this: pruned
    split_factor: float = 1.6       # children's std = parent's / split_factor


KEEP, PRUNE, CLONE, SPLIT = 0, 1, 2, 3


def _rotation(q):
    """Rotation matrix of a (w, x, y, z) quaternion, normalised first."""
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def densify_actions(scales, ext, grad_acc, grad_cnt, cfg: DensifyConfig):
    """Action of every Gaussian (KEEP, PRUNE, CLONE, SPLIT), decided in FP32:
    prune first (extinction below kappa_min, or footprint radius 3 s_max
    above max_radius), then clone or split where the mean gradient norm
    reaches the threshold (split when s_max exceeds split_scale)."""
    f = np.float32
    s = np.asarray(scales, f)
    smax = s.max(axis=1)
    kap = np.asarray(ext, f)
    acc = np.asarray(grad_acc, f)
    cnt = np.asarray(grad_cnt, f)
    act = np.full(len(s), KEEP, np.int64)
    for i in range(len(s)):
        if kap[i] < f(cfg.kappa_min) or f(3.0) * smax[i] > f(cfg.max_radius):
            act[i] = PRUNE
        elif cnt[i] > 0 and acc[i] / cnt[i] >= f(cfg.grad_threshold):
            act[i] = SPLIT if smax[i] > f(cfg.split_scale) else CLONE
    return act


def densify(params: dict, moments: dict, grad_acc, grad_cnt, grad_dir,
            cfg: DensifyConfig):
    """Densified and pruned Gaussians, in input order: each kept Gaussian,
    each cloned one followed by its copy, each split one replaced by its two
    children, each pruned one dropped. New Gaussians (copies, children) start
    with zero Adam moments; kept and cloned originals keep theirs.

    params: means [n,3], scales [n,3], quats [n,4], ext [n] and optional amp
    [n], sh [n,k]; moments: {group: (m, v)} for the same groups; grad_dir
    [n,3]: accumulated position gradient (its direction gives the
    displacement). Returns (params, moments, actions)."""
    act = densify_actions(params["scales"], params["ext"], grad_acc, grad_cnt, cfg)
    names = [k for k in GROUPS if params.get(k) is not None]
    out = {k: [] for k in names}
    mom = {k: ([], []) for k in names}

    def emit(i, mean, scale, fresh):
        for k in names:
            val = np.array(params[k][i], np.float64)
            if k == "means":
                val = mean
            elif k == "scales":
                val = scale
            out[k].append(val)
            m, v = moments[k]
            z = np.zeros_like(np.asarray(m[i], np.float64))
            mom[k][0].append(z if fresh else np.array(m[i], np.float64))
            mom[k][1].append(z if fresh else np.array(v[i], np.float64))

    for i, a in enumerate(act):
        mu = np.asarray(params["means"][i], np.float64)
        s = np.asarray(params["scales"][i], np.float64)
        if a == PRUNE:
            continue
        if a == KEEP:
            emit(i, mu, s, False)
            continue
        gd = np.asarray(grad_dir[i], np.float64)
        gn = np.linalg.norm(gd)
        ghat = gd / gn if gn > 0 else np.zeros(3)
        if a == CLONE:
            emit(i, mu, s, False)
            emit(i, mu - s.max() * ghat, s, True)
        else:
            axis = _rotation(params["quats"][i])[:, int(np.argmax(s))]
            cs = s / cfg.split_factor
            for sign in (1.0, -1.0):
                emit(i, mu + sign * s.max() * axis - cs.max() * ghat, cs, True)
    res = {k: np.array(out[k]) for k in names}
    mres = {k: (np.array(mom[k][0]), np.array(mom[k][1])) for k in names}
    return res, mres, act


# ------------------------------------------------------------------ metrics

def psnr(x, ref):
    """10 log10(MAX^2 / MSE) with MAX the reference image's maximum."""
    x, ref = np.asarray(x, np.float64), np.asarray(ref, np.float64)
    mse = np.mean((x - ref) ** 2)
    return 10.0 * math.log10(ref.max() ** 2 / mse) if mse > 0 else math.inf


def gaussian_window(size=11, sigma=1.5):
    r = np.arange(size) - (size - 1) / 2.0
    g = np.exp(-r * r / (2.0 * sigma * sigma))
    w = np.outer(g, g)
    return w / w.sum()


def ssim(x, ref, data_range, size=11, sigma=1.5):
    """Mean SSIM over the positions where the whole window fits: at each,
    the window-weighted means, variances and covariance enter the SSIM
    equation with C1 = (0.01 L)^2, C2 = (0.03 L)^2, L = data_range."""
    x, ref = np.asarray(x, np.float64), np.asarray(ref, np.float64)
    H, W = x.shape
    if H < size or W < size:
        raise ValueError("image smaller than the SSIM window")
    w = gaussian_window(size, sigma)
    c1, c2 = (0.01 * data_range) ** 2, (0.03 * data_range) ** 2
    vals = np.empty((H - size + 1, W - size + 1))
    for r in range(H - size + 1):
        for c in range(W - size + 1):
            a = x[r:r + size, c:c + size]
            b = ref[r:r + size, c:c + size]
            ma, mb = (w * a).sum(), (w * b).sum()
            va = (w * (a - ma) ** 2).sum()
            vb = (w * (b - mb) ** 2).sum()
            cov = (w * (a - ma) * (b - mb)).sum()
            vals[r, c] = ((2 * ma * mb + c1) * (2 * cov + c2)) / \
                ((ma * ma + mb * mb + c1) * (va + vb + c2))
    return float(vals.mean())


def nearest_sq(q, ref, chunk=2048):
    """Squared distance from every point of q to its nearest point of ref
    (exhaustive)."""
    q, ref = np.asarray(q, np.float64), np.asarray(ref, np.float64)
    out = np.empty(len(q))
    for a in range(0, len(q), chunk):
        d = ((q[a:a + chunk, None, :] - ref[None, :, :]) ** 2).sum(-1)
        out[a:a + chunk] = d.min(axis=1)
    return out


def chamfer_f1(recon, truth, tau):
    """The paper's Chamfer distance (half the sum of the two mean nearest
    squared distances) and precision, recall, F1 at distance tau; also the
    two directed means (truth -> recon, recon -> truth)."""
    r2g = nearest_sq(truth, recon)      # each truth point to the reconstruction
    g2r = nearest_sq(recon, truth)
    p = float(np.mean(np.sqrt(g2r) < tau))
    r = float(np.mean(np.sqrt(r2g) < tau))
    f1 = 2 * p * r / (p + r) if p + r > 0 else 0.0
    return dict(r2g=float(r2g.mean()), g2r=float(g2r.mean()),
                cd=0.5 * float(r2g.mean() + g2r.mean()), precision=p, recall=r, f1=f1)
