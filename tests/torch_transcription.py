"""Independent PyTorch float64 transcription of the rasterizer (test helper).

A second, vectorised formulation of the same definition (paper Sec. II-A),
written without looking at the C oracle's loops: every ray against every
Gaussian as dense tensors, the front-to-back transmittance as an exclusive
cumulative sum over the globally depth-sorted Gaussians, and gradients from
autograd. Used only on tiny scenes to pin the oracle's forward and its
hand-derived backward.
"""
import math

import numpy as np
import torch


def radar_axes(phi, theta):
    """Rows of R_r(phi, theta) (Sec. II-A): azimuth, elevation, range."""
    s, c = math.sin, math.cos
    ex = [-s(phi), -c(phi), 0.0]
    ey = [-s(theta) * c(phi), s(theta) * s(phi), c(theta)]
    ez = [-c(theta) * c(phi), c(theta) * s(phi), -s(theta)]
    return [torch.tensor(e, dtype=torch.float64) for e in (ex, ey, ez)]


def _rot(q):
    q = q / q.norm(dim=1, keepdim=True)
    w, x, y, z = q.unbind(1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], 1)


def _footprint(centres, c, cov, q_max):
    """f at every (cell, Gaussian) pair; cov is (n, 2, 2)."""
    conic = torch.linalg.inv(cov)
    d = centres[:, None, :] - c[None, :, :]
    q = torch.einsum("rni,nij,rnj->rn", d, conic, d)
    eps = math.exp(-0.5 * q_max)
    f = (torch.exp(-0.5 * q) - eps) / (1 - eps)
    return torch.where(q < q_max, f, torch.zeros_like(f))


def render(means, scales, quats, amp, ext, view, q_max=9.0, shadowing=True):
    """Returns (S[H, W], A[n]) for one view; inputs float64 tensors."""
    phi, theta = view.azimuth, view.grazing
    W, H = view.img_w, view.img_h
    Wc = view.comp_w or W
    Hc = view.comp_h or H
    dA, dR = view.d_az, view.d_rg
    dAc = view.comp_d_az or dA
    dEc = view.comp_d_el or dR * math.tan(theta)
    ex, ey, ez = radar_axes(phi, theta)

    R = _rot(quats)
    M = R * scales[:, None, :]
    Sig = M @ M.transpose(1, 2)

    def plane(u, w, su, sw, cols, rows):
        B = torch.stack([u / su, w / sw], 1)          # (3, 2)
        cov = B.T[None] @ Sig @ B[None]
        c = torch.stack([means @ u / su + cols / 2, means @ w / sw + rows / 2], 1)
        yy, xx = torch.meshgrid(torch.arange(rows, dtype=torch.float64) + 0.5,
                                torch.arange(cols, dtype=torch.float64) + 0.5,
                                indexing="ij")
        centres = torch.stack([xx.reshape(-1), yy.reshape(-1)], 1)
        return _footprint(centres, c, cov, q_max)

    gC = plane(ex, ey, dAc, dEc, Wc, Hc)             # (rays, n)
    gI = plane(ex, ez, dA, dR, W, H)                 # (pixels, n)

    depth = (means.detach() @ ez).numpy()
    key = depth.astype(np.float32)
    order = torch.as_tensor(np.lexsort((np.arange(len(key)), key)))
    x = ext[order][None, :] * gC[:, order]
    alpha = 1 - torch.exp(-x)
    if shadowing:
        T = torch.exp(-(torch.cumsum(x, 1) - x))
        contrib = alpha * T
    else:
        contrib = alpha
    A = torch.zeros_like(ext).index_add(0, order, contrib.sum(0))
    S = (gI * (amp * A)[None, :]).sum(1).reshape(H, W)
    return S, A
