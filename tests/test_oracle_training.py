"""Pins of the reconstruction loop's reference steps (optimiser, densify and
prune, metrics) against closed forms, hand-worked cases and library
routines."""
import math

import numpy as np
import pytest

from oracle import training as T


# ------------------------------------------------------------------- Adam

def test_adam_constant_gradient_moves_lr_per_step():
    """With a constant gradient the bias-corrected moments are exactly g and
    g^2, so every step moves each parameter by lr * g / (|g| + eps)."""
    x = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m = np.zeros(3)
    v = np.zeros(3)
    x0 = x.copy()
    for t in range(1, 51):
        x, m, v = T.adam_step(x, g, m, v, t, lr=0.01)
    assert np.allclose(x, x0 - 50 * 0.01 * g / (np.abs(g) + 1e-15), rtol=0, atol=1e-12)


def test_adam_log_space_is_adam_on_the_logarithm():
    rng = np.random.default_rng(1)
    x = rng.uniform(0.1, 2.0, 20)
    u = np.log(x)
    mx = vx = mu = vu = np.zeros(20)
    for t in range(1, 30):
        g = rng.standard_normal(20)
        x_new, mx, vx = T.adam_step(x, g, mx, vx, t, lr=0.05, log_space=True)
        u, mu, vu = T.adam_step(u, g * x, mu, vu, t, lr=0.05)   # chain rule d/du = x d/dx
        x = x_new
        assert np.allclose(np.log(x), u, rtol=0, atol=1e-12)
    assert np.all(x > 0)


def test_adam_clamp_bounds_the_result():
    x, m, v = np.array([1.0, 5.0, 49.9]), np.zeros(3), np.zeros(3)
    for t in range(1, 200):
        x, m, v = T.adam_step(x, -np.ones(3), m, v, t, lr=0.1, log_space=True, lo=1e-6, hi=50.0)
    assert np.all(x == 50.0)
    y, _, _ = T.adam_step(np.array([2.0]), np.array([1.0]), np.zeros(1), np.zeros(1), 1, lr=0.5,
                          lo=1.8, hi=3.0)
    assert y[0] == 1.8
    z, _, _ = T.adam_step(np.array([2.0]), np.array([1.0]), np.zeros(1), np.zeros(1), 1, lr=0.5)
    assert math.isclose(z[0], 1.5)


def test_adam_converges_on_a_quadratic():
    x, m, v = np.array([3.0, -1.5]), np.zeros(2), np.zeros(2)
    a = np.array([2.0, 0.5])
    for t in range(1, 3001):
        x, m, v = T.adam_step(x, a * x, m, v, t, lr=0.01)
    assert np.all(np.abs(x) < 1e-2)


# ------------------------------------------------------ densify and prune

def _case():
    """Six hand-made Gaussians, one per decision path."""
    ident = [1.0, 0.0, 0.0, 0.0]
    c, s = math.cos(math.pi / 4), math.sin(math.pi / 4)
    rot_z90 = [c, 0.0, 0.0, s]
    params = dict(
        means=np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0], [3, 0, 0], [4, 0, 0], [5, 0, 0]],
                       np.float64),
        scales=np.array([[0.05] * 3, [0.5, 0.1, 0.1], [0.05, 0.04, 0.03],
                         [0.2, 0.1, 0.1], [0.05] * 3, [0.3, 0.1, 0.1]]),
        quats=np.array([ident, ident, ident, rot_z90, ident, ident]),
        ext=np.array([0.001, 2.0, 2.0, 2.0, 2.0, 2.0]),
        amp=np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0]))
    acc = np.array([1.0, 1.0, 0.01, 0.004, 0.002, 0.0])
    cnt = np.array([1, 1, 2, 1, 1, 0])
    gdir = np.array([[0, 0, 1], [0, 0, 1], [0, 0, 2.0], [0, 3.0, 0], [1, 0, 0], [0, 0, 0]])
    moments = {k: (np.full_like(p, 0.5), np.full_like(p, 0.25)) for k, p in params.items()}
    return params, moments, acc, cnt, gdir


def test_densify_hand_worked_cases():
    """Prune by extinction, prune by radius, clone, split (rotated, so the
    largest axis is y), keep below the threshold, keep without gradient."""
    params, moments, acc, cnt, gdir = _case()
    cfg = T.DensifyConfig(grad_threshold=0.003, split_scale=0.1, max_radius=1.0,
                          kappa_min=0.005)
    out, mom, act = T.densify(params, moments, acc, cnt, gdir, cfg)
    assert list(act) == [T.PRUNE, T.PRUNE, T.CLONE, T.SPLIT, T.KEEP, T.KEEP]
    want_means = [[2, 0, 0], [2, 0, -0.05],
                  [3, 0.2, 0], [3, -0.2, 0], [4, 0, 0], [5, 0, 0]]
    # split children shifted against the gradient (+y) by their largest std
    want_means[2][1] -= 0.2 / 1.6
    want_means[3][1] -= 0.2 / 1.6
    assert np.allclose(out["means"], want_means, atol=1e-15)
    assert np.allclose(out["scales"][2], [0.2 / 1.6, 0.1 / 1.6, 0.1 / 1.6])
    assert np.allclose(out["scales"][1], params["scales"][2])
    assert list(out["amp"]) == [3.0, 3.0, 4.0, 4.0, 5.0, 6.0]
    fresh = [False, True, True, True, False, False]
    for k, (m, v) in mom.items():
        for row, f in zip(range(len(fresh)), fresh):
            assert np.all(m[row] == (0.0 if f else 0.5)) and np.all(v[row] == (0.0 if f else 0.25))


def test_densify_thresholds_are_inclusive_and_fp32():
    """The mean gradient reaching the threshold exactly densifies; the
    decision is taken on FP32 values."""
    f = np.float32
    scales = np.full((3, 3), 0.05)
    ext = np.full(3, 1.0)
    thr = f(0.003)
    acc = np.array([thr, np.nextafter(thr, f(0)), 2 * thr], np.float64)
    cnt = np.array([1, 1, 2])
    act = T.densify_actions(scales, ext, acc, cnt, T.DensifyConfig(grad_threshold=0.003))
    assert list(act) == [T.CLONE, T.KEEP, T.CLONE]


def test_rotation_of_unit_quaternions():
    rng = np.random.default_rng(3)
    for _ in range(20):
        q = rng.standard_normal(4)
        R = T._rotation(q)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-12) and np.isclose(np.linalg.det(R), 1.0)
        # the rotation of q sends v to q v q*
        w, x, y, z = q / np.linalg.norm(q)
        v = rng.standard_normal(3)
        qv = np.array([-x * v[0] - y * v[1] - z * v[2], w * v[0] + y * v[2] - z * v[1],
                       w * v[1] + z * v[0] - x * v[2], w * v[2] + x * v[1] - y * v[0]])
        rot = np.array([qv[1] * w - qv[0] * x - qv[2] * z + qv[3] * y,
                        qv[2] * w - qv[0] * y - qv[3] * x + qv[1] * z,
                        qv[3] * w - qv[0] * z - qv[1] * y + qv[2] * x])
        assert np.allclose(R @ v, rot, atol=1e-12)


# ----------------------------------------------------------------- metrics

def test_psnr_closed_form():
    ref = np.zeros((8, 8))
    ref[0, 0] = 1.0
    assert math.isclose(T.psnr(ref + 0.1, ref), 20.0, rel_tol=1e-12)
    assert T.psnr(ref, ref) == math.inf


def test_ssim_identity_constants_and_symmetry():
    rng = np.random.default_rng(4)
    x = rng.uniform(0, 1, (16, 14))
    y = rng.uniform(0, 1, (16, 14))
    assert math.isclose(T.ssim(x, x, 1.0), 1.0, rel_tol=1e-12)
    assert math.isclose(T.ssim(x, y, 1.0), T.ssim(y, x, 1.0), rel_tol=1e-12)
    a, b, L = 0.3, 0.7, 1.0
    c1 = (0.01 * L) ** 2
    want = (2 * a * b + c1) / (a * a + b * b + c1)
    assert math.isclose(T.ssim(np.full((12, 12), a), np.full((12, 12), b), L), want,
                        rel_tol=1e-12)


def test_ssim_matches_separable_gaussian_filtering():
    """The windowed statistics computed by scipy's separable Gaussian filter
    (radius 5, normalised), over the positions where the window fits."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 2, (24, 20))
    y = x + 0.3 * rng.standard_normal((24, 20))
    L = 2.0
    filt = lambda a: gaussian_filter(a, 1.5, truncate=5 / 1.5, mode="constant")[5:-5, 5:-5]
    mx, my = filt(x), filt(y)
    vx, vy, cxy = filt(x * x) - mx * mx, filt(y * y) - my * my, filt(x * y) - mx * my
    c1, c2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    want = ((2 * mx * my + c1) * (2 * cxy + c2) / ((mx ** 2 + my ** 2 + c1) * (vx + vy + c2))).mean()
    assert math.isclose(T.ssim(x, y, L), want, rel_tol=1e-10)


def test_chamfer_and_f1_closed_forms_and_kdtree():
    from scipy.spatial import cKDTree
    a = np.array([[0.0, 0.0, 0.0]])
    r = T.chamfer_f1(a + [0.3, 0.0, 0.4], a, tau=0.6)
    assert math.isclose(r["cd"], 0.25, rel_tol=1e-12) and r["f1"] == 1.0
    r = T.chamfer_f1(a + [0.3, 0.0, 0.4], a, tau=0.5)      # distance exactly tau: not matched
    assert r["precision"] == 0.0 and r["f1"] == 0.0
    rng = np.random.default_rng(6)
    P, Q = rng.standard_normal((700, 3)), rng.standard_normal((500, 3))
    assert np.allclose(T.nearest_sq(P, Q), cKDTree(Q).query(P)[0] ** 2, rtol=1e-12, atol=0)
    r = T.chamfer_f1(P, Q, 0.2)
    dq = cKDTree(P).query(Q)[0]
    dp = cKDTree(Q).query(P)[0]
    assert math.isclose(r["cd"], 0.5 * ((dq ** 2).mean() + (dp ** 2).mean()), rel_tol=1e-12)
    assert r["precision"] == np.mean(dp < 0.2) and r["recall"] == np.mean(dq < 0.2)
    same = T.chamfer_f1(P, P, 1e-9)
    assert same["cd"] == 0.0 and same["f1"] == 1.0
