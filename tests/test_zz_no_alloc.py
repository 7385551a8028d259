"""The forward entry point that allocates nothing (its workspace is a static
device array of the library) against the ordinary forward with caller-owned
workspaces and against the FP64 oracle, on two calls in a row, the second
with a smaller problem; a problem larger than the static workspace is
refused before any forward work."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2506_21633_amd import _capi as C
from paper_2506_21633_amd import scenes

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-4      # FP32 image against the FP64 oracle (max-normalised)
SAME_TOL = 1e-6     # against the ordinary forward (float atomics order only)


def _scene(seed, n, half):
    rng = scenes.make_rng(seed)
    return scenes.Scene(rng.uniform(-half, half, (n, 3)).astype(np.float32),
                        np.exp(rng.uniform(np.log(0.03), np.log(0.25), (n, 3))).astype(np.float32),
                        scenes.random_quats(rng, n),
                        rng.uniform(0.2, 1.0, n).astype(np.float32),
                        rng.uniform(1.0, 4.0, n).astype(np.float32))


def static_forward(r, cuda):
    from paper_2506_21633_amd import api
    images = torch.full((max(int(r.image_floats), 1),), float("nan"), dtype=torch.float32,
                        device=cuda)
    for k, (off, h, w) in enumerate(r.shapes):
        images[off:off + h * w] = 0.0
    rc = r.lib.sdgr_forward_static(r.scenes_c, len(r.scenes), r.views_c, r.nv,
                                   ctypes.byref(r.opts_c), images.data_ptr(),
                                   api._stream_ptr(cuda))
    return rc, images


def check_against_plain_and_oracle(sc, views, cuda):
    from paper_2506_21633_amd import api
    r = api.Renderer([api.GaussianTensors.from_numpy(sc, cuda)], views)
    rc, img_static = static_forward(r, cuda)
    C.check(rc)
    plain = r.forward()
    torch.cuda.synchronize()
    r.status(plain)
    _, _, S_ref = oracle.forward(sc, views)
    for v, (off, h, w) in enumerate(r.shapes):
        a = img_static[off:off + h * w].view(h, w).cpu().numpy()
        b = plain.image(v).cpu().numpy()
        assert np.isfinite(a).all()
        scale = max(np.abs(b).max(), 1e-30)
        assert np.abs(a - b).max() <= SAME_TOL * scale, v
        assert np.abs(a - S_ref[v]).max() <= IMG_TOL * np.abs(S_ref[v]).max(), v


def test_static_forward_two_calls_then_smaller(cuda):
    big = _scene(71, 4000, 1.5)
    big_views = [scenes.View.from_degrees(30.0 * k, 35.0 + 5 * k, 96, 0.06) for k in range(3)]
    check_against_plain_and_oracle(big, big_views, cuda)
    small = _scene(72, 500, 0.5)
    small_views = [scenes.View(azimuth=1.1, grazing=0.6, img_w=40, img_h=24, d_az=0.05,
                               d_rg=0.06)]
    check_against_plain_and_oracle(small, small_views, cuda)


def test_static_forward_refuses_oversized_problem(cuda):
    from paper_2506_21633_amd import api
    sc = scenes.vehicle(303, 200_000)
    views = scenes.vehicle_views(count=8)
    r = api.Renderer([api.GaussianTensors.from_numpy(sc, cuda)], views)
    rc, img = static_forward(r, cuda)
    assert rc == C.SDGR_EUNSUPPORTED
    assert "static workspace" in r.lib.sdgr_last_error().decode()
    torch.cuda.synchronize()
    # nothing was rendered: the images keep what the caller wrote
    for off, h, w in r.shapes:
        assert float(img[off:off + h * w].abs().sum()) == 0.0
