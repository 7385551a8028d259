"""Parity of the HIP path with the FP64 oracle for the phase-function and
extinction inputs: a spherical-harmonics phase function evaluated at the
direction from each Gaussian to the radar (plane wave and radars at finite
range), separate forward and backward extinctions, and intensities
normalised by the computation-plane cell area.

Bars as for the long lists (element by element, FP32 kernels against the
FP64 oracle): A and images within 2e-5 of their per-view maximum; every
gradient component within 1e-4 of its group's largest magnitude (1e-2 for
the rare Gaussians with a cell within rounding of the footprint cutoff,
where the cutoff's derivative jump makes the boundary term depend on the
precision), cosine >= 0.9999 per group. The SH basis in FP32 adds ~1e-7
relative error per evaluation and the direction's normalisation another
~1e-7, well inside them.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2506_21633_amd import scenes
from tests.test_gpu_deep_lists import (A_ELEM, EDGE_FRACTION, GRAD_COS, GRAD_EDGE, GRAD_ELEM,
                                       IMG_ELEM, cosine, elem_err, near_cutoff)

pytestmark = pytest.mark.gpu


def api():
    from paper_2506_21633_amd import api as _api
    return _api


def phase_scene(seed, n=3000, deg=3, half=1.5, ext_back=True, smin=0.03, smax=0.18):
    rng = scenes.make_rng(seed)
    sc = scenes.Scene(
        rng.uniform(-half, half, (n, 3)).astype(np.float32),
        np.exp(rng.uniform(math.log(smin), math.log(smax), (n, 3))).astype(np.float32),
        scenes.random_quats(rng, n),
        rng.uniform(0.2, 1.0, n).astype(np.float32),
        rng.uniform(0.5, 3.0, n).astype(np.float32))
    if deg is not None:
        sh = rng.normal(0.0, 0.3, (n, (deg + 1) ** 2))
        sh[:, 0] += 2.0
        sc.sh = sh.astype(np.float32)
    if ext_back:
        sc.ext_back = rng.uniform(0.2, 1.5, n).astype(np.float32)
    return sc


def views_with_ranges(ranges, w=70, h=52, spacing=0.06):
    out = []
    for k, rr in enumerate(ranges):
        v = scenes.View.from_degrees(15.0 + 47.0 * k, 35.0 + 7.0 * (k % 3), w, spacing,
                                     radar_range=rr)
        v.img_h = h
        out.append(v)
    return out


def groups_of(scene):
    names = ["means", "scales", "quats", "ext"]
    names.append("sh" if scene.sh is not None else "amp")
    if scene.ext_back is not None:
        names.append("ext_back")
    return names


def run(scene_list, views, Gs, options, cuda):
    """Forward + backward of all views in one launch; per-view images, A
    [V, n_scene], gradients per scene."""
    A_ = api()
    gts = [A_.GaussianTensors.from_numpy(s, cuda) for s in scene_list]
    r = A_.Renderer(gts, views, options)
    res = r.forward()
    flat = np.zeros(int(res.plan.image_floats), np.float32)
    for v, Gv in enumerate(Gs):
        off, h, w = res.shapes[v]
        flat[off:off + h * w] = np.asarray(Gv, np.float32).ravel()
    grads = r.backward(res, torch.as_tensor(flat, device=cuda))
    torch.cuda.synchronize()
    r.status(res)
    A = r.intensity_shares(res).cpu().numpy()
    Av, off = [], 0
    for v in views:
        n = scene_list[v.scene].n
        Av.append(A[off:off + n])
        off += n
    return dict(images=[res.image(v).cpu().numpy() for v in range(len(views))], A=Av,
                grads=[{k: t.cpu().numpy() for k, t in d.items()} for d in grads],
                plan=res.plan)


def compare(scene, views, Gs, out_images, out_A, out_grads, cell_area, shadowing=True):
    report = {}
    A_ref, _, S_ref = oracle.forward(scene, views, cell_area=cell_area, shadowing=shadowing)
    for v in range(len(views)):
        report[f"A{v}"] = elem_err(out_A[v], A_ref[v])
        report[f"S{v}"] = elem_err(out_images[v], S_ref[v])
    ref, auxes = oracle.backward(scene, views, Gs, cell_area=cell_area, shadowing=shadowing)
    edge, used = near_cutoff(auxes)
    report["edge"] = (int(edge.sum()), int(used.sum()))
    for k in groups_of(scene):
        a, b = out_grads[k], ref[k]
        scale = max(np.abs(b).max(), 1e-300)
        per = np.abs(a - b).reshape(scene.n, -1).max(axis=1) / scale
        report[k] = (float(per[~edge].max(initial=0.0)), float(per[edge].max(initial=0.0)),
                     cosine(a, b))
    if scene.sh is not None and "amp" in out_grads:
        assert np.all(out_grads["amp"] == 0.0)
    return report


def check(report):
    ne, nu = report["edge"]
    assert ne <= EDGE_FRACTION * max(nu, 1), report["edge"]
    for k, val in report.items():
        if k == "edge":
            continue
        if k[0] in "AS" and k[1:].isdigit():
            assert val <= (A_ELEM if k[0] == "A" else IMG_ELEM), (k, val)
        else:
            assert val[0] <= GRAD_ELEM and val[1] <= GRAD_EDGE and val[2] >= GRAD_COS, (k, val)


@pytest.mark.parametrize("mode", ["stored", "recompute", "deterministic"])
@pytest.mark.parametrize("cell_area", [False, True])
def test_sh_phase_and_split_extinction(cuda, mode, cell_area):
    """Degree-3 SH phase functions and separate extinctions on three views
    (a plane wave, radars 25 m and 400 m away) of ragged 70 x 52 images."""
    sc = phase_scene(501)
    views = views_with_ranges([0.0, 25.0, 400.0])
    rng = scenes.make_rng(502)
    Gs = [rng.standard_normal((v.img_h, v.img_w)) for v in views]
    opt = api().RenderOptions(recompute=mode == "recompute",
                              deterministic=mode == "deterministic", cell_area=cell_area)
    out = run([sc], views, Gs, opt, cuda)
    assert out["plan"].sh_coeffs == 16
    report = compare(sc, views, Gs, out["images"], out["A"], out["grads"][0], cell_area)
    print(f"\nsh mode={mode} cell_area={cell_area}: {report}")
    check(report)
    assert np.array_equal(out["grads"][0]["ext"], out["grads"][0]["ext_back"])


@pytest.mark.parametrize("deg", [0, 1, 2])
def test_lower_sh_degrees_without_shadowing(cuda, deg):
    sc = phase_scene(510 + deg, n=2000, deg=deg, ext_back=False)
    views = views_with_ranges([12.0, 0.0], w=64, h=64)
    rng = scenes.make_rng(520 + deg)
    Gs = [rng.standard_normal((v.img_h, v.img_w)) for v in views]
    out = run([sc], views, Gs, api().RenderOptions(shadowing=False), cuda)
    report = compare(sc, views, Gs, out["images"], out["A"], out["grads"][0], False,
                     shadowing=False)
    print(f"\nsh degree {deg}: {report}")
    check(report)


def test_mixed_scenes_many_views(cuda):
    """A scene with a degree-2 expansion and one with the scalar amplitude
    and a single extinction in one launch of 10 views (more than one group
    of views in the parameter adjoint, whose parts then hold the larger
    scene's coefficient count for both)."""
    sh_scene = phase_scene(530, n=1500, deg=2)
    plain = phase_scene(531, n=1800, deg=None, ext_back=False)
    views = []
    for k in range(10):
        v = scenes.View.from_degrees(36.0 * k, 30.0 + 3.0 * k, 40, 0.08,
                                     radar_range=0.0 if k % 3 == 0 else 20.0 + 10.0 * k)
        v.scene = k % 2
        views.append(v)
    rng = scenes.make_rng(532)
    Gs = [rng.standard_normal((40, 40)) for _ in views]
    out = run([sh_scene, plain], views, Gs, api().RenderOptions(cell_area=True), cuda)
    assert out["plan"].sh_coeffs == 9
    for s, sc in enumerate((sh_scene, plain)):
        ids = [k for k, v in enumerate(views) if v.scene == s]
        report = compare(sc, [views[k] for k in ids], [Gs[k] for k in ids],
                         [out["images"][k] for k in ids], [out["A"][k] for k in ids],
                         out["grads"][s], True)
        print(f"\nmixed scene {s}: {report}")
        check(report)


def test_degree0_matches_scalar_amplitude(cuda):
    """c_00 = P / Y_00 renders the scalar-amplitude images to FP32 rounding."""
    sc = phase_scene(540, n=2000, deg=None, ext_back=False)
    sh = sc.copy()
    sh.sh = (sc.amp / (0.5 / math.sqrt(math.pi)))[:, None].astype(np.float32)
    views = views_with_ranges([30.0, 0.0], w=64, h=64)
    rng = scenes.make_rng(541)
    Gs = [rng.standard_normal((64, 64)) for _ in views]
    a = run([sc], views, Gs, api().RenderOptions(), cuda)
    b = run([sh], views, Gs, api().RenderOptions(), cuda)
    for v in range(len(views)):
        assert elem_err(b["images"][v], a["images"][v]) <= 1e-6
    for k in ("means", "scales", "quats", "ext"):
        assert elem_err(b["grads"][0][k], a["grads"][0][k]) <= 1e-5, k


def test_autograd_with_sh_and_split_extinction(cuda):
    """render() returns the same images and gradients as the renderer and
    fills the grads of ext_back and sh (amp None)."""
    A_ = api()
    sc = phase_scene(550, n=1500, deg=3)
    views = views_with_ranges([15.0, 15.0], w=48, h=48)
    g = A_.GaussianTensors.from_numpy(sc, cuda)
    leaves = {k: t.clone().requires_grad_(True) for k, t in g.named().items() if k != "amp"}
    imgs = A_.render(leaves["means"], leaves["scales"], leaves["quats"], None, leaves["ext"],
                     views, ext_back=leaves["ext_back"], sh=leaves["sh"])
    rng = scenes.make_rng(551)
    Gs = [rng.standard_normal((48, 48)) for _ in views]
    Gt = torch.as_tensor(np.stack(Gs), dtype=torch.float32, device=cuda)
    (imgs * Gt).sum().backward()
    g_noamp = A_.GaussianTensors(g.means, g.scales, g.quats, None, g.ext, g.ext_back, g.sh)
    r = A_.Renderer([g_noamp], views)
    res = r.forward()
    d = r.backward(res, Gt.reshape(-1).contiguous())[0]
    assert "amp" not in d
    assert torch.allclose(imgs.detach(), res.stacked(), rtol=1e-5, atol=1e-6)
    for k, t in leaves.items():
        assert torch.allclose(t.grad, d[k], rtol=1e-5, atol=1e-6 * float(d[k].abs().max())), k
