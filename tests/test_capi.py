"""Host-side checks of the C ABI (no GPU compute): the library loads, exports
every function include/*.h declares, its structs match the headers'
layout, and argument validation rejects bad input before any device work."""
import ctypes
import math
import os
import re
import subprocess

import pytest

from paper_2506_21633_amd import _capi as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sdgr.h")
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(sdgr_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_function():
    L = C.lib()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(C.EXPORTED)
    assert L.sdgr_version() == 1


def test_struct_layout_matches_header(tmp_path):
    layouts = [("sdgr_view", C.View), ("sdgr_plan", C.Plan), ("sdgr_options", C.Options),
               ("sdgr_scene", C.Scene), ("sdgr_scene_grad", C.SceneGrad),
               ("sdgr_param_group", C.ParamGroup), ("sdgr_adam_config", C.AdamConfig),
               ("sdgr_densify_config", C.DensifyConfig), ("sdgr_gaussian_set", C.GaussianSet)]
    fields = [("sdgr_view", "img_w", C.View), ("sdgr_view", "radar_range", C.View),
              ("sdgr_plan", "records", C.Plan), ("sdgr_plan", "sh_coeffs", C.Plan),
              ("sdgr_scene", "sh_stride", C.Scene), ("sdgr_param_group", "lr", C.ParamGroup),
              ("sdgr_gaussian_set", "sh_coeffs", C.GaussianSet)]
    exprs = [f"sizeof({n})" for n, _ in layouts] + [f"offsetof({n}, {f})" for n, f, _ in fields]
    src = tmp_path / "sizes.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "sdgr_train.h"\n'
                   'int main(void){' +
                   "".join(f'printf("%zu\\n", (size_t){e});' for e in exprs) + '}\n')
    exe = tmp_path / "sizes"
    subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(t) for _, t in layouts] + \
        [getattr(t, f).offset for _, f, t in fields]
    assert got == want


def test_default_options():
    o = C.Options()
    C.lib().sdgr_default_options(ctypes.byref(o))
    assert (o.shadowing, o.recompute, o.q_max, o.tau_max, o.dilation, o.deterministic, o.tile,
            o.cell_area, o.reserved) == (1, 0, 9.0, 16.0, 0.0, 0, 0, 0, 0)


def _args(grazing=math.radians(45), nv=1, n=10, q_max=9.0, scene=0, w=64, sh_degree=None,
          amp=0x1000, radar_range=0.0, cell_area=0, sh_stride=0):
    sc = (C.Scene * 1)(C.Scene(n, 0x1000, 0x1000, 0x1000, amp, 0x1000))
    if sh_degree is not None:
        sc[0].sh, sc[0].sh_degree = 0x1000, sh_degree
    sc[0].sh_stride = sh_stride
    views = (C.View * max(nv, 1))()
    for v in views:
        v.azimuth, v.grazing, v.d_az, v.d_rg = 0.0, grazing, 0.1, 0.1
        v.img_w, v.img_h, v.scene = w, 64, scene
        v.radar_range = radar_range
    o = C.Options()
    C.lib().sdgr_default_options(ctypes.byref(o))
    o.q_max = q_max
    o.cell_area = cell_area
    return sc, views, o


@pytest.mark.parametrize("kw,code", [
    (dict(grazing=0.0), C.SDGR_EINVAL),
    (dict(grazing=math.pi / 2), C.SDGR_EINVAL),
    (dict(nv=0), C.SDGR_EINVAL),
    (dict(n=-1), C.SDGR_EINVAL),
    (dict(q_max=0.0), C.SDGR_EINVAL),
    (dict(q_max=float("nan")), C.SDGR_EINVAL),
    (dict(scene=3), C.SDGR_EINVAL),
    (dict(w=0), C.SDGR_EINVAL),
    (dict(w=8 * 70000), C.SDGR_EUNSUPPORTED),
    (dict(sh_degree=4), C.SDGR_EUNSUPPORTED),
    (dict(sh_degree=-1), C.SDGR_EUNSUPPORTED),
    (dict(amp=0), C.SDGR_EINVAL),
    (dict(radar_range=-1.0), C.SDGR_EINVAL),
    (dict(radar_range=float("inf")), C.SDGR_EINVAL),
    (dict(cell_area=2), C.SDGR_EINVAL),
    (dict(sh_degree=2, sh_stride=8), C.SDGR_EINVAL),
])
def test_plan_query_rejects_bad_arguments(kw, code):
    L = C.lib()
    sc, views, o = _args(**kw)
    nv = kw.get("nv", 1)
    plan = C.Plan()
    rc = L.sdgr_plan_query(sc, 1, views, nv, ctypes.byref(o), None, 0, None,
                           ctypes.byref(plan))
    assert rc == code
    assert L.sdgr_last_error()


def test_sh_scene_needs_no_amplitude():
    """With an SH phase function amp may be NULL: validation passes and the
    query stops only at its missing scratch."""
    L = C.lib()
    sc, views, o = _args(sh_degree=3, amp=0, radar_range=50.0, cell_area=1)
    plan = C.Plan()
    rc = L.sdgr_plan_query(sc, 1, views, 1, ctypes.byref(o), None, 0, None, ctypes.byref(plan))
    assert rc == C.SDGR_EWORKSPACE


@pytest.mark.parametrize("missing", ["d_sh", "d_ext_back"])
def test_backward_needs_gradients_of_the_optional_inputs(missing):
    L = C.lib()
    sc, views, o = _args(sh_degree=2, amp=0)
    sc[0].ext_back = 0x1000
    p = _host_plan(10, 1, 64)
    p.sh_coeffs = 9
    C.check(L.sdgr_plan_resize(ctypes.byref(p), 100, 100))
    g = C.SceneGrad(0x1000, 0x1000, 0x1000, 0, 0x1000, 0x1000, 0x1000)
    setattr(g, missing, 0)
    rc = L.sdgr_backward(sc, 1, views, 1, ctypes.byref(o), ctypes.byref(p), 0x1000, 0x1000,
                         0x1000, (C.SceneGrad * 1)(g), None)
    assert rc == C.SDGR_EINVAL and b"gradient" in L.sdgr_last_error()


def test_plan_must_carry_the_sh_coefficient_count():
    L = C.lib()
    sc, views, o = _args(sh_degree=1)
    p = _host_plan(10, 1, 64)
    C.check(L.sdgr_plan_resize(ctypes.byref(p), 100, 100))   # sh_coeffs 0: no SH scene
    rc = L.sdgr_forward(sc, 1, views, 1, ctypes.byref(o), ctypes.byref(p), 0x1000, 0x1000,
                        0x1000, None)
    assert rc == C.SDGR_EINVAL and b"plan" in L.sdgr_last_error()


def test_sh_plans_hold_the_coefficient_parts():
    """More than one group of views (40 views: at least two groups of up to
    16): the parameter-gradient parts grow by the coefficient count per
    Gaussian and group."""
    L = C.lib()
    got = []
    for shc in (0, 16):
        p = _host_plan(100_000, 40, 256)
        p.sh_coeffs = shc
        C.check(L.sdgr_plan_resize(ctypes.byref(p), 1_000_000, 1_000_000))
        got.append(p.bwd_scratch_bytes)
    assert got[1] - got[0] >= 2 * 16 * 4 * 100_000


def test_plan_query_needs_scratch():
    L = C.lib()
    sc, views, o = _args()
    plan = C.Plan()
    rc = L.sdgr_plan_query(sc, 1, views, 1, ctypes.byref(o), None, 0, None, ctypes.byref(plan))
    assert rc == C.SDGR_EWORKSPACE
    assert b"scratch" in L.sdgr_last_error()


def test_forward_rejects_mismatched_plan():
    L = C.lib()
    sc, views, o = _args()
    plan = C.Plan()
    plan.records, plan.nviews, plan.nscenes, plan.tile = 999, 1, 1, 8
    rc = L.sdgr_forward(sc, 1, views, 1, ctypes.byref(o), ctypes.byref(plan), 0x1000, 0x1000,
                        0x1000, None)
    assert rc == C.SDGR_EINVAL
    assert b"plan" in L.sdgr_last_error()


def test_query_bytes_small_and_monotone():
    L = C.lib()
    a, b = L.sdgr_query_bytes(1, 1), L.sdgr_query_bytes(8, 512)
    assert 0 < a <= b < 1 << 20


def _host_plan(n, nv, size, recompute=0):
    """A plan as sdgr_plan_query would fill it for one scene of n Gaussians
    and nv views of size x size (counts only; host-side)."""
    p = C.Plan()
    tiles = ((size + 7) // 8) ** 2
    p.records, p.gaussians, p.nviews, p.nscenes, p.tile = n * nv, n, nv, 1, 8
    p.tiles_c = p.tiles_i = nv * tiles
    p.rays = nv * size * size
    p.recompute = recompute
    p.image_floats = nv * size * size
    return p


@pytest.mark.parametrize("recompute", [0, 1])
def test_plan_resize_keeps_parameter_gradient_scratch(recompute):
    """A resized plan's backward scratch must hold the per-view-group parts
    of the parameter gradients (they grow with the Gaussian count once there
    is more than one group of views), as the query's own plan does."""
    L = C.lib()
    sizes = []
    for n in (1000, 2_000_000):
        p = _host_plan(n, 32, 1024, recompute)
        p.records = 32 * 2_000_000   # same records: only the Gaussian count differs
        C.check(L.sdgr_plan_resize(ctypes.byref(p), 5_000_000, 4_000_000))
        sizes.append(p.bwd_scratch_bytes)
        again = C.Plan()
        ctypes.pointer(again)[0] = p
        C.check(L.sdgr_plan_resize(ctypes.byref(again), 5_000_000, 4_000_000))
        assert again.bwd_scratch_bytes == p.bwd_scratch_bytes
    # 32 views, at least two groups: at least 2 x 12 floats per extra Gaussian
    assert sizes[1] - sizes[0] >= 2 * 12 * 4 * (2_000_000 - 1000)


def test_forward_rejects_plan_with_short_workspaces():
    L = C.lib()
    sc, views, o = _args()
    p = _host_plan(10, 1, 64)
    C.check(L.sdgr_plan_resize(ctypes.byref(p), 100, 100))
    p.bwd_scratch_bytes -= 256
    rc = L.sdgr_backward(sc, 1, views, 1, ctypes.byref(o), ctypes.byref(p), 0x1000, 0x1000,
                         0x1000, (C.SceneGrad * 1)(C.SceneGrad(0x1000, 0x1000, 0x1000, 0x1000,
                                                               0x1000)), None)
    assert rc == C.SDGR_EWORKSPACE


def test_plan_stored_hit_stream():
    """The stream in which the forward keeps each tile's used hits for the
    backward: 8 bytes per computation-plane pair plus 16 MiB by default, none
    in recompute or deterministic mode; a caller may lower it (down to 0)
    but not make it negative or larger than its state holds; a resize takes
    the default for the new capacities."""
    L = C.lib()
    sc, views, o = _args(nv=3)
    p = C.Plan()
    C.check(L.sdgr_plan_host(sc, 1, views, 3, ctypes.byref(o), 5000, 700, ctypes.byref(p)))
    assert p.hit_bytes == 8 * 5000 + (16 << 20)

    def forward_rc(plan):   # stops at the null workspaces once the plan is accepted
        return L.sdgr_forward(sc, 1, views, 3, ctypes.byref(o), ctypes.byref(plan), None, None,
                              None, None)
    q = C.Plan()
    for hb, rc in ((0, C.SDGR_EINVAL), (4096, C.SDGR_EINVAL), (-16, C.SDGR_EINVAL),
                   (p.hit_bytes + (1 << 30), C.SDGR_EWORKSPACE)):
        ctypes.pointer(q)[0] = p
        q.hit_bytes = hb
        assert forward_rc(q) == rc, hb
        assert (b"workspace" in L.sdgr_last_error()) == (hb >= 0), hb
    C.check(L.sdgr_plan_resize(ctypes.byref(p), 10000, 700))
    assert p.hit_bytes == 8 * 10000 + (16 << 20)
    for field in ("recompute", "deterministic"):
        _, _, o2 = _args(nv=3)
        setattr(o2, field, 1)
        C.check(L.sdgr_plan_host(sc, 1, views, 3, ctypes.byref(o2), 5000, 700, ctypes.byref(q)))
        assert q.hit_bytes == 0, field


# ---------------------------------------------------- reconstruction loop

def test_adam_rejects_bad_arguments():
    L = C.lib()
    cfg = C.AdamConfig(0.9, 0.999, 1e-15, 0)
    g = (C.ParamGroup * 1)(C.ParamGroup(0x1000, 0x1000, 0x1000, 0x1000, 10, 0.1, 0, 0.0, 0.0, 0))
    assert L.sdgr_adam_step(g, 1, 0, ctypes.byref(cfg), None) == C.SDGR_EINVAL
    bad = C.AdamConfig(1.0, 0.999, 1e-15, 0)
    assert L.sdgr_adam_step(g, 1, 1, ctypes.byref(bad), None) == C.SDGR_EINVAL
    assert L.sdgr_adam_step(g, C.ADAM_MAX_GROUPS + 1, 1, ctypes.byref(cfg), None) == C.SDGR_EINVAL
    nul = (C.ParamGroup * 1)(C.ParamGroup(0x1000, 0, 0x1000, 0x1000, 10, 0.1, 0, 0.0, 0.0, 0))
    assert L.sdgr_adam_step(nul, 1, 1, ctypes.byref(cfg), None) == C.SDGR_EINVAL
    nan = (C.ParamGroup * 1)(C.ParamGroup(0x1000, 0x1000, 0x1000, 0x1000, 10, 0.1, 0,
                                          float("nan"), 1.0, 0))
    assert L.sdgr_adam_step(nan, 1, 1, ctypes.byref(cfg), None) == C.SDGR_EINVAL
    res = (C.ParamGroup * 1)(C.ParamGroup(0x1000, 0x1000, 0x1000, 0x1000, 10, 0.1, 0, 0, 0, 1))
    assert L.sdgr_adam_step(res, 1, 1, ctypes.byref(cfg), None) == C.SDGR_EINVAL
    empty = (C.ParamGroup * 1)(C.ParamGroup(0, 0, 0, 0, 0, 0.1, 0))
    assert L.sdgr_adam_step(empty, 1, 1, ctypes.byref(cfg), None) == C.SDGR_OK


def _set(**kw):
    s = C.GaussianSet()
    for g in ("means", "scales", "quats", "ext"):
        for pre in ("", "m_", "v_"):
            setattr(s, pre + g, 0x1000)
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def test_densify_rejects_bad_arguments():
    L = C.lib()
    cfg = C.DensifyConfig(0.003, 0.1, 1.0, 0.005, 1.6, 0)
    n = 1000
    ws = L.sdgr_densify_workspace_bytes(n)
    assert ws >= n
    a, b = _set(), _set()
    def call(inp=a, out=b, cap=2 * n, c=cfg, wsb=ws, work=0x1000):
        return L.sdgr_densify(ctypes.byref(inp), n, 0x1000, 0x1000, 0x1000, ctypes.byref(c),
                              ctypes.byref(out), cap, 0x1000, work, wsb, None)
    assert call(cap=2 * n - 1) == C.SDGR_EINVAL
    assert call(wsb=ws - 1) == C.SDGR_EWORKSPACE
    assert call(work=0x1010) == C.SDGR_EINVAL
    assert call(c=C.DensifyConfig(0.003, 0.1, 1.0, 0.005, 1.0, 0)) == C.SDGR_EINVAL
    assert call(out=_set(amp=0x1000, m_amp=0x1000, v_amp=0x1000)) == C.SDGR_EINVAL
    assert call(inp=_set(m_means=0)) == C.SDGR_EINVAL
    assert call(inp=_set(sh=0x1000, m_sh=0x1000, v_sh=0x1000, sh_coeffs=16),
                out=_set(sh=0x1000, m_sh=0x1000, v_sh=0x1000, sh_coeffs=9)) == C.SDGR_EINVAL


def test_metrics_reject_bad_arguments():
    L = C.lib()
    assert L.sdgr_image_metrics(0x1000, 0x1000, 1, 10, 64, 1.0, 0x1000, 0x1000, 0x1000,
                                None) == C.SDGR_EINVAL
    assert L.sdgr_image_metrics(0x1000, 0x1000, 1, 64, 64, 0.0, 0x1000, 0x1000, 0x1000,
                                None) == C.SDGR_EINVAL
    assert L.sdgr_nearest_sq(0x1000, -1, 0x1000, 5, 0x1000, None) == C.SDGR_EINVAL
    assert L.sdgr_nearest_sq(0, 0, 0, 0, 0, None) == C.SDGR_OK


def test_plan_host_matches_the_problem_without_device_work():
    """sdgr_plan_host fills a plan from host data alone (the pointers here
    are never dereferenced); forward accepts it as matching the problem and
    then stops only at its null workspaces."""
    L = C.lib()
    sc, views, o = _args(nv=3)
    p = C.Plan()
    C.check(L.sdgr_plan_host(sc, 1, views, 3, ctypes.byref(o), 5000, 700, ctypes.byref(p)))
    assert (p.records, p.pairs_c, p.pairs_i, p.nviews, p.tile) == (30, 5000, 700, 3, 8)
    assert p.tiles_c == p.tiles_i == 3 * 64 and p.rays == 3 * 64 * 64
    assert p.state_bytes > 0 and p.bwd_scratch_bytes > 0
    rc = L.sdgr_forward(sc, 1, views, 3, ctypes.byref(o), ctypes.byref(p), None, None, None, None)
    assert rc == C.SDGR_EINVAL and b"workspace" in L.sdgr_last_error()
    assert L.sdgr_plan_host(sc, 1, views, 3, ctypes.byref(o), -1, 0,
                            ctypes.byref(p)) == C.SDGR_EUNSUPPORTED
