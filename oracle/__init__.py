"""FP64 CPU oracle of the SAR Differentiable Gaussian Rasterizer.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product path never
does, and this package imports nothing from the product.

The arithmetic lives in ``sdgr_oracle.c`` (plain C, FP64, OpenMP, brute force
over every Gaussian, ray and pixel); this module marshals numpy arrays in and
out of it. Scenes and views are duck-typed: any object with the attributes of
the input generator's ``Scene`` (means, scales, quats, amp, ext) and ``View``
(azimuth, grazing, img_w, img_h, d_az, d_rg, comp_w, comp_h, comp_d_az,
comp_d_el) works.

Defaults follow the readings documented in the C file: footprint cutoff
q_max = 9 (three standard deviations), no dilation, shadowing on.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sdgr_oracle.c")
LIB = os.path.join(HERE, "libsdgr_oracle.so")

Q_MAX = 9.0

_lib = None
_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, OpenMP)."""
    if force or not os.path.exists(LIB) or \
            os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp",
                               "-ffp-contract=off", "-fPIC", "-shared",
                               "-D_GNU_SOURCE", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(LIB)
        L.orc_version.restype = ctypes.c_int
        L.orc_threads.restype = ctypes.c_int
        L.orc_axes.argtypes = [ctypes.c_double, ctypes.c_double, _dp, _dp, _dp]
        L.orc_view.argtypes = [_dp, _dp]
        L.orc_project.argtypes = [_i64, _dp, _dp, _dp, _dp, ctypes.c_double,
                                  ctypes.c_double, _dp]
        X = [_dp, _dp, _i64, _i64]   # ext_back, sh, sh_deg, cell_area
        L.orc_forward.argtypes = [_i64, _dp, _dp, _dp, _dp, _dp, *X, _dp,
                                  ctypes.c_double, ctypes.c_double,
                                  ctypes.c_int, _dp, _dp, _dp]
        L.orc_backward.argtypes = [_i64, _dp, _dp, _dp, _dp, _dp, *X, _dp,
                                   ctypes.c_double, ctypes.c_double,
                                   ctypes.c_int, _dp, _dp, _dp, _dp, _dp,
                                   _dp, _dp, _dp, _dp]
        L.orc_sparse_forward.argtypes = [_i64, _dp, _dp, _dp, _dp, _dp, *X, _dp,
                                         ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int, _i64, _ip, _dp, _i64,
                                         _ip, _dp]
        L.orc_fd_linear.argtypes = [_i64, _dp, _dp, _dp, _dp, _dp, *X, _dp,
                                    ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int, _dp, _i64, ctypes.c_int,
                                    ctypes.c_double, _dp]
        L.orc_sh_basis.argtypes = [_i64, _dp, _i64, _dp]
        _lib = L
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(_dp)


def view_params(v) -> np.ndarray:
    return np.array([v.azimuth, v.grazing, v.img_w, v.img_h, v.d_az, v.d_rg,
                     getattr(v, "comp_w", 0), getattr(v, "comp_h", 0),
                     getattr(v, "comp_d_az", 0.0),
                     getattr(v, "comp_d_el", 0.0),
                     getattr(v, "radar_range", 0.0)], dtype=np.float64)


def resolved_view(v) -> dict:
    out = np.zeros(19)
    if lib().orc_view(_p(view_params(v)), _p(out)):
        raise ValueError("invalid view")
    return dict(W=int(out[0]), H=int(out[1]), dA=out[2], dR=out[3],
                Wc=int(out[4]), Hc=int(out[5]), dAc=out[6], dEc=out[7],
                range=out[8], ex=out[10:13].copy(), ey=out[13:16].copy(),
                ez=out[16:19].copy())


def axes(phi: float, theta: float):
    ex, ey, ez = np.zeros(3), np.zeros(3), np.zeros(3)
    lib().orc_axes(phi, theta, _p(ex), _p(ey), _p(ez))
    return ex, ey, ez


def _params(scene):
    return (_d(scene.means), _d(scene.scales), _d(scene.quats),
            _d(scene.amp), _d(scene.ext))


def _extra(scene, cell_area):
    """(ext_back, sh, sh_deg, cell_area) arguments and the arrays kept alive
    behind them: the optional backward extinction and SH coefficients."""
    eb = getattr(scene, "ext_back", None)
    sh = getattr(scene, "sh", None)
    eb = None if eb is None else _d(eb)
    deg = 0
    if sh is not None:
        sh = _d(sh)
        deg = int(round(np.sqrt(sh.shape[1]))) - 1
        if (deg + 1) ** 2 != sh.shape[1] or not 0 <= deg <= 3:
            raise ValueError("sh must hold (d+1)^2 coefficients per Gaussian, d <= 3")
    args = (None if eb is None else _p(eb), None if sh is None else _p(sh), deg,
            int(bool(cell_area)))
    return args, (eb, sh)


def project(scene, view, q_max: float = Q_MAX, dilation: float = 0.0) -> dict:
    m, s, q, _, _ = _params(scene)
    n = m.shape[0]
    out = np.zeros((n, 21))
    if lib().orc_project(n, _p(m), _p(s), _p(q), _p(view_params(view)),
                         dilation, q_max, _p(out)):
        raise ValueError("invalid arguments")
    return dict(valid=out[:, 0] > 0, x=out[:, 1], y=out[:, 2],
                depth=out[:, 3], key=out[:, 4].astype(np.float32),
                cC=out[:, 5:7], covC=out[:, 7:10], conC=out[:, 10:13],
                cI=out[:, 13:15], covI=out[:, 15:18], conI=out[:, 18:21])


def forward_view(scene, view, q_max=Q_MAX, dilation=0.0, shadowing=True,
                 cell_area=False):
    """One view: returns (A[n], tau[Hc, Wc], S[H, W])."""
    m, s, q, a, e = _params(scene)
    x, keep = _extra(scene, cell_area)
    n = m.shape[0]
    rv = resolved_view(view)
    A = np.zeros(n)
    tau = np.zeros((rv["Hc"], rv["Wc"]))
    S = np.zeros((rv["H"], rv["W"]))
    if lib().orc_forward(n, _p(m), _p(s), _p(q), _p(a), _p(e), *x,
                         _p(view_params(view)), q_max, dilation,
                         int(bool(shadowing)), _p(A), _p(tau), _p(S)):
        raise ValueError("invalid arguments")
    return A, tau, S


def forward(scene, views: Sequence, **kw):
    """All views: returns (A[V, n], [tau_v], [S_v])."""
    outs = [forward_view(scene, v, **kw) for v in views]
    return (np.stack([o[0] for o in outs]), [o[1] for o in outs],
            [o[2] for o in outs])


def backward_view(scene, view, G, q_max=Q_MAX, dilation=0.0, shadowing=True,
                  cell_area=False):
    """Gradients of L with dL/dS = G for one view.

    Returns (grads dict, aux[n, 16]) where aux holds the per-Gaussian
    intermediate quantities documented in the C source. The dict has
    ext_back and sh entries when the scene has those inputs."""
    m, s, q, a, e = _params(scene)
    x, keep = _extra(scene, cell_area)
    n = m.shape[0]
    G = _d(G)
    dm, ds = np.zeros((n, 3)), np.zeros((n, 3))
    dq, da, de, deb = np.zeros((n, 4)), np.zeros(n), np.zeros(n), np.zeros(n)
    dsh = np.zeros((n, 16 if keep[1] is None else keep[1].shape[1]))
    aux = np.zeros((n, 16))
    if lib().orc_backward(n, _p(m), _p(s), _p(q), _p(a), _p(e), *x,
                          _p(view_params(view)), q_max, dilation,
                          int(bool(shadowing)), _p(G), _p(dm), _p(ds),
                          _p(dq), _p(da), _p(de), _p(deb), _p(dsh), _p(aux)):
        raise ValueError("invalid arguments")
    out = dict(means=dm, scales=ds, quats=dq, amp=da, ext=de)
    if keep[0] is not None:
        out["ext_back"] = deb
    if keep[1] is not None:
        out["sh"] = dsh
    return out, aux


def backward(scene, views: Sequence, Gs: Sequence, **kw):
    """Sum over views of the per-view gradients; also returns per-view aux."""
    tot, auxes = None, []
    for v, G in zip(views, Gs):
        g, aux = backward_view(scene, v, G, **kw)
        auxes.append(aux)
        tot = g if tot is None else {k: tot[k] + g[k] for k in tot}
    return tot, auxes


def sparse_forward(scene, view, pix_ids, gids, q_max=Q_MAX, dilation=0.0,
                   shadowing=True, cell_area=False):
    """S at flat pixel ids (row * W + col) and A of Gaussians `gids`."""
    m, s, q, a, e = _params(scene)
    x, keep = _extra(scene, cell_area)
    n = m.shape[0]
    pix = np.ascontiguousarray(pix_ids, dtype=np.int64)
    gid = np.ascontiguousarray(gids, dtype=np.int64)
    S = np.zeros(pix.shape[0])
    A = np.zeros(gid.shape[0])
    if lib().orc_sparse_forward(n, _p(m), _p(s), _p(q), _p(a), _p(e), *x,
                                _p(view_params(view)), q_max, dilation,
                                int(bool(shadowing)), pix.shape[0],
                                pix.ctypes.data_as(_ip), _p(S), gid.shape[0],
                                gid.ctypes.data_as(_ip), _p(A)):
        raise ValueError("invalid arguments")
    return S, A


# parameter components of one Gaussian, in the order orc_fd_linear numbers them
FD_COMPONENTS = [("means", 0), ("means", 1), ("means", 2), ("scales", 0),
                 ("scales", 1), ("scales", 2), ("quats", 0), ("quats", 1),
                 ("quats", 2), ("quats", 3), ("amp", None), ("ext", None),
                 ("ext_back", None)] + [("sh", k) for k in range(16)]


def fd_components(scene):
    """(comp, name, index) of the parameter components `scene` has."""
    out = []
    nsh = 0 if getattr(scene, "sh", None) is None else scene.sh.shape[1]
    for c, (name, j) in enumerate(FD_COMPONENTS):
        if name == "ext_back" and getattr(scene, "ext_back", None) is None:
            continue
        if name == "sh" and j >= nsh:
            continue
        if name == "amp" and nsh:
            continue
        out.append((c, name, j))
    return out


def fd_linear(scene, view, V, k, comp, h, q_max=Q_MAX, dilation=0.0,
              shadowing=True, cell_area=False):
    """Central difference of L = <V, S> for one view when component `comp`
    (see FD_COMPONENTS; 12 needs ext_back, 13 + j the SH coefficients) of
    Gaussian k moves by +h and -h, recomputing exactly only the rays and
    pixels the change reaches. Returns (L(+h) - L(-h), order_changed)."""
    m, s, q, a, e = _params(scene)
    x, keep = _extra(scene, cell_area)
    n = m.shape[0]
    Vd = _d(V)
    out = np.zeros(2)
    if lib().orc_fd_linear(n, _p(m), _p(s), _p(q), _p(a), _p(e), *x,
                           _p(view_params(view)), q_max, dilation,
                           int(bool(shadowing)), _p(Vd), int(k), int(comp),
                           float(h), _p(out)):
        raise ValueError("invalid arguments")
    return float(out[0]), bool(out[1])


def sh_basis(dirs, deg: int) -> np.ndarray:
    """Real spherical harmonics of degree <= deg at unit vectors dirs [m, 3]:
    [m, (deg + 1)^2], index l*l + l + m."""
    d = _d(np.atleast_2d(dirs))
    Y = np.zeros((d.shape[0], (deg + 1) ** 2))
    if lib().orc_sh_basis(d.shape[0], _p(d), deg, _p(Y)):
        raise ValueError("invalid arguments")
    return Y


def threads() -> int:
    return int(lib().orc_threads())
