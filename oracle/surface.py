"""FP64 CPU oracle of the reflectometry workload (Sec. 6.2) -- TEST
INFRASTRUCTURE ONLY, like the rest of ``oracle``.

ctypes wrappers of ``surface_oracle.c``: forward path tracing from the point
light at theta_ref = (kappa_s, gamma), the recycled images
F(theta_t | theta_ref), the loss gradient with respect to (kappa_s, gamma) and
the correction factors.  Paths are kept with a fixed stride of max_order
vertices per path: vertex b of path i is pos[i, b] with surface id sid[i, b]
(b < B[i]).  Loss and Adam with the box projection are written here in numpy.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _CamsHolder, _ptr, lib as _base_lib

_P = C.c_void_p
_D2 = C.c_double * 2


class _SScene(C.Structure):
    _fields_ = [("box", C.c_double), ("wall_albedo", C.c_double * 6), ("light", C.c_double * 3),
                ("intensity", C.c_double), ("n_spheres", C.c_int32), ("phong", C.c_int32),
                ("max_order", C.c_int32), ("pad", C.c_int32), ("center", C.POINTER(C.c_double)),
                ("radius", C.POINTER(C.c_double)), ("albedo", C.POINTER(C.c_double))]


class _CamsStruct(C.Structure):
    _fields_ = [("n", C.c_int32), ("width", C.c_int32), ("height", C.c_int32), ("pad", C.c_int32),
                ("pos", C.POINTER(C.c_double)), ("rot", C.POINTER(C.c_double)),
                ("f_px", C.POINTER(C.c_double))]


_ready = False


def lib():
    global _ready
    L = _base_lib()
    if not _ready:
        S, K = C.POINTER(_SScene), C.POINTER(_CamsStruct)
        L.psso_normal.argtypes = [S, C.c_int, _P, _P]
        L.psso_sphere_hit.argtypes = [_P, C.c_double, _P, _P]
        L.psso_sphere_hit.restype = C.c_double
        L.psso_nearest.argtypes = [S, _P, _P, C.c_int, C.POINTER(C.c_double)]
        L.psso_nearest.restype = C.c_int
        L.psso_phong.argtypes = [C.c_double, C.c_double, C.c_double]
        L.psso_phong.restype = C.c_double
        L.psso_phong_deriv.argtypes = [C.c_double, C.c_double, C.c_double, _P]
        L.psso_phong_pdf.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double]
        L.psso_phong_pdf.restype = C.c_double
        L.psso_bounce.argtypes = [S, C.c_int, _P, _P, _P, _P, _P, C.POINTER(C.c_double)]
        L.psso_bounce.restype = C.c_int
        L.psso_sample.argtypes = [S, _P, C.c_uint64, C.c_uint64, C.c_int64, _P, _P, _P]
        L.psso_render.argtypes = [S, K, _P, _P, C.c_int64, C.c_int64, _P, _P, _P, _P]
        L.psso_grad.argtypes = [S, K, _P, _P, C.c_int64, C.c_int64, _P, _P, _P, _P, _P]
        L.psso_log_r.argtypes = [S, _P, _P, C.c_int64, _P, _P, _P, _P]
        _ready = True
    return L


class _SceneHolder:
    def __init__(self, scene):
        self.c = np.ascontiguousarray(scene.centers, np.float64).reshape(-1, 3)
        self.r = np.ascontiguousarray(scene.radii, np.float64)
        self.a = np.ascontiguousarray(scene.albedo, np.float64)
        dp = C.POINTER(C.c_double)
        self.s = _SScene(float(scene.box), _to_c(scene.wall_albedo, 6), _to_c(scene.light, 3),
                         float(scene.intensity), scene.n_spheres, scene.phong, scene.max_order, 0,
                         self.c.ctypes.data_as(dp), self.r.ctypes.data_as(dp), self.a.ctypes.data_as(dp))


def _to_c(a, n):
    return (C.c_double * n)(*[float(x) for x in np.asarray(a, np.float64).ravel()])


def _cams(cams):
    h = _CamsHolder(cams)
    dp = C.POINTER(C.c_double)
    h.ss = _CamsStruct(cams.n, cams.width, cams.height, 0, h.pos.ctypes.data_as(dp), h.rot.ctypes.data_as(dp),
                       h.f.ctypes.data_as(dp))
    return h


def _theta(t):
    return np.ascontiguousarray(np.asarray(t, np.float64).ravel()[:2])


@dataclass
class SurfacePaths:
    """Light paths of the surface scene: B[i] surface vertices pos[i, :B[i]]
    (FP64) on surfaces sid[i, :B[i]], drawn at theta_ref."""
    B: np.ndarray          # [n] int32
    pos: np.ndarray        # [n][M][3] float64
    sid: np.ndarray        # [n][M] int32
    theta_ref: np.ndarray  # [2]
    n_total: int
    seed: int

    @property
    def n(self) -> int:
        return int(self.B.shape[0])


# ---------------------------------------------------------- small pieces

def normal(scene, sid: int, x) -> np.ndarray:
    h = _SceneHolder(scene)
    xx = np.ascontiguousarray(x, np.float64)
    out = np.zeros(3)
    lib().psso_normal(C.byref(h.s), sid, _ptr(xx), _ptr(out))
    return out


def sphere_hit(center, radius: float, p, w) -> float:
    c, pp, ww = (np.ascontiguousarray(a, np.float64) for a in (center, p, w))
    return float(lib().psso_sphere_hit(_ptr(c), radius, _ptr(pp), _ptr(ww)))


def nearest(scene, p, w, skip: int = -1):
    h = _SceneHolder(scene)
    pp, ww = np.ascontiguousarray(p, np.float64), np.ascontiguousarray(w, np.float64)
    t = C.c_double(0.0)
    sid = lib().psso_nearest(C.byref(h.s), _ptr(pp), _ptr(ww), skip, C.byref(t))
    return int(sid), float(t.value)


def phong(kappa: float, gamma: float, c: float) -> float:
    return float(lib().psso_phong(kappa, gamma, c))


def phong_deriv(kappa: float, gamma: float, c: float) -> np.ndarray:
    out = np.zeros(2)
    lib().psso_phong_deriv(kappa, gamma, c, _ptr(out))
    return out


def phong_pdf(kappa: float, gamma: float, ncos: float, c: float) -> float:
    return float(lib().psso_phong_pdf(kappa, gamma, ncos, c))


def bounce(scene, sid: int, theta, x, w_in, u):
    """One direction draw at surface sid: (alive, w_out, weight f|n.w|/pdf)."""
    h = _SceneHolder(scene)
    th, xx, wi, uu = (np.ascontiguousarray(a, np.float64) for a in (_theta(theta), x, w_in, u))
    wo = np.zeros(3)
    wt = C.c_double(0.0)
    ok = lib().psso_bounce(C.byref(h.s), sid, _ptr(th), _ptr(xx), _ptr(wi), _ptr(uu), _ptr(wo), C.byref(wt))
    return bool(ok), wo, float(wt.value)


# ------------------------------------------------------- paths and sums

def sample(scene, theta_ref, seed: int, n: int, first_id: int = 0, n_total: int | None = None) -> SurfacePaths:
    """Forward path tracing from the light at theta_ref (paths first_id ..
    first_id + n - 1 of the stream `seed`)."""
    h = _SceneHolder(scene)
    th = _theta(theta_ref)
    M = scene.max_order
    B = np.zeros(n, np.int32)
    pos = np.zeros((n, M, 3), np.float64)
    sid = np.full((n, M), -1, np.int32)
    lib().psso_sample(C.byref(h.s), _ptr(th), seed, first_id, n, _ptr(B), _ptr(pos), _ptr(sid))
    return SurfacePaths(B, pos, sid, th.copy(), n if n_total is None else n_total, seed)


def render(scene, cams, paths: SurfacePaths, theta_t) -> np.ndarray:
    """Recycled images F(theta_t | theta_ref), FP64 [n_cams][H][W]."""
    h, k = _SceneHolder(scene), _cams(cams)
    tt, tr = _theta(theta_t), _theta(paths.theta_ref)
    img = np.zeros((cams.n, cams.height, cams.width), np.float64)
    lib().psso_render(C.byref(h.s), C.byref(k.ss), _ptr(tt), _ptr(tr), paths.n_total, paths.n,
                      _ptr(np.ascontiguousarray(paths.B)), _ptr(np.ascontiguousarray(paths.pos)),
                      _ptr(np.ascontiguousarray(paths.sid)), _ptr(img))
    return img


def grad(scene, cams, paths: SurfacePaths, residual, theta_t) -> np.ndarray:
    """d loss / d (kappa_s, gamma) on the stored paths for the residual
    images F - Y."""
    h, k = _SceneHolder(scene), _cams(cams)
    tt, tr = _theta(theta_t), _theta(paths.theta_ref)
    res = np.ascontiguousarray(residual, np.float64)
    out = np.zeros(2)
    lib().psso_grad(C.byref(h.s), C.byref(k.ss), _ptr(tt), _ptr(tr), paths.n_total, paths.n,
                    _ptr(np.ascontiguousarray(paths.B)), _ptr(np.ascontiguousarray(paths.pos)),
                    _ptr(np.ascontiguousarray(paths.sid)), _ptr(res), _ptr(out))
    return out


def log_r(scene, paths: SurfacePaths, theta_t) -> np.ndarray:
    h = _SceneHolder(scene)
    tt, tr = _theta(theta_t), _theta(paths.theta_ref)
    out = np.zeros(paths.n)
    lib().psso_log_r(C.byref(h.s), _ptr(tt), _ptr(tr), paths.n, _ptr(np.ascontiguousarray(paths.B)),
                     _ptr(np.ascontiguousarray(paths.pos)), _ptr(np.ascontiguousarray(paths.sid)), _ptr(out))
    return out


def reweight(scene, paths: SurfacePaths, theta_t):
    """(mean r, effective sample size (sum r)^2 / sum r^2)."""
    r = np.exp(log_r(scene, paths, theta_t))
    return float(r.mean()), float(r.sum() ** 2 / (r * r).sum())


def adam_step(theta, g, m, v, t: int, lr, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step (Kingma & Ba, Alg. 1) per parameter with its own step
    size lr[k], then projection onto 0 <= kappa_s <= 1, gamma >= 0."""
    theta, g, m, v, lr = (np.asarray(a, np.float64) for a in (theta, g, m, v, lr))
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    theta = theta - lr * mh / (np.sqrt(vh) + eps)
    theta = np.array([min(max(theta[0], 0.0), 1.0), max(theta[1], 0.0)])
    return theta, m, v


def param_errors(theta_est, theta_true):
    """Sec. 6 error measures on the parameter vector: epsilon = sum |est -
    true| / sum |true| and delta = (sum est - sum true) / sum true."""
    e, t = np.asarray(theta_est, np.float64), np.asarray(theta_true, np.float64)
    return float(np.abs(e - t).sum() / np.abs(t).sum()), float((e.sum() - t.sum()) / t.sum())
