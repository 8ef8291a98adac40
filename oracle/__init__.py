"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or runs anything here.

The numerics live in ``prt_oracle.c`` and, for the reflectometry workload,
``surface_oracle.c`` (plain C, FP64, OpenMP over paths with thread-private
tallies reduced in a fixed order; Python wrappers of the latter in
``oracle.surface``); this module only builds them
with gcc, declares the ctypes signatures and converts numpy arrays.  Each C
function cites the passage of the paper it follows.  Loss and Adam (plain
definitions, Eq. appearance_loss and Kingma & Ba's update) are written in numpy
here.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "prt_oracle.c")
_SRC_SURFACE = os.path.join(_HERE, "surface_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libprt_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99 + OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, _SRC_SURFACE, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Scene(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("max_order", C.c_int32),
                ("voxel_km", C.c_double), ("beta_air", C.c_double), ("albedo_cloud", C.c_double),
                ("albedo_air", C.c_double), ("g", C.c_double), ("sun_zenith_deg", C.c_double),
                ("sun_azimuth_deg", C.c_double), ("sun_flux", C.c_double)]


class _Cams(C.Structure):
    _fields_ = [("n", C.c_int32), ("width", C.c_int32), ("height", C.c_int32), ("pad", C.c_int32),
                ("pos", C.POINTER(C.c_double)), ("rot", C.POINTER(C.c_double)),
                ("f_px", C.POINTER(C.c_double))]


_P = C.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = C.CDLL(_LIB_PATH)
        L.prto_philox4x32_10.argtypes = [_P, _P, _P]
        L.prto_uniforms.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, _P]
        L.prto_phase_hg.argtypes = [C.c_double, C.c_double]
        L.prto_phase_hg.restype = C.c_double
        L.prto_phase_rayleigh.argtypes = [C.c_double]
        L.prto_phase_rayleigh.restype = C.c_double
        L.prto_sample_hg.argtypes = [C.c_double, C.c_double]
        L.prto_sample_hg.restype = C.c_double
        L.prto_sample_rayleigh.argtypes = [C.c_double]
        L.prto_sample_rayleigh.restype = C.c_double
        L.prto_new_direction.argtypes = [_P, C.c_double, C.c_double, _P]
        L.prto_ray_pieces.argtypes = [C.POINTER(_Scene), _P, _P, C.c_double, _P, _P, _P]
        L.prto_ray_pieces.restype = C.c_int
        L.prto_source_weight.argtypes = [C.POINTER(_Scene)]
        L.prto_source_weight.restype = C.c_double
        L.prto_sample.argtypes = [C.POINTER(_Scene), _P, C.c_uint64, C.c_uint64, _P, C.c_int64,
                                  _P, _P, _P, _P]
        L.prto_project.argtypes = [C.POINTER(_Cams), C.c_int, _P]
        L.prto_project.restype = C.c_int
        L.prto_pixel_solid_angles.argtypes = [C.c_double, C.c_int, C.c_int, _P]
        L.prto_render.argtypes = [C.POINTER(_Scene), C.POINTER(_Cams), _P, _P, C.c_int64, C.c_int64,
                                  _P, _P, _P, _P, C.c_int32, _P, _P]
        L.prto_render.restype = C.c_int
        L.prto_grad.argtypes = [C.POINTER(_Scene), C.POINTER(_Cams), _P, _P, C.c_int64, C.c_int64,
                                _P, _P, _P, _P, _P, _P]
        L.prto_grad.restype = C.c_int
        L.prto_reweight.argtypes = [C.POINTER(_Scene), _P, _P, C.c_int64, _P, _P, _P, _P, _P]
        L.prto_reweight.restype = C.c_int
        L.prto_num_threads.restype = C.c_int
        L.prto_space_carve.argtypes = [C.POINTER(_Scene), C.POINTER(_Cams), _P, _P, _P]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _scene_struct(scene) -> _Scene:
    return _Scene(scene.nx, scene.ny, scene.nz, scene.max_order, scene.voxel_km, scene.beta_air,
                  scene.albedo_cloud, scene.albedo_air, scene.g, scene.sun_zenith_deg,
                  scene.sun_azimuth_deg, scene.sun_flux)


class _CamsHolder:
    def __init__(self, cams):
        self.pos = np.ascontiguousarray(cams.pos, dtype=np.float64)
        self.rot = np.ascontiguousarray(cams.rot, dtype=np.float64)
        self.f = np.ascontiguousarray(cams.f_px, dtype=np.float64)
        dp = C.POINTER(C.c_double)
        self.s = _Cams(cams.n, cams.width, cams.height, 0, self.pos.ctypes.data_as(dp),
                       self.rot.ctypes.data_as(dp), self.f.ctypes.data_as(dp))


def _f64(beta) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(beta, dtype=np.float32).astype(np.float64).ravel())


def num_threads() -> int:
    return int(lib().prto_num_threads())


# ------------------------------------------------------------------ RNG

def philox4x32_10(key, ctr) -> np.ndarray:
    k = np.ascontiguousarray(key, dtype=np.uint32)
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().prto_philox4x32_10(_ptr(k), _ptr(c), _ptr(out))
    return out


def uniforms(seed: int, path: int, event: int) -> np.ndarray:
    out = np.zeros(4, dtype=np.float64)
    lib().prto_uniforms(seed, path, event, _ptr(out))
    return out


# ------------------------------------------------------- phase functions

def phase_hg(mu: float, g: float) -> float:
    return lib().prto_phase_hg(float(mu), float(g))


def phase_rayleigh(mu: float) -> float:
    return lib().prto_phase_rayleigh(float(mu))


def sample_hg(u: float, g: float) -> float:
    return lib().prto_sample_hg(float(u), float(g))


def sample_rayleigh(u: float) -> float:
    return lib().prto_sample_rayleigh(float(u))


def new_direction(n, mu: float, phi: float) -> np.ndarray:
    nn = np.ascontiguousarray(n, dtype=np.float64)
    out = np.zeros(3)
    lib().prto_new_direction(_ptr(nn), float(mu), float(phi), _ptr(out))
    return out


def ray_pieces(scene, p, w, tmax):
    """(voxel ids, lengths in grid units, t_end) of the ray p + t w inside the box."""
    sc = _scene_struct(scene)
    cap = scene.nx + scene.ny + scene.nz + 8
    vox = np.zeros(cap, np.int32)
    ln = np.zeros(cap, np.float64)
    te = np.zeros(1, np.float64)
    pp = np.ascontiguousarray(p, dtype=np.float64)
    ww = np.ascontiguousarray(w, dtype=np.float64)
    n = lib().prto_ray_pieces(C.byref(sc), _ptr(pp), _ptr(ww), float(tmax), _ptr(vox), _ptr(ln), _ptr(te))
    return vox[:n].copy(), ln[:n].copy(), float(te[0])


def source_weight(scene) -> float:
    sc = _scene_struct(scene)
    return lib().prto_source_weight(C.byref(sc))


def pixel_solid_angles(f_px: float, width: int, height: int) -> np.ndarray:
    out = np.zeros((height, width), np.float64)
    lib().prto_pixel_solid_angles(float(f_px), int(width), int(height), _ptr(out))
    return out


def project(cams, d: int, xkm) -> int:
    h = _CamsHolder(cams)
    x = np.ascontiguousarray(xkm, dtype=np.float64)
    return int(lib().prto_project(C.byref(h.s), int(d), _ptr(x)))


# --------------------------------------------------------------- paths

@dataclass
class Paths:
    """Stored light paths in CSR form (the shared path-store format):
    vertex k of path i is xyz[off[i] + k] (FP32, grid units) with voxel vox[...]
    (-1 for the exit point on the box boundary).  B[i] = number of scatters."""
    off: np.ndarray
    xyz: np.ndarray
    vox: np.ndarray
    B: np.ndarray
    n_total: int
    seed: int
    beta_ref: np.ndarray   # FP32 cloud field the paths were sampled under

    @property
    def n(self) -> int:
        return int(self.B.shape[0])

    def subset(self, idx) -> "Paths":
        idx = np.asarray(idx, dtype=np.int64)
        nv = (self.off[1:] - self.off[:-1])[idx]
        off = np.zeros(len(idx) + 1, np.int64)
        off[1:] = np.cumsum(nv)
        rows = np.concatenate([np.arange(self.off[i], self.off[i + 1]) for i in idx]) if len(idx) else \
            np.zeros(0, np.int64)
        return Paths(off, self.xyz[rows].copy(), self.vox[rows].copy(), self.B[idx].copy(),
                     self.n_total, self.seed, self.beta_ref)


def sample(scene, seed: int, n: int | None = None, ids=None, first_id: int = 0, n_total: int | None = None) -> Paths:
    """Sample paths under scene.beta_cloud (Sec. 3.4 with the sun source).
    Paths are identified by their ids (first_id + i, or the explicit ids)."""
    L = lib()
    sc = _scene_struct(scene)
    bc = _f64(scene.beta_cloud)
    if ids is not None:
        ids_a = np.ascontiguousarray(ids, dtype=np.int64)
        n = len(ids_a)
        idp = _ptr(ids_a)
    else:
        ids_a = None
        idp = None
    cap = scene.max_order + 2
    xyz = np.zeros((n * cap, 3), np.float32)
    vox = np.zeros(n * cap, np.int32)
    B = np.zeros(n, np.int32)
    nv = np.zeros(n, np.int32)
    L.prto_sample(C.byref(sc), _ptr(bc), seed, first_id, idp, n, _ptr(xyz), _ptr(vox), _ptr(B), _ptr(nv))
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum(nv)
    rows = (np.arange(cap)[None, :] < nv[:, None]).ravel()
    return Paths(off, xyz[rows].copy(), vox[rows].copy(), B, n if n_total is None else n_total, seed,
                 np.asarray(scene.beta_cloud, np.float32).copy())


# ----------------------------------------------------- render / grad / r

def render(scene, cams, paths: Paths, beta_t=None, max_order_render: int | None = None,
           return_counters: bool = False):
    """Recycled forward model F(beta_t | beta_ref) on the stored paths (FP64)."""
    L = lib()
    sc = _scene_struct(scene)
    h = _CamsHolder(cams)
    bt = _f64(scene.beta_cloud if beta_t is None else beta_t)
    br = _f64(paths.beta_ref)
    img = np.zeros((cams.n, cams.height, cams.width), np.float64)
    cnt = np.zeros(2, np.int64)
    Br = scene.max_order if max_order_render is None else int(max_order_render)
    rc = L.prto_render(C.byref(sc), C.byref(h.s), _ptr(bt), _ptr(br), paths.n_total, paths.n,
                       _ptr(paths.off), _ptr(paths.xyz), _ptr(paths.vox), _ptr(paths.B), Br, _ptr(img), _ptr(cnt))
    if rc != 0:
        raise RuntimeError("oracle render failed (path longer than 78 vertices?)")
    return (img, cnt) if return_counters else img


def grad(scene, cams, paths: Paths, residual, beta_t=None) -> np.ndarray:
    """dL/dbeta_c for L with dL/dI = residual (Eq. loss_gradient, recycled)."""
    L = lib()
    sc = _scene_struct(scene)
    h = _CamsHolder(cams)
    bt = _f64(scene.beta_cloud if beta_t is None else beta_t)
    br = _f64(paths.beta_ref)
    res = np.ascontiguousarray(residual, dtype=np.float64)
    assert res.shape == (cams.n, cams.height, cams.width)
    g = np.zeros(scene.nz * scene.ny * scene.nx, np.float64)
    rc = L.prto_grad(C.byref(sc), C.byref(h.s), _ptr(bt), _ptr(br), paths.n_total, paths.n,
                     _ptr(paths.off), _ptr(paths.xyz), _ptr(paths.vox), _ptr(paths.B), _ptr(res), _ptr(g))
    if rc != 0:
        raise RuntimeError("oracle grad failed")
    return g.reshape(scene.nz, scene.ny, scene.nx)


def log_r(scene, paths: Paths, beta_t=None) -> np.ndarray:
    """Per-path log correction factor log mu(x|beta_t) - log mu(x|beta_ref)."""
    L = lib()
    sc = _scene_struct(scene)
    bt = _f64(scene.beta_cloud if beta_t is None else beta_t)
    br = _f64(paths.beta_ref)
    out = np.zeros(paths.n, np.float64)
    rc = L.prto_reweight(C.byref(sc), _ptr(bt), _ptr(br), paths.n, _ptr(paths.off), _ptr(paths.xyz),
                         _ptr(paths.vox), _ptr(paths.B), _ptr(out))
    if rc != 0:
        raise RuntimeError("oracle reweight failed")
    return out


def reweight(scene, paths: Paths, beta_t=None):
    """(mean r, effective sample size) over all N paths (Eq. correction factor)."""
    lr = log_r(scene, paths, beta_t)
    r = np.exp(lr)
    return float(r.sum() / paths.n_total), float(r.sum() ** 2 / (r * r).sum())


def sort_permutation(B) -> np.ndarray:
    """Stable order of paths by size B (Alg. 2, 'Sort'; Sec. 5.3): sorted
    position -> path id, equal sizes keeping their id order."""
    return np.argsort(np.asarray(B), kind="stable")


def space_carve(scene, cams, images, threshold) -> np.ndarray:
    """Photo-hull mask [nz][ny][nx] (uint8, 1 = kept): a voxel is removed when
    a camera sees its centre on a pixel at or below that camera's threshold
    (Sec. 6.1, initialisation by space carving)."""
    sc = _scene_struct(scene)
    h = _CamsHolder(cams)
    img = np.ascontiguousarray(images, dtype=np.float64)
    assert img.shape == (cams.n, cams.height, cams.width)
    thr = np.ascontiguousarray(np.broadcast_to(np.asarray(threshold, np.float64), (cams.n,)))
    mask = np.zeros(scene.nz * scene.ny * scene.nx, np.uint8)
    lib().prto_space_carve(C.byref(sc), C.byref(h.s), _ptr(img), _ptr(thr), _ptr(mask))
    return mask.reshape(scene.nz, scene.ny, scene.nx)


# ------------------------------------------------------------ loop glue

def loss_and_residual(images, target):
    """L = 1/2 ||F - I_gt||^2 and its derivative F - I_gt (Eq. appearance_loss)."""
    res = np.asarray(images, np.float64) - np.asarray(target, np.float64)
    return 0.5 * float((res * res).sum()), res


def downsample_images(cams, images, factor: int) -> np.ndarray:
    """Measurements at a coarser resolution (Sec. 6.1, coarse to fine): with
    images as pixel-averaged radiance (tally / Omega_p), coarse pixel P, the
    union of factor x factor fine pixels p, holds the average of the radiance
    over its solid angle, sum_p Omega_p I_p / sum_p Omega_p.  Cameras keep
    their pinhole; the coarse camera has focal length f / factor."""
    img = np.asarray(images, np.float64)
    n, H, W = img.shape
    k = int(factor)
    out = np.zeros((n, H // k, W // k))
    for d in range(n):
        om = pixel_solid_angles(float(cams.f_px[d]), W, H)
        num = (om * img[d]).reshape(H // k, k, W // k, k).sum(axis=(1, 3))
        den = om.reshape(H // k, k, W // k, k).sum(axis=(1, 3))
        out[d] = num / den
    return out


def volume_errors(beta_est, beta_true):
    """Reconstruction errors of Sec. 6: relative L1 distance
    epsilon = ||b* - b||_1 / ||b*||_1 and relative mass bias
    delta = (||b*||_1 - ||b||_1) / ||b*||_1 (b* the true field)."""
    b = np.asarray(beta_est, np.float64).ravel()
    t = np.asarray(beta_true, np.float64).ravel()
    nt = np.abs(t).sum()
    return float(np.abs(t - b).sum() / nt), float((nt - np.abs(b).sum()) / nt)


def adam_step(beta, grad_, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step (Kingma & Ba, Alg. 1), then projection onto beta >= 0.
    Returns new (beta, m, v); arrays are FP64."""
    m = b1 * m + (1.0 - b1) * grad_
    v = b2 * v + (1.0 - b2) * grad_ * grad_
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    beta = beta - lr * mh / (np.sqrt(vh) + eps)
    return np.maximum(beta, 0.0), m, v
