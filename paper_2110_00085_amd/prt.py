"""Thin ctypes binding of libprt.so (include/prt.h): argument marshalling only.

Every function here has the name of the C entry point it calls.  Device
buffers are torch tensors (their data pointers are passed through); host
arrays are numpy arrays.  A nonzero status raises PrtError with the
library's message.  The binding refuses to run without the built HIP
library: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libprt.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "prt.h")

PRT_OK, PRT_E_INVALID, PRT_E_NOMEM, PRT_E_CAPACITY, PRT_E_MISMATCH, PRT_E_HIP = 0, -1, -2, -3, -4, -5
PRT_TRAVERSAL_FP32, PRT_ALL_FP64 = 0, 1
PRT_ORDER_BY_SIZE, PRT_ORDER_BY_ID = 0, 1
PRT_MAX_CAMERAS, PRT_MAX_ORDER = 24, 64


class PrtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"prt error {code}: {msg}")
        self.code = code


class prt_scene(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("max_order", C.c_int32),
                ("voxel_km", C.c_double), ("beta_air", C.c_double), ("albedo_cloud", C.c_double),
                ("albedo_air", C.c_double), ("g", C.c_double), ("sun_zenith_deg", C.c_double),
                ("sun_azimuth_deg", C.c_double), ("sun_flux", C.c_double), ("beta_cloud", C.c_void_p)]


class prt_cameras(C.Structure):
    _fields_ = [("n", C.c_int32), ("width", C.c_int32), ("height", C.c_int32), ("pad", C.c_int32),
                ("pos", C.c_void_p), ("rot", C.c_void_p), ("f_px", C.c_void_p)]


class prt_surface_scene(C.Structure):
    _fields_ = [("box", C.c_double), ("wall_albedo", C.c_double * 6), ("light", C.c_double * 3),
                ("intensity", C.c_double), ("n_spheres", C.c_int32), ("phong", C.c_int32),
                ("max_order", C.c_int32), ("pad", C.c_int32), ("center", C.c_void_p), ("radius", C.c_void_p),
                ("albedo", C.c_void_p)]


class prt_counters_t(C.Structure):
    _fields_ = [("voxel_segments", C.c_uint64), ("local_estimates", C.c_uint64), ("paths", C.c_uint64),
                ("overhead_segments", C.c_uint64)]


class prt_paths_info_t(C.Structure):
    _fields_ = [("n_paths", C.c_uint64), ("n_vertices", C.c_uint64), ("n_batches", C.c_uint64),
                ("seed", C.c_uint64), ("bytes", C.c_uint64), ("max_order", C.c_int32), ("nx", C.c_int32),
                ("ny", C.c_int32), ("nz", C.c_int32)]


_lib = None
_V, _I32, _I64, _U64, _D = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double


def lib():
    """Load libprt.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        sig = {
            "prt_create": ([C.c_int, _V, C.c_int, C.POINTER(_V)], C.c_int),
            "prt_destroy": ([_V], None),
            "prt_set_stream": ([_V, _V], C.c_int),
            "prt_set_sample_scratch_limit": ([_V, _U64], C.c_int),
            "prt_last_error": ([], C.c_char_p),
            "prt_sample": ([_V, C.POINTER(prt_scene), _U64, _U64, C.POINTER(_V)], C.c_int),
            "prt_resample": ([_V, C.POINTER(prt_scene), _U64, _U64, _V], C.c_int),
            "prt_paths_import": ([_V, C.POINTER(prt_scene), _U64, _V, _V, _V, _V, _V, _U64, C.POINTER(_V)], C.c_int),
            "prt_paths_export": ([_V, _V, _V, _V, _V, _V, _V], C.c_int),
            "prt_paths_permutation": ([_V, _V, _V], C.c_int),
            "prt_paths_info": ([_V, C.POINTER(prt_paths_info_t)], C.c_int),
            "prt_paths_destroy": ([_V], None),
            "prt_render": ([_V, C.POINTER(prt_scene), C.POINTER(prt_cameras), _V, _I32, _V], C.c_int),
            "prt_grad": ([_V, C.POINTER(prt_scene), C.POINTER(prt_cameras), _V, _V, _V], C.c_int),
            "prt_tpp_render": ([_V, C.POINTER(prt_scene), C.POINTER(prt_cameras), _V, _I32, _V], C.c_int),
            "prt_tpp_grad": ([_V, C.POINTER(prt_scene), C.POINTER(prt_cameras), _V, _I32, _V, _V], C.c_int),
            "prt_reweight": ([_V, C.POINTER(prt_scene), _V, C.POINTER(_D), C.POINTER(_D)], C.c_int),
            "prt_loss": ([_V, _I64, _V, _V, _V, _V], C.c_int),
            "prt_reweight_noalloc": ([_V, C.POINTER(prt_scene), _V, _V], C.c_int),
            "prt_adam": ([_V, _I64, _V, _V, _V, _V, _V, _I32, _D, _D, _D, _D], C.c_int),
            "prt_downsample_images": ([_V, C.POINTER(prt_cameras), _V, _I32, _V], C.c_int),
            "prt_volume_errors": ([_V, _I64, _V, _V, _V], C.c_int),
            "prt_space_carve": ([_V, C.POINTER(prt_scene), C.POINTER(prt_cameras), _V, _V, _D, _V, _V], C.c_int),
            "prt_counters": ([_V, C.POINTER(prt_counters_t), C.c_int], C.c_int),
            "prt_enable_timing": ([_V, C.c_int], C.c_int),
            "prt_enable_timing_mask": ([_V, C.c_uint32], C.c_int),
            "prt_kernel_times": ([_V, _V, _V, C.c_int, C.c_int], C.c_int),
            "prt_kernel_name": ([C.c_int], C.c_char_p),
            "prt_surface_sample": ([_V, C.POINTER(prt_surface_scene), C.POINTER(prt_cameras), _V, _U64, _I64,
                                    C.POINTER(_V)], C.c_int),
            "prt_surface_resample": ([_V, _V, C.POINTER(prt_surface_scene), C.POINTER(prt_cameras), _V, _U64, _I64],
                                     C.c_int),
            "prt_surface_resample_device": ([_V, _V, C.POINTER(prt_surface_scene), C.POINTER(prt_cameras), _V, _U64,
                                             _I64], C.c_int),
            "prt_surface_import": ([_V, C.POINTER(prt_surface_scene), C.POINTER(prt_cameras), _V, _I64, _V, _V, _V,
                                    C.POINTER(_V)], C.c_int),
            "prt_surface_export": ([_V, _V, _V, _V, _V], C.c_int),
            "prt_surface_info": ([_V, C.POINTER(_I64), C.POINTER(_I32)], C.c_int),
            "prt_surface_work": ([_V, _V, C.POINTER(_U64), C.POINTER(_U64)], C.c_int),
            "prt_surface_render": ([_V, _V, _V, _V], C.c_int),
            "prt_surface_grad": ([_V, _V, _V, _V, _V], C.c_int),
            "prt_surface_reweight": ([_V, _V, _V, _V], C.c_int),
            "prt_surface_adam": ([_V, _V, _V, _V, _V, _I32, _D, _D, _D, _D, _D], C.c_int),
            "prt_surface_destroy": ([_V], None),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(rc: int):
    if rc != PRT_OK:
        raise PrtError(rc, lib().prt_last_error().decode())


def _dptr(t) -> int:
    """Device pointer of a contiguous torch tensor."""
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _hptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# ------------------------------------------------------------ marshalling

def make_scene(params, beta_cloud) -> prt_scene:
    """prt_scene from an object with the scene attributes and a device
    float32 tensor beta_cloud [nz][ny][nx]."""
    import torch
    if beta_cloud.dtype != torch.float32 or not beta_cloud.is_cuda:
        raise ValueError("beta_cloud must be a float32 device tensor")
    if beta_cloud.numel() != params.nx * params.ny * params.nz:
        raise ValueError("beta_cloud size does not match the grid")
    return prt_scene(params.nx, params.ny, params.nz, params.max_order, params.voxel_km, params.beta_air,
                     params.albedo_cloud, params.albedo_air, params.g, params.sun_zenith_deg,
                     params.sun_azimuth_deg, params.sun_flux, _dptr(beta_cloud))


class CamerasHost:
    """prt_cameras with its host arrays kept alive."""

    def __init__(self, cams):
        self.pos = np.ascontiguousarray(cams.pos, dtype=np.float64)
        self.rot = np.ascontiguousarray(cams.rot, dtype=np.float64)
        self.f = np.ascontiguousarray(cams.f_px, dtype=np.float64)
        self.n, self.width, self.height = int(cams.n), int(cams.width), int(cams.height)
        self.s = prt_cameras(self.n, self.width, self.height, 0, _hptr(self.pos).value, _hptr(self.rot).value,
                             _hptr(self.f).value)

    @property
    def image_shape(self):
        return (self.n, self.height, self.width)


class SurfaceSceneHost:
    """prt_surface_scene with its host sphere arrays kept alive, from an
    object with the attributes of inputs.SurfaceScene."""

    def __init__(self, scene):
        self.c = np.ascontiguousarray(np.asarray(scene.centers, np.float64).reshape(-1, 3))
        self.r = np.ascontiguousarray(scene.radii, np.float64)
        self.a = np.ascontiguousarray(scene.albedo, np.float64)
        self.max_order = int(scene.max_order)
        wa = (C.c_double * 6)(*[float(x) for x in np.asarray(scene.wall_albedo, np.float64)])
        li = (C.c_double * 3)(*[float(x) for x in np.asarray(scene.light, np.float64)])
        self.s = prt_surface_scene(float(scene.box), wa, li, float(scene.intensity), len(self.r), int(scene.phong),
                                   self.max_order, 0, _hptr(self.c).value, _hptr(self.r).value, _hptr(self.a).value)


# ---------------------------------------------------------- entry points

def prt_create(device: int = 0, stream: int | None = None, precision: int = PRT_TRAVERSAL_FP32):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device).cuda_stream
    h = _V()
    _check(lib().prt_create(device, stream, precision, C.byref(h)))
    return h


def prt_destroy(ctx):
    lib().prt_destroy(ctx)


def prt_set_stream(ctx, stream: int):
    _check(lib().prt_set_stream(ctx, stream))


def prt_set_sample_scratch_limit(ctx, n_bytes: int):
    _check(lib().prt_set_sample_scratch_limit(ctx, int(n_bytes)))


def prt_sample(ctx, scene: prt_scene, seed: int, n_paths: int):
    h = _V()
    _check(lib().prt_sample(ctx, C.byref(scene), seed, n_paths, C.byref(h)))
    return h


def prt_resample(ctx, scene: prt_scene, seed: int, n_paths: int, paths):
    _check(lib().prt_resample(ctx, C.byref(scene), seed, n_paths, paths))


def prt_paths_import(ctx, scene: prt_scene, off, xyz, vox, B, beta_ref, seed: int = 0):
    off = np.ascontiguousarray(off, np.int64)
    xyz = np.ascontiguousarray(xyz, np.float32)
    vox = np.ascontiguousarray(vox, np.int32)
    B = np.ascontiguousarray(B, np.int32)
    br = np.ascontiguousarray(beta_ref, np.float32).ravel()
    h = _V()
    _check(lib().prt_paths_import(ctx, C.byref(scene), len(B), _hptr(off), _hptr(xyz), _hptr(vox), _hptr(B),
                                  _hptr(br), seed, C.byref(h)))
    return h


def prt_paths_info(paths) -> prt_paths_info_t:
    info = prt_paths_info_t()
    _check(lib().prt_paths_info(paths, C.byref(info)))
    return info


def prt_paths_export(ctx, paths, vertices: bool = True):
    """(off, xyz, vox, B, beta_ref) as numpy arrays in path-id order."""
    info = prt_paths_info(paths)
    n = int(info.n_paths)
    off = np.zeros(n + 1, np.int64)
    B = np.zeros(n, np.int32)
    _check(lib().prt_paths_export(ctx, paths, _hptr(off), None, None, _hptr(B), None))
    if not vertices:
        return off, None, None, B, None
    nv = int(off[-1])
    xyz = np.zeros((nv, 3), np.float32)
    vox = np.zeros(nv, np.int32)
    br = np.zeros(info.nx * info.ny * info.nz, np.float32)
    _check(lib().prt_paths_export(ctx, paths, _hptr(off), _hptr(xyz), _hptr(vox), _hptr(B), _hptr(br)))
    return off, xyz, vox, B, br.reshape(info.nz, info.ny, info.nx)


def prt_paths_permutation(ctx, paths) -> np.ndarray:
    n = int(prt_paths_info(paths).n_paths)
    perm = np.zeros(n, np.int32)
    _check(lib().prt_paths_permutation(ctx, paths, _hptr(perm)))
    return perm


def prt_paths_destroy(paths):
    lib().prt_paths_destroy(paths)


def prt_render(ctx, scene: prt_scene, cams: CamerasHost, paths, max_order_render: int, images):
    _check(lib().prt_render(ctx, C.byref(scene), C.byref(cams.s), paths, int(max_order_render), _dptr(images)))


def prt_grad(ctx, scene: prt_scene, cams: CamerasHost, paths, residual, grad):
    _check(lib().prt_grad(ctx, C.byref(scene), C.byref(cams.s), paths, _dptr(residual), _dptr(grad)))


def prt_tpp_render(ctx, scene: prt_scene, cams: CamerasHost, paths, order: int, images):
    _check(lib().prt_tpp_render(ctx, C.byref(scene), C.byref(cams.s), paths, int(order), _dptr(images)))


def prt_tpp_grad(ctx, scene: prt_scene, cams: CamerasHost, paths, order: int, residual, grad):
    _check(lib().prt_tpp_grad(ctx, C.byref(scene), C.byref(cams.s), paths, int(order), _dptr(residual),
                              _dptr(grad)))


def prt_reweight(ctx, scene: prt_scene, paths):
    m, e = _D(), _D()
    _check(lib().prt_reweight(ctx, C.byref(scene), paths, C.byref(m), C.byref(e)))
    return m.value, e.value


def prt_reweight_noalloc(ctx, scene: prt_scene, paths, stats):
    """stats: device float64 tensor of 2 elements, set to (mean r, ess)."""
    if stats.dtype.itemsize != 8 or stats.numel() < 2:
        raise ValueError("stats must hold 2 float64 values")
    _check(lib().prt_reweight_noalloc(ctx, C.byref(scene), paths, _dptr(stats)))


def prt_loss(ctx, images, target, residual, loss):
    _check(lib().prt_loss(ctx, images.numel(), _dptr(images), _dptr(target), _dptr(residual), _dptr(loss)))


def prt_adam(ctx, beta, beta_f32, grad, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999,
             eps: float = 1e-8):
    _check(lib().prt_adam(ctx, beta.numel(), _dptr(beta), _dptr(beta_f32), _dptr(grad), _dptr(m), _dptr(v),
                          int(t), lr, b1, b2, eps))


def prt_downsample_images(ctx, cams: CamerasHost, images, factor: int, coarse):
    _check(lib().prt_downsample_images(ctx, C.byref(cams.s), _dptr(images), int(factor), _dptr(coarse)))


def prt_volume_errors(ctx, beta_est, beta_true, errors):
    """errors: device float64 tensor of 2, set to (epsilon, delta)."""
    if beta_est.numel() != beta_true.numel():
        raise ValueError("fields differ in size")
    _check(lib().prt_volume_errors(ctx, beta_est.numel(), _dptr(beta_est), _dptr(beta_true), _dptr(errors)))


def prt_space_carve(ctx, scene: prt_scene, cams: CamerasHost, images, threshold, fill_value: float, mask,
                    beta_out=None):
    """images: device float64 [n][H][W]; threshold: per-camera sequence or a
    scalar; mask: device uint8 [nz][ny][nx]; beta_out: optional device float32."""
    thr = np.ascontiguousarray(np.broadcast_to(np.asarray(threshold, np.float64), (cams.n,)))
    _check(lib().prt_space_carve(ctx, C.byref(scene), C.byref(cams.s), _dptr(images), _hptr(thr),
                                 float(fill_value), _dptr(mask), None if beta_out is None else _dptr(beta_out)))


def prt_counters(ctx, reset: bool = False) -> dict:
    c = prt_counters_t()
    _check(lib().prt_counters(ctx, C.byref(c), int(reset)))
    return {"voxel_segments": c.voxel_segments, "local_estimates": c.local_estimates, "paths": c.paths,
            "overhead_segments": c.overhead_segments}


def prt_enable_timing(ctx, enable: bool = True):
    _check(lib().prt_enable_timing(ctx, int(enable)))


def prt_enable_timing_mask(ctx, kernel_ids):
    """Time only the kernels named (or numbered) in kernel_ids."""
    names = {prt_kernel_name(i): i for i in range(32)}
    mask = 0
    for k in kernel_ids:
        mask |= 1 << (names[k] if isinstance(k, str) else int(k))
    _check(lib().prt_enable_timing_mask(ctx, mask))


def prt_kernel_times(ctx, reset: bool = False) -> dict:
    ms = np.zeros(32, np.float64)
    cnt = np.zeros(32, np.int64)
    k = lib().prt_kernel_times(ctx, _hptr(ms), _hptr(cnt), 32, int(reset))
    if k < 0:
        _check(k)
    return {lib().prt_kernel_name(i).decode(): (float(ms[i]), int(cnt[i])) for i in range(k)}


def prt_kernel_name(i: int) -> str:
    return lib().prt_kernel_name(i).decode()


# ---------------------------------------------------- reflectometry (prt_surface.h)

def _theta_host(theta) -> np.ndarray:
    t = np.ascontiguousarray(np.asarray(theta, np.float64).ravel())
    if t.size != 2:
        raise ValueError("theta_ref must hold (kappa_s, gamma)")
    return t


def _pair(t, what: str):
    if t.dtype.itemsize != 8 or t.numel() < 2 or not t.is_cuda:
        raise ValueError(f"{what} must be a device float64 tensor of 2 elements")
    return _dptr(t)


def prt_surface_sample(ctx, scene: SurfaceSceneHost, cams: CamerasHost, theta_ref, seed: int, n_paths: int):
    t = _theta_host(theta_ref)
    h = _V()
    _check(lib().prt_surface_sample(ctx, C.byref(scene.s), C.byref(cams.s), _hptr(t), seed, int(n_paths),
                                    C.byref(h)))
    return h


def prt_surface_resample(ctx, paths, scene: SurfaceSceneHost, cams: CamerasHost, theta_ref, seed: int,
                         n_paths: int):
    t = _theta_host(theta_ref)
    _check(lib().prt_surface_resample(ctx, paths, C.byref(scene.s), C.byref(cams.s), _hptr(t), seed,
                                      int(n_paths)))


def prt_surface_resample_device(ctx, paths, scene: SurfaceSceneHost, cams: CamerasHost, theta_ref, seed: int,
                                n_paths: int):
    """theta_ref: device float64 tensor of 2 elements (clamped by the draw)."""
    _check(lib().prt_surface_resample_device(ctx, paths, C.byref(scene.s), C.byref(cams.s),
                                             _pair(theta_ref, "theta_ref"), seed, int(n_paths)))


def prt_surface_import(ctx, scene: SurfaceSceneHost, cams: CamerasHost, theta_ref, B, pos, sid):
    """B [n], pos [n][M][3], sid [n][M] host arrays (M = max_order)."""
    t = _theta_host(theta_ref)
    B = np.ascontiguousarray(B, np.int32)
    n, M = len(B), scene.max_order
    pos = np.ascontiguousarray(pos, np.float64).reshape(n, M, 3)
    sid = np.ascontiguousarray(sid, np.int32).reshape(n, M)
    h = _V()
    _check(lib().prt_surface_import(ctx, C.byref(scene.s), C.byref(cams.s), _hptr(t), n, _hptr(B), _hptr(pos),
                                    _hptr(sid), C.byref(h)))
    return h


def prt_surface_info(paths):
    n, m = _I64(), _I32()
    _check(lib().prt_surface_info(paths, C.byref(n), C.byref(m)))
    return int(n.value), int(m.value)


def prt_surface_export(ctx, paths):
    """(B [n], pos [n][M][3], sid [n][M]) as numpy arrays."""
    n, M = prt_surface_info(paths)
    B = np.zeros(n, np.int32)
    pos = np.zeros((n, M, 3), np.float64)
    sid = np.zeros((n, M), np.int32)
    _check(lib().prt_surface_export(ctx, paths, _hptr(B), _hptr(pos), _hptr(sid)))
    return B, pos, sid


def prt_surface_work(ctx, paths):
    """(ray-sphere tests, vertices) of the store's last draw."""
    t, v = _U64(), _U64()
    _check(lib().prt_surface_work(ctx, paths, C.byref(t), C.byref(v)))
    return int(t.value), int(v.value)


def prt_surface_render(ctx, paths, theta, images):
    _check(lib().prt_surface_render(ctx, paths, _pair(theta, "theta"), _dptr(images)))


def prt_surface_grad(ctx, paths, theta, residual, grad):
    _check(lib().prt_surface_grad(ctx, paths, _pair(theta, "theta"), _dptr(residual), _pair(grad, "grad")))


def prt_surface_reweight(ctx, paths, theta, stats):
    _check(lib().prt_surface_reweight(ctx, paths, _pair(theta, "theta"), _pair(stats, "stats")))


def prt_surface_adam(ctx, theta, grad, m, v, t: int, lr_kappa: float, lr_gamma: float, b1: float = 0.9,
                     b2: float = 0.999, eps: float = 1e-8):
    _check(lib().prt_surface_adam(ctx, _pair(theta, "theta"), _pair(grad, "grad"), _pair(m, "m"), _pair(v, "v"),
                                  int(t), lr_kappa, lr_gamma, b1, b2, eps))


def prt_surface_destroy(paths):
    lib().prt_surface_destroy(paths)


def header_entry_points() -> list[str]:
    """Names of the functions declared in include/*.h."""
    import glob
    import re
    names = set()
    for h in glob.glob(os.path.join(os.path.dirname(HEADER), "*.h")):
        names |= set(re.findall(r"^\s*(?:int|void|const char\*)\s+(prt_\w+)\s*\(", open(h).read(), re.M))
    return sorted(names)


def prt_last_error() -> str:
    return lib().prt_last_error().decode()
