"""Convenience layer over the C ABI: owning handles and the autograd.Function.

All numerics run in libprt.so; this module only owns handles, allocates
torch device tensors for outputs, and wires prt_render / prt_grad into
torch.autograd so that any torch loss on the images drives the path-reuse
gradient kernel (Eq. loss_gradient generalised to dL/dI from autograd).
"""
from __future__ import annotations

import atexit
import weakref

import torch

from . import prt as P

_live_stores: "weakref.WeakSet" = weakref.WeakSet()
_live_contexts: "weakref.WeakSet[Context]" = weakref.WeakSet()


@atexit.register
def _close_all():
    """Release library handles while the HIP runtime is still up: stores
    first, then contexts (finalizer order at interpreter exit is arbitrary)."""
    for s in list(_live_stores):
        s.close()
    for c in list(_live_contexts):
        c.close()


class Context:
    """A prt_ctx bound to a device and torch's current stream on it."""

    def __init__(self, device: int = 0, precision: int = P.PRT_TRAVERSAL_FP32):
        self.device = device
        self.precision = precision
        self.handle = P.prt_create(device, torch.cuda.current_stream(device).cuda_stream, precision)
        _live_contexts.add(self)

    def close(self):
        if self.handle is not None:
            P.prt_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PathStore:
    """Owning handle of a library path store."""

    def __init__(self, ctx: Context, handle):
        self.ctx = ctx
        self.handle = handle
        _live_stores.add(self)

    @classmethod
    def sample(cls, ctx: Context, params, beta_cloud, seed: int, n_paths: int) -> "PathStore":
        return cls(ctx, P.prt_sample(ctx.handle, P.make_scene(params, beta_cloud), seed, n_paths))

    @classmethod
    def from_host(cls, ctx: Context, params, beta_cloud, off, xyz, vox, B, beta_ref, seed: int = 0) -> "PathStore":
        return cls(ctx, P.prt_paths_import(ctx.handle, P.make_scene(params, beta_cloud), off, xyz, vox, B,
                                           beta_ref, seed))

    def resample(self, params, beta_cloud, seed: int, n_paths: int) -> "PathStore":
        P.prt_resample(self.ctx.handle, P.make_scene(params, beta_cloud), seed, n_paths, self.handle)
        return self

    def info(self):
        return P.prt_paths_info(self.handle)

    def export(self, vertices: bool = True):
        return P.prt_paths_export(self.ctx.handle, self.handle, vertices)

    def close(self):
        if self.handle is not None:
            P.prt_paths_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SurfacePaths:
    """Owning handle of a reflectometry path store (include/prt_surface.h):
    paths drawn at theta_ref in a box of spheres, with their tape for the
    cameras they were drawn for."""

    def __init__(self, ctx: Context, handle, scene, cams):
        self.ctx = ctx
        self.handle = handle
        self.scene = P.SurfaceSceneHost(scene)
        self.cams = P.CamerasHost(cams) if not isinstance(cams, P.CamerasHost) else cams
        _live_stores.add(self)

    @classmethod
    def sample(cls, ctx: Context, scene, cams, theta_ref, seed: int, n_paths: int) -> "SurfacePaths":
        sh, ch = P.SurfaceSceneHost(scene), P.CamerasHost(cams)
        return cls(ctx, P.prt_surface_sample(ctx.handle, sh, ch, theta_ref, seed, n_paths), scene, ch)

    @classmethod
    def from_host(cls, ctx: Context, scene, cams, theta_ref, B, pos, sid) -> "SurfacePaths":
        sh, ch = P.SurfaceSceneHost(scene), P.CamerasHost(cams)
        return cls(ctx, P.prt_surface_import(ctx.handle, sh, ch, theta_ref, B, pos, sid), scene, ch)

    def resample(self, theta_ref, seed: int, n_paths: int) -> "SurfacePaths":
        """theta_ref: host pair, or a device float64 tensor (read by the draw,
        clamped to kappa_s <= 0.999, 0 <= gamma <= 1e4)."""
        if hasattr(theta_ref, "is_cuda") and theta_ref.is_cuda:
            P.prt_surface_resample_device(self.ctx.handle, self.handle, self.scene, self.cams, theta_ref, seed,
                                          n_paths)
        else:
            P.prt_surface_resample(self.ctx.handle, self.handle, self.scene, self.cams, theta_ref, seed, n_paths)
        return self

    @property
    def n(self) -> int:
        return P.prt_surface_info(self.handle)[0]

    def export(self):
        return P.prt_surface_export(self.ctx.handle, self.handle)

    def render(self, theta, images=None):
        if images is None:
            images = torch.empty(self.cams.image_shape, dtype=torch.float64, device=theta.device)
        P.prt_surface_render(self.ctx.handle, self.handle, theta, images)
        return images

    def grad(self, theta, residual, out=None):
        if out is None:
            out = torch.empty(2, dtype=torch.float64, device=theta.device)
        P.prt_surface_grad(self.ctx.handle, self.handle, theta, residual.contiguous(), out)
        return out

    def reweight(self, theta, out=None):
        if out is None:
            out = torch.empty(2, dtype=torch.float64, device=theta.device)
        P.prt_surface_reweight(self.ctx.handle, self.handle, theta, out)
        return out

    def close(self):
        if self.handle is not None:
            P.prt_surface_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def render(ctx: Context, params, beta_cloud, cams: P.CamerasHost, paths: PathStore, max_order_render=None):
    out = torch.empty(cams.image_shape, dtype=torch.float64, device=beta_cloud.device)
    P.prt_render(ctx.handle, P.make_scene(params, beta_cloud), cams, paths.handle,
                 params.max_order if max_order_render is None else max_order_render, out)
    return out


def grad(ctx: Context, params, beta_cloud, cams: P.CamerasHost, paths: PathStore, residual):
    g = torch.empty((params.nz, params.ny, params.nx), dtype=torch.float64, device=beta_cloud.device)
    P.prt_grad(ctx.handle, P.make_scene(params, beta_cloud), cams, paths.handle, residual.contiguous(), g)
    return g


class RenderFn(torch.autograd.Function):
    """images = F(beta | beta_ref) on recycled paths; backward = prt_grad.

    Input beta is the FP64 cloud field (the optimiser's master copy); the
    kernels read an FP32 copy.  The gradient is returned in FP64."""

    @staticmethod
    def forward(fctx, beta64, ctx: Context, params, cams: P.CamerasHost, paths: PathStore):
        beta32 = beta64.detach().to(torch.float32).contiguous()
        images = render(ctx, params, beta32, cams, paths)
        fctx.save_for_backward(beta32)
        fctx.prt = (ctx, params, cams, paths)
        return images

    @staticmethod
    def backward(fctx, grad_images):
        (beta32,) = fctx.saved_tensors
        ctx, params, cams, paths = fctx.prt
        g = grad(ctx, params, beta32, cams, paths, grad_images.to(torch.float64).contiguous())
        return g, None, None, None, None
