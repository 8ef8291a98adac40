"""Alg. 2 (inverse rendering with path recycling) driven through the C ABI.

Every numerical step runs in libprt.so; this module holds only the loop's
control flow: when to resample, when to move to the next stage of the
coarse-to-fine schedule, and what to record.

One iteration t (Alg. 2):

1. if the resampling policy asks for it (or no paths exist yet): draw N
   paths at beta_t, snapshot beta_ref = beta_t and sort them by size
   (``prt_resample``);
2. render the recycled estimate F(beta_t | beta_ref) (``prt_render``);
3. loss and residual against the measured images (``prt_loss``);
4. the loss gradient on the same paths (``prt_grad``);
5. Adam with projection onto beta >= 0 (``prt_adam``);
6. the correction-factor statistics at the updated field (``prt_reweight``):
   mean r and the effective sample size;
7. with a known true field, the reconstruction errors epsilon (relative L1
   distance) and delta (relative mass bias) of Sec. 6 (``prt_volume_errors``).

Resampling policy: Alg. 2 resamples every N_r iterations; the drift test
|mean r - 1| > drift and a floor on the effective sample size are the
alternative triggers (any may be set).

Coarse-to-fine (Sec. 6.1): the reconstruction runs through stages of camera
resolution and path count; a stage's measurements are the full-resolution
images down-sampled to its resolution (``prt_downsample_images``), and the
next stage starts when the loss saturates (its relative decrease over a
window of iterations falls below a tolerance) or the stage's iteration
budget is spent.  Space carving (``prt_space_carve``) gives the initial
field: the photo hull of the measured images filled with a constant
extinction.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import torch

import inputs

from . import api, prt as P


@dataclass
class Policy:
    """When to draw new paths: every `period` iterations (Alg. 2's N_r), when
    the mean correction factor drifts from 1 by more than `drift`, and/or when
    the effective sample size falls below `min_ess` times N (any that is set)."""
    period: int | None = None
    drift: float | None = 0.2
    min_ess: float | None = None

    def resample(self, t: int, t_ref: int, mean_r: float | None, ess_fraction: float | None = None) -> bool:
        if self.period is not None and t - t_ref >= self.period:
            return True
        if self.drift is not None and mean_r is not None and not abs(mean_r - 1.0) <= self.drift:
            return True  # (a NaN mean r also resamples)
        if self.min_ess is not None and ess_fraction is not None and not ess_fraction >= self.min_ess:
            return True
        return False


@dataclass
class Stage:
    """One stage of the coarse-to-fine schedule: cameras down-sampled by
    `factor` (image sides divided by it), `n_paths` paths per store, at most
    `max_iters` iterations; the stage ends early when the loss decreased by
    less than `tol` (relative) over the last `window` iterations."""
    factor: int
    n_paths: int
    max_iters: int
    window: int = 10
    tol: float = 1e-3


def saturated(losses, window: int, tol: float) -> bool:
    """The loss saturates when it fell by less than tol (relative) over the
    last `window` iterations."""
    if len(losses) <= window:
        return False
    old, new = losses[-window - 1], losses[-1]
    return not (old - new > tol * abs(old))


@dataclass
class Record:
    stage: int
    iteration: int
    loss: float
    mean_r: float
    ess: float
    resampled: bool
    seconds: float
    epsilon: float | None = None
    delta: float | None = None


@dataclass
class Reconstruction:
    """State of one reconstruction: the FP64 master field with its Adam
    moments and FP32 copy, the path store, and the per-iteration records."""
    ctx: api.Context
    scene: object                  # scene parameters (grid, optics, max_order)
    cams: object                   # full-resolution cameras
    measured: torch.Tensor         # device FP64 [n][H][W] at full resolution
    beta: torch.Tensor             # device FP32 initial field [nz][ny][nx]
    lr: float = 0.1
    policy: Policy = field(default_factory=Policy)
    seed: int = 1
    beta_true: torch.Tensor | None = None   # device FP32, for epsilon and delta
    records: list = field(default_factory=list)

    def __post_init__(self):
        dev = self.beta.device
        self.beta32 = self.beta.to(torch.float32).contiguous().clone()
        self.beta64 = self.beta32.double()
        self.m = torch.zeros_like(self.beta64)
        self.v = torch.zeros_like(self.beta64)
        self.t = 0
        self.store = None
        self.errors = torch.zeros(2, dtype=torch.float64, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)

    def close(self):
        if self.store is not None:
            self.store.close()
            self.store = None

    def run_stage(self, k: int, stage: Stage, callback=None):
        h = self.ctx.handle
        cams = inputs.coarse_cameras(self.cams, stage.factor) if stage.factor > 1 else self.cams
        ch = P.CamerasHost(cams)
        full = P.CamerasHost(self.cams)
        if stage.factor > 1:
            target = torch.empty(ch.image_shape, dtype=torch.float64, device=self.beta32.device)
            P.prt_downsample_images(h, full, self.measured, stage.factor, target)
        else:
            target = self.measured.contiguous()
        img = torch.empty(ch.image_shape, dtype=torch.float64, device=self.beta32.device)
        res = torch.empty_like(img)
        grad = torch.empty_like(self.beta64)
        sc = P.make_scene(self.scene, self.beta32)
        losses = []
        mean_r = ess_fraction = None
        t_ref = self.t
        new_stage = True
        for _ in range(stage.max_iters):
            t0 = time.perf_counter()
            resampled = False
            if self.store is None or new_stage or self.policy.resample(self.t, t_ref, mean_r, ess_fraction):
                if self.store is None:
                    self.store = api.PathStore.sample(self.ctx, self.scene, self.beta32, self.seed + self.t,
                                                      stage.n_paths)
                else:
                    self.store.resample(self.scene, self.beta32, self.seed + self.t, stage.n_paths)
                t_ref = self.t
                resampled = True
                new_stage = False
            self.t += 1
            P.prt_render(h, sc, ch, self.store.handle, self.scene.max_order, img)
            P.prt_loss(h, img, target, res, self.loss)
            P.prt_grad(h, sc, ch, self.store.handle, res, grad)
            P.prt_adam(h, self.beta64, self.beta32, grad.view(-1), self.m, self.v, self.t, self.lr)
            mean_r, ess = P.prt_reweight(h, sc, self.store.handle)
            ess_fraction = ess / stage.n_paths
            eps = dlt = None
            if self.beta_true is not None:
                P.prt_volume_errors(h, self.beta64, self.beta_true, self.errors)
                eps, dlt = (float(x) for x in self.errors.cpu())
            loss = float(self.loss.item())
            losses.append(loss)
            rec = Record(k, self.t, loss, mean_r, ess, resampled, time.perf_counter() - t0, eps, dlt)
            self.records.append(rec)
            if callback:
                callback(rec)
            if saturated(losses, stage.window, stage.tol):
                break

    def run(self, stages, callback=None):
        for k, st in enumerate(stages):
            self.run_stage(k, st, callback)
        return self.records


def space_carved_start(ctx: api.Context, scene, cams, measured: torch.Tensor, threshold, fill_value: float):
    """Initial field of Sec. 6.1: the photo hull of the measured images
    (voxels whose centre no camera sees on a pixel at or below its
    threshold) filled with `fill_value` (the cloud's mean extinction)."""
    dev = measured.device
    mask = torch.empty((scene.nz, scene.ny, scene.nx), dtype=torch.uint8, device=dev)
    beta = torch.empty((scene.nz, scene.ny, scene.nx), dtype=torch.float32, device=dev)
    dummy = torch.zeros_like(beta)
    P.prt_space_carve(ctx.handle, P.make_scene(scene, dummy), P.CamerasHost(cams), measured.contiguous(),
                      threshold, fill_value, mask, beta)
    return beta, mask


# ------------------------------------------------------------ reflectometry

@dataclass
class SurfaceRecord:
    iteration: int
    loss: float
    mean_r: float
    ess: float
    resampled: bool
    seconds: float
    theta: tuple
    epsilon: float | None = None
    delta: float | None = None


def param_errors(theta, truth):
    """Sec. 6's error measures on the parameter vector (kappa_s, gamma):
    epsilon = sum |est - true| / sum |true|, delta = (sum est - sum true) /
    sum true."""
    e = [float(x) for x in theta]
    t = [float(x) for x in truth]
    st = sum(abs(x) for x in t)
    return sum(abs(a - b) for a, b in zip(e, t)) / st, (sum(e) - sum(t)) / st


# largest kappa_s the draws use: at kappa_ref = 1 no diffuse direction could
# be drawn, and recycled estimates at kappa_s < 1 would miss them
KAPPA_REF_MAX = 0.999


class SurfaceReconstruction:
    """Alg. 2 for the reflectometry workload (Sec. 6.2): theta = (kappa_s,
    gamma) of the unknown sphere lives on the device with its Adam moments;
    each iteration renders the recycled images, the loss and residual, the
    gradient in theta, one Adam step (per-parameter step sizes, box
    projection) and the correction-factor statistics at the new theta; the
    policy decides when to draw new paths at the current theta (Alg. 2's N_r
    or the drift / ESS triggers)."""

    def __init__(self, ctx: api.Context, scene, cams, measured: torch.Tensor, theta0, n_paths: int,
                 lr=(0.03, 3.0), policy: Policy | None = None, seed: int = 1, theta_true=None):
        self.ctx, self.scene, self.cams = ctx, scene, cams
        self.measured = measured.to(torch.float64).contiguous()
        dev = self.measured.device
        self.theta = torch.tensor([float(x) for x in theta0], dtype=torch.float64, device=dev)
        self.m = torch.zeros(2, dtype=torch.float64, device=dev)
        self.v = torch.zeros(2, dtype=torch.float64, device=dev)
        self.grad = torch.zeros(2, dtype=torch.float64, device=dev)
        self.stats = torch.zeros(2, dtype=torch.float64, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        self.img = torch.empty_like(self.measured)
        self.res = torch.empty_like(self.measured)
        self.n_paths, self.lr = int(n_paths), (float(lr[0]), float(lr[1]))
        self.policy = policy if policy is not None else Policy(period=30, drift=None)
        self.seed, self.theta_true = seed, theta_true
        self.t = 0
        self.t_ref = 0
        self.mean_r = self.ess_fraction = None
        self.store = None
        self.records: list = []

    def theta_host(self):
        return tuple(float(x) for x in self.theta.cpu())

    def close(self):
        if self.store is not None:
            self.store.close()
            self.store = None

    def step(self) -> SurfaceRecord:
        h = self.ctx.handle
        t0 = time.perf_counter()
        resampled = False
        if self.store is None or self.policy.resample(self.t, self.t_ref, self.mean_r, self.ess_fraction):
            if self.store is None:
                k, g = self.theta_host()
                ref = (min(k, KAPPA_REF_MAX), g)
                self.store = api.SurfacePaths.sample(self.ctx, self.scene, self.cams, ref, self.seed + self.t,
                                                     self.n_paths)
            else:
                # at the current theta on the device (the draw clamps kappa_s
                # to KAPPA_REF_MAX itself)
                self.store.resample(self.theta, self.seed + self.t, self.n_paths)
            self.t_ref = self.t
            resampled = True
        self.t += 1
        P.prt_surface_render(h, self.store.handle, self.theta, self.img)
        P.prt_loss(h, self.img, self.measured, self.res, self.loss)
        P.prt_surface_grad(h, self.store.handle, self.theta, self.res, self.grad)
        P.prt_surface_adam(h, self.theta, self.grad, self.m, self.v, self.t, *self.lr)
        P.prt_surface_reweight(h, self.store.handle, self.theta, self.stats)
        mean_r, ess = (float(x) for x in self.stats.cpu())
        self.mean_r, self.ess_fraction = mean_r, ess / self.n_paths
        theta = self.theta_host()
        eps = dlt = None
        if self.theta_true is not None:
            eps, dlt = param_errors(theta, self.theta_true)
        rec = SurfaceRecord(self.t, float(self.loss.item()), mean_r, ess, resampled, time.perf_counter() - t0, theta,
                            eps, dlt)
        self.records.append(rec)
        return rec

    def run(self, iters: int, callback=None, stop_epsilon: float | None = None):
        for _ in range(iters):
            rec = self.step()
            if callback:
                callback(rec)
            if stop_epsilon is not None and rec.epsilon is not None and rec.epsilon <= stop_epsilon:
                break
        return self.records
