"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds no arithmetic of the method: only extinction fields, optical
constants, camera placement and target images.  The paper's datasets (LES
clouds, the Mitsuba plume) are not available; these fields stand in for them
with the paper's shapes (Sec. 6.1, Table scene_settings):

- ``cloud8``     8^3 grid, 50 m voxels, a log-normal sphere of cloud.
- ``cloud32``    32^3 grid, 20 m voxels, a smoothed-and-thresholded Gaussian
                 random field (stands in for the single LES cloud, 32x36x25).
- ``plume64``    64^3 grid, 20 m voxels, a noisy Gaussian plume.
- ``field128``   128x128x64 grid, 20 m voxels, ten log-normal ellipsoid blobs
                 (stands in for the LES cloud field, 79x84x27).

- ``smallpaint``  reflectometry box (Sec. 6.2): a unit box, one large sphere
                 with the unknown Phong BRDF, 14 small diffuse spheres, a
                 point light and one 60x60 camera (stands in for the
                 Smallpaint scene).

Air: constant 0.01 1/km, albedo 1, Rayleigh.  Sun at 30 deg zenith, F0 = 1.
Cameras sit on an arc in the x-z plane, look at the box centre with +y up, at
distance 2.5 x the box's bounding radius, field of view 2 asin(1/2.5).
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np


@dataclass
class Scene:
    nx: int
    ny: int
    nz: int
    voxel_km: float
    beta_cloud: np.ndarray          # float32 [nz][ny][nx], 1/km, x fastest
    beta_air: float = 0.01
    albedo_cloud: float = 0.99
    albedo_air: float = 1.0
    g: float = 0.85
    sun_zenith_deg: float = 30.0
    sun_azimuth_deg: float = 0.0
    sun_flux: float = 1.0
    max_order: int = 10

    @property
    def n_voxels(self) -> int:
        return self.nx * self.ny * self.nz

    def with_beta(self, beta) -> "Scene":
        return replace(self, beta_cloud=np.ascontiguousarray(beta, dtype=np.float32).reshape(self.nz, self.ny, self.nx))


@dataclass
class Cameras:
    n: int
    width: int
    height: int
    pos: np.ndarray     # [n][3] km
    rot: np.ndarray     # [n][3][3] world->camera rows: right, up, forward
    f_px: np.ndarray    # [n] focal length in pixels


def arc_cameras(scene: Scene, zeniths_deg, width: int, height: int, dist_factor: float = 2.5) -> Cameras:
    """Pinhole cameras on an arc in the x-z plane looking at the box centre."""
    L = np.array([scene.nx, scene.ny, scene.nz], np.float64) * scene.voxel_km
    centre = 0.5 * L
    r_box = 0.5 * float(np.linalg.norm(L))
    R = dist_factor * r_box
    fov = 2.0 * np.arcsin(r_box / R)
    f_px = 0.5 * width / np.tan(0.5 * fov)
    pos, rot = [], []
    for z in zeniths_deg:
        th = np.deg2rad(abs(z))
        ph = 0.0 if z >= 0 else np.pi
        p = centre + R * np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
        fwd = centre - p
        fwd /= np.linalg.norm(fwd)
        right = np.cross(fwd, np.array([0.0, 1.0, 0.0]))
        right /= np.linalg.norm(right)
        up = np.cross(right, fwd)
        pos.append(p)
        rot.append(np.stack([right, up, fwd]))
    n = len(pos)
    return Cameras(n, width, height, np.array(pos), np.array(rot), np.full(n, f_px))


def cameras_at(positions_km, targets_km, width: int, height: int, f_px: float) -> Cameras:
    """Pinhole cameras at given positions looking at given targets (+y up,
    falling back to +x up when looking along y)."""
    pos, rot = [], []
    for p, t in zip(np.asarray(positions_km, float), np.asarray(targets_km, float)):
        fwd = t - p
        fwd /= np.linalg.norm(fwd)
        hint = np.array([0.0, 1.0, 0.0]) if abs(fwd[1]) < 0.9 else np.array([1.0, 0.0, 0.0])
        right = np.cross(fwd, hint)
        right /= np.linalg.norm(right)
        up = np.cross(right, fwd)
        pos.append(p)
        rot.append(np.stack([right, up, fwd]))
    n = len(pos)
    return Cameras(n, width, height, np.array(pos), np.array(rot), np.full(n, float(f_px)))


def coarse_cameras(cams: Cameras, factor: int) -> Cameras:
    """The same pinhole cameras with images `factor` times smaller per side
    (focal length and image sides divided by `factor`), so that coarse pixel
    (r, c) covers fine pixels factor*r .. factor*r + factor - 1 (same for c)."""
    if cams.width % factor or cams.height % factor:
        raise ValueError("image sides must be multiples of the factor")
    return Cameras(cams.n, cams.width // factor, cams.height // factor, cams.pos, cams.rot,
                   np.asarray(cams.f_px, np.float64) / factor)


# ------------------------------------------------------------ fields

def _centre_dist(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    return np.sqrt((x - nx / 2) ** 2 + (y - ny / 2) ** 2 + (z - nz / 2) ** 2)


def cloud8(seed: int = 1) -> Scene:
    """8^3, 50 m voxels: beta = 20 exp(0.5 z), z ~ N(0,1), inside a centred
    sphere of radius 3 voxels, 0 elsewhere; w_c 0.99, g 0.85, 10 orders."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((8, 8, 8))
    beta = np.where(_centre_dist(8, 8, 8) <= 3.0, 20.0 * np.exp(0.5 * z), 0.0).astype(np.float32)
    return Scene(8, 8, 8, 0.05, beta, albedo_cloud=0.99, g=0.85, max_order=10)


def cloud8_cameras(scene: Scene) -> Cameras:
    return arc_cameras(scene, [-30.0, 0.0, 30.0], 16, 16)


def gaussian_field_cloud(n: int, seed: int, peak: float = 60.0, sigma: float = 3.0, thresh: float = 0.6):
    """White N(0,1) -> Gaussian filter (sigma voxels, periodic) -> min-max to
    [0,1] -> peak*(u - thresh)/(1 - thresh) where u > thresh, else 0."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    w = gaussian_filter(rng.standard_normal((n, n, n)), sigma, mode="wrap")
    u = (w - w.min()) / (w.max() - w.min())
    return np.where(u > thresh, peak * (u - thresh) / (1.0 - thresh), 0.0).astype(np.float32)


def cloud32(seed: int = 2, max_order: int = 20) -> Scene:
    """32^3, 20 m voxels, smoothed random cloud (0-60 1/km); w 0.99, g 0.85."""
    return Scene(32, 32, 32, 0.02, gaussian_field_cloud(32, seed), albedo_cloud=0.99, g=0.85,
                 max_order=max_order)


def cloud32_cameras(scene: Scene, width: int = 64) -> Cameras:
    return arc_cameras(scene, np.arange(-60.0, 61.0, 15.0), width, width)


def plume64(seed: int = 4, max_order: int = 20) -> Scene:
    """64^3, 20 m voxels: 80 exp(-r^2/(2*12^2)) (1 + 0.3 n), n smoothed
    (sigma 2), re-standardised white noise clipped to +-3; w 0.9, g 0.6."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    nz = gaussian_filter(rng.standard_normal((64, 64, 64)), 2.0, mode="wrap")
    nz = np.clip((nz - nz.mean()) / nz.std(), -3.0, 3.0)
    r = _centre_dist(64, 64, 64)
    beta = (80.0 * np.exp(-r * r / (2 * 12.0 ** 2)) * (1.0 + 0.3 * nz)).astype(np.float32)
    return Scene(64, 64, 64, 0.02, beta, albedo_cloud=0.9, g=0.6, max_order=max_order)


def plume64_cameras(scene: Scene, width: int = 128) -> Cameras:
    return arc_cameras(scene, np.arange(-60.0, 61.0, 15.0), width, width)


def field128(seed: int = 5, max_order: int = 30) -> Scene:
    """128x128x64, 20 m voxels: 10 ellipsoid blobs with i.i.d. lognormal(3, 0.7)
    extinction inside; w 0.999, g 0.85."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = 128, 128, 64
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    inside = np.zeros((nz, ny, nx), bool)
    for _ in range(10):
        cx, cy = rng.uniform(16, 112, 2)
        cz = rng.uniform(16, 40)
        rh = rng.uniform(6, 14)
        rv = 0.7 * rh
        inside |= ((x - cx) ** 2 + (y - cy) ** 2) / rh ** 2 + (z - cz) ** 2 / rv ** 2 <= 1.0
    beta = np.where(inside, rng.lognormal(3.0, 0.7, (nz, ny, nx)), 0.0).astype(np.float32)
    return Scene(nx, ny, nz, 0.02, beta, albedo_cloud=0.999, g=0.85, max_order=max_order)


def field128_cameras(scene: Scene, width: int = 256) -> Cameras:
    return arc_cameras(scene, np.linspace(-60.0, 60.0, 20), width, width)


def homogeneous(n=(4, 4, 4), voxel_km=0.1, beta=5.0, **kw) -> Scene:
    nx, ny, nz = n
    return Scene(nx, ny, nz, voxel_km, np.full((nz, ny, nx), beta, np.float32), **kw)


def random_field(n=(4, 4, 4), voxel_km=0.1, lo=0.5, hi=8.0, seed=0, **kw) -> Scene:
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    return Scene(nx, ny, nz, voxel_km, rng.uniform(lo, hi, (nz, ny, nx)).astype(np.float32), **kw)


def target_images(shape, mean_value: float, seed: int = 11) -> np.ndarray:
    """Random target images I_gt = U(0,1) * 2 * mean_value."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, shape) * 2.0 * mean_value


# ------------------------------------------------------------ reflectometry

@dataclass
class SurfaceScene:
    """Closed box [0, box]^3 with diffuse walls and spheres; sphere `phong`
    carries the unknown BRDF.  Walls in the order x=0, x=box, y=0, y=box, z=0,
    z=box.  An isotropic point light of radiant intensity `intensity` sits at
    `light`.  Paths keep at most `max_order` surface vertices."""
    box: float
    wall_albedo: np.ndarray     # [6]
    light: np.ndarray           # [3]
    intensity: float
    centers: np.ndarray         # [n][3]
    radii: np.ndarray           # [n]
    albedo: np.ndarray          # [n] (the Phong sphere's entry is unused)
    phong: int
    max_order: int = 10

    @property
    def n_spheres(self) -> int:
        return int(len(self.radii))


def smallpaint(seed: int = 7, max_order: int = 10) -> SurfaceScene:
    """Stand-in for the Smallpaint box of the reflectometry test: a unit box,
    a large sphere of radius 0.2 at its centre (the unknown BRDF) and 14 small
    diffuse spheres (radius 0.04-0.07, albedo 0.4-0.9) placed at seeded random
    positions that keep clear of each other, the walls, the light, and the
    lines from the camera and from the light to the large sphere; the light
    hangs under the ceiling."""
    rng = np.random.default_rng(seed)
    centre = np.array([0.5, 0.42, 0.6])
    light = np.array([0.5, 0.92, 0.45])
    cam = np.array([0.5, 0.5, 0.03])
    centers, radii = [centre], [0.2]

    def seg_dist(c, a, b):
        t = np.clip(np.dot(c - a, b - a) / np.dot(b - a, b - a), 0.0, 1.0)
        return np.linalg.norm(c - (a + t * (b - a)))

    while len(radii) < 15:
        r = rng.uniform(0.04, 0.07)
        c = rng.uniform(r + 0.02, 1.0 - r - 0.02, 3)
        c[2] = max(c[2], 0.2)
        if all(np.linalg.norm(c - c2) > r + r2 + 0.02 for c2, r2 in zip(centers, radii)) and \
                seg_dist(c, cam, centre) > r + 0.2 and seg_dist(c, light, centre) > r + 0.2 and \
                np.linalg.norm(c - light) > r + 0.05:
            centers.append(c)
            radii.append(r)
    albedo = np.concatenate([[0.0], rng.uniform(0.4, 0.9, 14)])
    return SurfaceScene(1.0, np.array([0.75, 0.75, 0.8, 0.8, 0.6, 0.8]), light, 1.0, np.array(centers),
                        np.array(radii), albedo, 0, max_order)


def smallpaint_camera(scene: SurfaceScene, width: int = 60) -> Cameras:
    """One pinhole camera inside the box near the front wall, looking at the
    large sphere, 60 degree field of view."""
    f_px = 0.5 * width / np.tan(np.deg2rad(30.0))
    return cameras_at([[0.5, 0.5, 0.03]], [[0.5, 0.42, 0.6]], width, width, f_px)


def surface_box(spheres=(), phong: int = -1, wall_albedo=0.7, light=(0.5, 0.85, 0.5), max_order: int = 10,
                intensity: float = 1.0) -> SurfaceScene:
    """Unit box with the given spheres [(centre, radius, albedo), ...];
    `phong` names the sphere with the unknown BRDF (-1: none)."""
    c = np.array([s[0] for s in spheres], np.float64).reshape(-1, 3)
    r = np.array([s[1] for s in spheres], np.float64)
    a = np.array([s[2] for s in spheres], np.float64)
    wa = np.full(6, wall_albedo, np.float64) if np.isscalar(wall_albedo) else np.asarray(wall_albedo, np.float64)
    return SurfaceScene(1.0, wa, np.asarray(light, np.float64), intensity, c, r, a, phong, max_order)


# reflectometry workload registry: name -> (scene factory, camera factory,
# paths, seed, true (kappa_s, gamma)); Sec. 6.2: one 60x60 camera, 1.8e6
# paths, truth kappa_s = 0.7, gamma = 50
SURFACE_WORKLOADS = {
    "smallpaint60": (smallpaint, smallpaint_camera, 1_800_000, 2001, (0.7, 50.0)),
}


# workload registry: name -> (scene factory, camera factory, paths, seed)
WORKLOADS = {
    "cloud8": (cloud8, cloud8_cameras, 10_000, 1001),
    "cloud32": (cloud32, cloud32_cameras, 1 << 22, 1002),
    "plume64": (plume64, plume64_cameras, 1 << 26, 1004),
    "field128": (field128, field128_cameras, 1 << 28, 1005),
}
