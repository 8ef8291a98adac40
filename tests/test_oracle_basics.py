"""Pins of the oracle's building blocks against facts fixed outside the oracle:
an independent Philox implementation (rocRAND), closed forms, quadrature,
brute force and library routines."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import integrate, stats
from scipy.spatial import ConvexHull

import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


# ------------------------------------------------------------------ RNG

@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.check_call(["hipcc", "-x", "hip", "--offload-arch=gfx950", "-O1", "-o", exe,
                           os.path.join(HERE, "ref", "philox_rocrand_ref.cpp")])
    return exe


def test_philox_matches_rocrand(oracle_lib, rocrand_ref):
    """Philox4x32-10 (Salmon et al., SC'11) bit-equal to rocRAND's engine on
    2000 random (seed, path, event) triples, counter = (path, event, 0); paths below 2^62 so that rocRAND's
    4*path offset does not wrap."""
    rng = np.random.default_rng(7)
    triples = [(int(rng.integers(0, 2**63)), int(rng.integers(0, 2**40)), int(rng.integers(0, 64)))
               for _ in range(2000)] + [(0, 0, 0), (2**64 - 1, 2**62 - 1, 2**32 - 1)]
    inp = "\n".join(f"{s} {p} {e}" for s, p, e in triples) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(x) for x in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)
    for (s, p, e), r in zip(triples, ref):
        k = [s & 0xFFFFFFFF, s >> 32]
        c = [p & 0xFFFFFFFF, (p >> 32) & 0xFFFFFFFF, e, 0]
        assert (oracle_lib.philox4x32_10(k, c).astype(np.uint64) == r).all(), (s, p, e)


def test_uniforms_open_interval_and_uniform(oracle_lib):
    u = np.array([oracle_lib.uniforms(99, i, e) for i in range(4000) for e in range(3)]).ravel()
    assert (u > 0).all() and (u < 1).all()
    assert stats.kstest(u, "uniform").pvalue > 1e-4


# ------------------------------------------------------- phase functions

@pytest.mark.parametrize("g", [0.85, 0.6, 0.0, -0.3])
def test_hg_normalised_mean_cosine_and_cdf(oracle_lib, g):
    """int f dOmega = 1 (Eq. phase_conservation) and <mu> = g by quadrature;
    the sampler inverts the numerically integrated CDF."""
    f = lambda mu: oracle_lib.phase_hg(mu, g)
    norm = 2 * np.pi * integrate.quad(f, -1, 1, epsabs=1e-13, epsrel=1e-12, limit=200)[0]
    mean = 2 * np.pi * integrate.quad(lambda m: m * f(m), -1, 1, epsabs=1e-13, epsrel=1e-12, limit=200)[0]
    assert abs(norm - 1) < 1e-10
    assert abs(mean - g) < 1e-10
    for u in [1e-6, 0.01, 0.3, 0.5, 0.77, 0.999]:
        mu = oracle_lib.sample_hg(u, g)
        cdf = 2 * np.pi * integrate.quad(f, -1, mu, epsabs=1e-14, epsrel=1e-12, limit=200)[0]
        assert abs(cdf - u) < 1e-9, (u, mu, cdf)


def test_rayleigh_normalised_moments_and_cdf(oracle_lib):
    f = oracle_lib.phase_rayleigh
    assert abs(2 * np.pi * integrate.quad(f, -1, 1)[0] - 1) < 1e-12
    assert abs(2 * np.pi * integrate.quad(lambda m: m * f(m), -1, 1)[0]) < 1e-12
    assert abs(2 * np.pi * integrate.quad(lambda m: m * m * f(m), -1, 1)[0] - 0.4) < 1e-12
    for u in [1e-7, 0.1, 0.5, 0.9, 1 - 1e-7]:
        mu = oracle_lib.sample_rayleigh(u)
        cdf = 2 * np.pi * integrate.quad(f, -1, mu)[0]
        assert abs(cdf - u) < 1e-11


def test_new_direction_orthonormal_basis(oracle_lib):
    rng = np.random.default_rng(3)
    for _ in range(300):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        mu = rng.uniform(-1, 1)
        phi = rng.uniform(0, 2 * np.pi)
        w = oracle_lib.new_direction(n, mu, phi)
        assert abs(np.linalg.norm(w) - 1) < 1e-14
        assert abs(w @ n - mu) < 1e-12
        # azimuth phi and phi+pi give opposite perpendicular parts; phi and
        # phi+pi/2 give orthogonal ones (an orthonormal basis around n)
        e_a = oracle_lib.new_direction(n, 0.0, phi)
        e_b = oracle_lib.new_direction(n, 0.0, phi + np.pi / 2)
        e_c = oracle_lib.new_direction(n, 0.0, phi + np.pi)
        assert abs(e_a @ e_b) < 1e-12 and abs(e_a @ n) < 1e-12
        assert np.allclose(e_a, -e_c, atol=1e-12)
    # the pole n = (0,0,-1) and n = (0,0,1) are handled
    for nz in (-1.0, 1.0):
        w = oracle_lib.new_direction([0, 0, nz], 0.3, 1.0)
        assert abs(w[2] * nz - 0.3) < 1e-14


# ------------------------------------------------------------ ray pieces

def _brute_lengths(scene, p, w, tmax, m=400_000):
    """Per-voxel lengths by dense midpoint sampling of the segment."""
    t = (np.arange(m) + 0.5) / m * tmax
    x = p[None, :] + t[:, None] * w[None, :]
    n = np.array([scene.nx, scene.ny, scene.nz])
    inside = np.all((x >= 0) & (x < n), axis=1)
    idx = np.floor(x[inside]).astype(int)
    v = idx[:, 0] + scene.nx * (idx[:, 1] + scene.ny * idx[:, 2])
    return np.bincount(v, minlength=scene.n_voxels) * (tmax / m)


def test_ray_pieces_sum_and_brute_force(oracle_lib):
    scene = inputs.homogeneous((5, 7, 6))
    rng = np.random.default_rng(11)
    for _ in range(40):
        p = rng.uniform([0, 0, 0], [5, 7, 6])
        q = rng.uniform([0, 0, 0], [5, 7, 6])
        d = q - p
        L = np.linalg.norm(d)
        vox, ln, tend = oracle_lib.ray_pieces(scene, p, d / L, L)
        assert abs(ln.sum() - L) < 1e-12 * max(1, L)
        assert abs(tend - L) < 1e-12
        got = np.bincount(vox, weights=ln, minlength=scene.n_voxels)
        ref = _brute_lengths(scene, p, d / L, L)
        assert np.abs(got - ref).max() < 3 * L / 400_000 + 1e-12


def test_ray_pieces_axis_aligned_edges_and_clipping(oracle_lib):
    scene = inputs.homogeneous((4, 4, 4))
    # along x through the interior of row (iy, iz) = (1, 2)
    vox, ln, _ = oracle_lib.ray_pieces(scene, [0.0, 1.5, 2.5], [1.0, 0.0, 0.0], 10.0)
    assert list(vox) == [0 + 4 * (1 + 4 * 2) + i for i in range(4)] and np.allclose(ln, 1.0)
    # exactly along a grid edge x=y (through corners): total length preserved
    w = np.array([1.0, 1.0, 0.0]) / np.sqrt(2)
    vox, ln, tend = oracle_lib.ray_pieces(scene, [0.0, 0.0, 0.5], w, 100.0)
    assert abs(ln.sum() - 4 * np.sqrt(2)) < 1e-12 and abs(tend - 4 * np.sqrt(2)) < 1e-12
    # a ray starting outside the box is clipped to the box
    vox, ln, tend = oracle_lib.ray_pieces(scene, [-1.0, 0.5, 0.5], [1.0, 0.0, 0.0], 100.0)
    assert abs(ln.sum() - 4.0) < 1e-12 and abs(tend - 5.0) < 1e-12


# --------------------------------------------------------- camera model

def test_pixel_solid_angles_by_quadrature(oracle_lib):
    f, W, H = 20.0, 6, 4
    om = oracle_lib.pixel_solid_angles(f, W, H)
    dens = lambda y, x: f / (x * x + y * y + f * f) ** 1.5
    for r, c in [(0, 0), (1, 2), (3, 5)]:
        x1, y1 = c - W / 2, r - H / 2
        ref = integrate.dblquad(dens, x1, x1 + 1, y1, y1 + 1, epsabs=1e-14, epsrel=1e-12)[0]
        assert abs(om[r, c] - ref) < 1e-12
    total = integrate.dblquad(dens, -W / 2, W / 2, -H / 2, H / 2, epsabs=1e-14, epsrel=1e-12)[0]
    assert abs(om.sum() - total) < 1e-12


def test_projection_centre_and_behind(oracle_lib):
    cams = inputs.cameras_at([[0.0, 0.0, 10.0]], [[0.0, 0.0, 0.0]], 8, 6, 50.0)
    assert oracle_lib.project(cams, 0, [0.001, 0.001, 0.0]) == 3 * 8 + 4
    assert oracle_lib.project(cams, 0, [0.0, 0.0, 20.0]) == -1      # behind
    assert oracle_lib.project(cams, 0, [100.0, 0.0, 0.0]) == -1     # outside the image


def test_source_weight_is_flux_times_projected_box_area(oracle_lib):
    """w0 = F0 * (area of the box projected along the sun direction), checked
    against the convex hull of the projected corners."""
    for zen, az in [(30.0, 0.0), (0.0, 0.0), (55.0, 130.0)]:
        sc = inputs.homogeneous((3, 5, 2), voxel_km=0.2, sun_zenith_deg=zen, sun_azimuth_deg=az, sun_flux=2.5)
        th, ph = np.deg2rad(zen), np.deg2rad(az)
        w = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), -np.cos(th)])
        a = np.cross(w, [1.0, 0.0, 0.0] if abs(w[0]) < 0.9 else [0.0, 1.0, 0.0])
        a /= np.linalg.norm(a)
        b = np.cross(w, a)
        L = np.array([3, 5, 2]) * 0.2
        corners = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)]) * L
        area = ConvexHull(np.stack([corners @ a, corners @ b], 1)).volume
        assert abs(oracle_lib.source_weight(sc) - 2.5 * area) < 1e-12
