"""Pins of the oracle's sampler, recycled renderer, correction factor and
gradient against closed forms, independent estimators and exact identities."""
import numpy as np
import pytest
from scipy import stats

import inputs


def _batches(values, k=20):
    """Mean and standard error of the mean from k equal batches."""
    v = np.asarray(values, float)
    b = v[: len(v) // k * k].reshape(k, -1).sum(axis=1) / (len(v) // k)
    return b.mean(), b.std(ddof=1) / np.sqrt(k)


# ------------------------------------------------------------- sampling

def test_sampled_vertices_are_consistent(oracle_lib):
    """Vertices lie in their stored voxel, exits lie on the boundary, and at
    albedo 1 with a high order cap every path leaves the box."""
    sc = inputs.random_field((6, 5, 4), voxel_km=0.1, lo=0.5, hi=6.0, seed=2, albedo_cloud=1.0,
                             albedo_air=1.0, max_order=60)
    P = oracle_lib.sample(sc, 123, 20000)
    n = np.array([sc.nx, sc.ny, sc.nz])
    nv = np.diff(P.off)
    assert (nv == P.B + 2).all()            # all exited (none capped at 60)
    for i in range(0, P.n, 37):
        xs = P.xyz[P.off[i]:P.off[i + 1]].astype(float)
        vs = P.vox[P.off[i]:P.off[i + 1]]
        assert (xs >= -1e-5).all() and (xs <= n + 1e-5).all()
        for x, v in zip(xs[1:-1], vs[1:-1]):
            idx = np.array([v % sc.nx, (v // sc.nx) % sc.ny, v // (sc.nx * sc.ny)])
            assert (x >= idx - 1e-5).all() and (x <= idx + 1 + 1e-5).all()
        assert vs[-1] == -1 and np.min(np.minimum(np.abs(xs[-1]), np.abs(xs[-1] - n))) < 1e-5


def test_free_flight_depth_is_truncated_exponential(oracle_lib):
    """Sec. 3.4.1: with the sun at zenith over a homogeneous column, the first
    scatter depth follows Exp(beta) truncated at the column height."""
    beta = 2.0
    sc = inputs.homogeneous((4, 4, 40), voxel_km=0.1, beta=beta, beta_air=0.0, sun_zenith_deg=0.0,
                            max_order=1)
    P = oracle_lib.sample(sc, 5, 40000)
    first = P.off[:-1] + 1
    depth = (sc.nz - P.xyz[first, 2].astype(float)) * sc.voxel_km
    depth = depth[P.B >= 1]
    H = sc.nz * sc.voxel_km
    cdf = lambda s: (1 - np.exp(-beta * s)) / (1 - np.exp(-beta * H))
    assert stats.kstest(depth, cdf).pvalue > 1e-4


def _hg_cdf(mu, g):
    return (1 - g * g) / (2 * g) * (1 / np.sqrt(1 + g * g - 2 * g * mu) - 1 / (1 + g))


def _ray_cdf(mu):
    return (mu ** 3 + 3 * mu + 4) / 8


def _first_cosines(P):
    rows = P.B >= 1
    i0 = P.off[:-1][rows]
    x0, x1, x2 = (P.xyz[i0 + k].astype(float) for k in range(3))
    w0 = (x1 - x0) / np.linalg.norm(x1 - x0, axis=1)[:, None]
    w1 = (x2 - x1) / np.linalg.norm(x2 - x1, axis=1)[:, None]
    return (w0 * w1).sum(1)


@pytest.mark.parametrize("mix", ["cloud", "air", "both"])
def test_direction_sampling_distribution(oracle_lib, mix):
    """Sec. 3.4.2: the first scattering cosine follows HG (cloud), Rayleigh
    (air), or their mixture with weights beta_s^(j)/beta_s (reading of the
    particle-choice probability that makes the albedo weight exact)."""
    g = 0.6
    if mix == "cloud":
        sc = inputs.homogeneous((6, 6, 6), beta=4.0, beta_air=0.0, g=g, albedo_cloud=0.8)
        cdf = lambda m: _hg_cdf(m, g)
    elif mix == "air":
        sc = inputs.homogeneous((6, 6, 6), beta=0.0, beta_air=4.0, g=g, albedo_air=0.8)
        cdf = _ray_cdf
    else:
        sc = inputs.homogeneous((6, 6, 6), beta=1.0, beta_air=1.0, g=g, albedo_cloud=0.5, albedo_air=1.0)
        pc = 0.5 / 1.5
        cdf = lambda m: pc * _hg_cdf(m, g) + (1 - pc) * _ray_cdf(m)
    sc.max_order = 3
    P = oracle_lib.sample(sc, 17, 60000)
    mu = _first_cosines(P)
    assert stats.kstest(mu, cdf).pvalue > 1e-4


def test_unscattered_fraction_beer_lambert(oracle_lib):
    """Eq. transmittance: P(B = 0) = (1/A) int exp(-beta L(x0)) dA over the
    projected box, by midpoint quadrature over the lit faces."""
    beta, vk = 3.0, 0.1
    sc = inputs.homogeneous((4, 4, 4), voxel_km=vk, beta=beta, beta_air=0.0, sun_zenith_deg=30.0, max_order=2)
    N = 200000
    P = oracle_lib.sample(sc, 77, N)
    p_hat = (P.B == 0).mean()
    L = 0.4
    th = np.deg2rad(30.0)
    w = np.array([np.sin(th), 0.0, -np.cos(th)])
    m = 600
    g = (np.arange(m) + 0.5) / m * L
    # top face (z = L): chord until x = L or z = 0
    X, Y = np.meshgrid(g, g, indexing="ij")
    t_top = np.minimum((L - X) / w[0], L / -w[2])
    # x = 0 face: chord until x = L or z = 0
    Yx, Zx = np.meshgrid(g, g, indexing="ij")
    t_x = np.minimum(L / w[0], Zx / -w[2])
    a_top, a_x = L * L * abs(w[2]), L * L * abs(w[0])
    p_ref = (a_top * np.exp(-beta * t_top).mean() + a_x * np.exp(-beta * t_x).mean()) / (a_top + a_x)
    sig = np.sqrt(p_ref * (1 - p_ref) / N)
    assert abs(p_hat - p_ref) < 4 * sig + 1e-4, (p_hat, p_ref, sig)


# ------------------------------------------------------------ rendering

def test_single_scatter_slab_closed_form(oracle_lib):
    """Order-1 image of a wide homogeneous slab seen from nadir against the
    single-scattering radiance L = w F0 f(Theta) mu0/(mu0+mu) (1 - exp(-tau (1/mu0 + 1/mu)))
    (integrated RTE, Eq. integrated_RTE, truncated at one scattering)."""
    beta, g, alb = 5.0, 0.85, 0.9
    sc = inputs.homogeneous((40, 40, 2), voxel_km=0.05, beta=beta, beta_air=0.0, g=g, albedo_cloud=alb,
                            sun_zenith_deg=30.0, max_order=1)
    H = 2 * 0.05
    cx = cy = 1.0
    Zc = 10.0
    cams = inputs.cameras_at([[cx, cy, H + Zc]], [[cx, cy, 0.0]], 8, 8, 4 / (0.25 / Zc))
    N = 4_000_000
    P = oracle_lib.sample(sc, 31, N)
    k = 16
    parts = []
    for j in range(k):
        sub = P.subset(np.arange(j * N // k, (j + 1) * N // k))
        sub.n_total = N // k
        parts.append(oracle_lib.render(sc, cams, sub, max_order_render=1)[0])
    parts = np.array(parts)
    img = parts.mean(0)
    se = parts.std(0, ddof=1) / np.sqrt(k)
    # per-pixel reference: view direction through the pixel centre
    mu0 = np.cos(np.deg2rad(30.0))
    w0 = np.array([np.sin(np.deg2rad(30.0)), 0.0, -mu0])
    R = cams.rot[0]
    f = cams.f_px[0]
    ref = np.zeros((8, 8))
    for r in range(8):
        for c in range(8):
            dcam = np.array([c + 0.5 - 4, r + 0.5 - 4, f])
            dworld = R.T @ dcam
            dworld /= np.linalg.norm(dworld)
            to_cam = -dworld
            mu = to_cam[2]
            cos_t = w0 @ to_cam
            fhg = (1 - g * g) / (4 * np.pi * (1 + g * g - 2 * g * cos_t) ** 1.5)
            tau = beta * H
            ref[r, c] = alb * 1.0 * fhg * mu0 / (mu0 + mu) * (1 - np.exp(-tau * (1 / mu0 + 1 / mu)))
    rel = abs(img.mean() - ref.mean()) / ref.mean()
    assert rel < 0.005, rel
    assert np.all(np.abs(img - ref) < 5 * se), np.abs(img - ref).max() / se.min()


def _exit_estimator(sc, P, cone_dir, alpha):
    """Far-field radiant intensity averaged over a cone, estimated from the
    escaping scattered paths (weight w0 * prod of effective albedos)."""
    w0 = None
    nv = np.diff(P.off)
    vals = np.zeros(P.n)
    bc = sc.beta_cloud.ravel().astype(float)
    alb = (sc.albedo_cloud * bc + sc.albedo_air * sc.beta_air) / (bc + sc.beta_air)
    cosa = np.cos(alpha)
    for i in np.nonzero((P.B >= 1) & (nv == P.B + 2))[0]:
        a, b = P.off[i], P.off[i + 1]
        xl, xp = P.xyz[b - 1].astype(float), P.xyz[b - 2].astype(float)
        d = xl - xp
        d /= np.linalg.norm(d)
        if d @ cone_dir >= cosa:
            vals[i] = np.prod(alb[P.vox[a + 1:b - 1]])
    return vals


@pytest.mark.parametrize("view", ["zenith", "side"])
def test_local_estimation_matches_escape_counting(oracle_lib, view):
    """All scattering orders: the local estimate to far cameras (Sec. 3.4.3,
    Eq. Qd) and counting the escaping paths are two estimators of the same
    radiant intensity; their cone averages agree within 4 sigma."""
    sc = inputs.random_field((6, 6, 6), voxel_km=0.1, lo=1.0, hi=4.0, seed=8, beta_air=0.01,
                             albedo_cloud=0.7, albedo_air=1.0, g=0.5, sun_zenith_deg=30.0, max_order=60)
    axis = np.array([0.0, 0.0, 1.0]) if view == "zenith" else np.array([-np.sin(1.0), 0.0, np.cos(1.0)])
    alpha = np.deg2rad(25.0)
    # cameras on Gauss-Legendre nodes in cos(theta) x uniform azimuths within the cone
    xg, wg = np.polynomial.legendre.leggauss(3)
    cth = np.cos(alpha) + (1 - np.cos(alpha)) * (xg + 1) / 2
    e1 = np.cross(axis, [0.0, 1.0, 0.0]); e1 /= np.linalg.norm(e1)
    e2 = np.cross(axis, e1)
    centre = 0.3 * np.ones(3)
    Rd = 500.0
    dirs, wts = [], []
    for c, wc in zip(cth, wg):
        for k in range(6):
            ph = 2 * np.pi * (k + 0.5) / 6
            s = np.sqrt(1 - c * c)
            dirs.append(c * axis + s * (np.cos(ph) * e1 + np.sin(ph) * e2))
            wts.append(wc)
    dirs, wts = np.array(dirs), np.array(wts) / np.sum(wts)
    cams = inputs.cameras_at(centre + Rd * dirs, np.repeat(centre[None], len(dirs), 0), 4, 4,
                             2.0 / np.tan(0.7 / Rd))
    N = 200000
    P = oracle_lib.sample(sc, 2024, N)
    img = oracle_lib.render(sc, cams, P)
    om = oracle_lib.pixel_solid_angles(cams.f_px[0], 4, 4)
    pos = cams.pos
    J = np.array([(img[d] * om).sum() * np.sum((pos[d] - centre) ** 2) for d in range(cams.n)])
    J_le = float(wts @ J)
    vals = _exit_estimator(sc, P, axis, alpha) * oracle_lib.source_weight(sc) / (2 * np.pi * (1 - np.cos(alpha)))
    mean, se = _batches(vals)
    assert abs(J_le - mean) < 4 * se, (J_le, mean, se)


def _qd_image(oracle_lib, sc, cams, P):
    """Plain local-estimation estimator (Eq. Qd): w0 * prod_{k<=b} albedo(x_k) *
    f_p(x_b, cos to camera) * T(x_b, camera) / r^2 / Omega_p, summed in numpy."""
    bc = sc.beta_cloud.ravel().astype(float)
    img = np.zeros((cams.n, cams.height, cams.width))
    w0 = oracle_lib.source_weight(sc)
    om = [oracle_lib.pixel_solid_angles(f, cams.width, cams.height) for f in cams.f_px]
    g = sc.g
    for i in range(P.n):
        xs = P.xyz[P.off[i]:P.off[i + 1]].astype(float)
        vs = P.vox[P.off[i]:P.off[i + 1]]
        prod = 1.0
        for b in range(1, P.B[i] + 1):
            v = vs[b]
            bs = sc.albedo_cloud * bc[v] + sc.albedo_air * sc.beta_air
            bt = bc[v] + sc.beta_air
            prod *= bs / bt
            win = (xs[b] - xs[b - 1]) / np.linalg.norm(xs[b] - xs[b - 1])
            for d in range(cams.n):
                pix = oracle_lib.project(cams, d, xs[b] * sc.voxel_km)
                if pix < 0:
                    continue
                cg = cams.pos[d] / sc.voxel_km
                dv = cg - xs[b]
                dist = np.linalg.norm(dv)
                wd = dv / dist
                mu = win @ wd
                fp = (sc.albedo_cloud * bc[v] * (1 - g * g) / (4 * np.pi * (1 + g * g - 2 * g * mu) ** 1.5)
                      + sc.albedo_air * sc.beta_air * 3 * (1 + mu * mu) / (16 * np.pi)) / bs
                vox, ln, _ = oracle_lib.ray_pieces(sc, xs[b], wd, dist)
                T = np.exp(-np.sum((bc[vox] + sc.beta_air) * ln) * sc.voxel_km)
                r2 = (dist * sc.voxel_km) ** 2
                img[d].flat[pix] += w0 * prod * fp * T / r2 / om[d].flat[pix]
    return img / P.n_total


def test_recycled_render_reduces_to_plain_estimator_at_reference(oracle_lib):
    """At beta_t = beta_ref the recycled estimator (f/mu with the correction
    factor, Eq. forward_simualtion_recycling_factor) equals Eq. Qd term by term."""
    sc = inputs.cloud8()
    cams = inputs.cloud8_cameras(sc)
    P = oracle_lib.sample(sc, 1001, 400)
    img = oracle_lib.render(sc, cams, P)
    ref = _qd_image(oracle_lib, sc, cams, P)
    assert np.abs(img - ref).max() <= 1e-11 * np.abs(ref).max()
    assert np.abs(ref).max() > 0


def test_recycled_render_is_unbiased_and_mean_r_is_one(oracle_lib):
    """IS unbiasedness (Eq. unbiasedness): images rendered at beta_t from paths
    drawn at beta_ref agree with images from paths drawn at beta_t; and the
    correction factor has mean 1 under the reference pdf."""
    base = inputs.random_field((5, 5, 5), voxel_km=0.1, lo=0.5, hi=6.0, seed=4, g=0.7, max_order=30)
    rng = np.random.default_rng(9)
    beta_t = (base.beta_cloud * (1 + 0.3 * rng.uniform(-1, 1, base.beta_cloud.shape))).astype(np.float32)
    cams = inputs.arc_cameras(base, [-30.0, 20.0], 6, 6)
    N = 120000
    P_ref = oracle_lib.sample(base, 55, N)
    P_new = oracle_lib.sample(base.with_beta(beta_t), 56, N)
    k = 20
    per = []
    for P, bt in ((P_ref, beta_t), (P_new, beta_t)):
        imgs = []
        for j in range(k):
            sub = P.subset(np.arange(j * N // k, (j + 1) * N // k))
            sub.n_total = N // k
            imgs.append(oracle_lib.render(base, cams, sub, beta_t=bt).sum(axis=(1, 2)))
        imgs = np.array(imgs)
        per.append((imgs.mean(0), imgs.std(0, ddof=1) / np.sqrt(k)))
    (m1, s1), (m2, s2) = per
    assert np.all(np.abs(m1 - m2) < 4 * np.sqrt(s1 ** 2 + s2 ** 2)), (m1, m2, s1, s2)
    r = np.exp(oracle_lib.log_r(base, P_ref, beta_t=beta_t))
    mean, se = _batches(r)
    assert abs(mean - 1) < 4 * se, (mean, se)
    # at beta_t = beta_ref the factor is exactly 1
    assert np.abs(oracle_lib.log_r(base, P_ref)).max() == 0.0


def test_correction_factor_is_zero_exactly_for_impossible_paths(oracle_lib):
    """The path pdf (Eq. final_mu) carries the extinction of every scatter
    vertex: with no air and beta_t = 0 in one voxel, exactly the paths that
    scatter in that voxel have r = 0 (log r = -inf), every other r is finite
    and positive, and no NaN appears."""
    sc = inputs.cloud8()
    sc.beta_air = 0.0
    P = oracle_lib.sample(sc, 77, 4000)
    scat = [set(P.vox[P.off[i] + 1:P.off[i] + 1 + P.B[i]].tolist()) for i in range(P.n)]
    v0 = int(np.bincount(np.concatenate([list(x) for x in scat if x])).argmax())
    beta_t = sc.beta_cloud.ravel().copy()
    beta_t[v0] = 0.0
    lr = oracle_lib.log_r(sc, P, beta_t=beta_t.reshape(sc.beta_cloud.shape))
    hits = np.array([v0 in x for x in scat])
    assert hits.sum() > 20
    assert np.array_equal(np.isneginf(lr), hits)
    assert np.isfinite(lr[~hits]).all()


# --------------------------------------------------------------- gradient

def test_gradient_matches_central_differences(oracle_lib):
    """For fixed stored paths the recycled estimator is a smooth function of
    beta_t; its derivative (Eq. gradient_simualtion_recycling with the
    tomography PSF) must match central finite differences on every voxel of a
    4^3 grid."""
    sc = inputs.random_field((4, 4, 4), voxel_km=0.1, lo=0.5, hi=8.0, seed=21, beta_air=0.01,
                             albedo_cloud=0.9, g=0.85, max_order=12)
    cams = inputs.arc_cameras(sc, [-40.0, 0.0, 35.0], 8, 8)
    P = oracle_lib.sample(sc, 404, 3000)
    rng = np.random.default_rng(5)
    beta_t = (sc.beta_cloud * (1 + 0.2 * rng.uniform(-1, 1, sc.beta_cloud.shape))).astype(np.float64)
    rho = rng.standard_normal((cams.n, cams.height, cams.width))
    phi = lambda b: float((rho * oracle_lib.render(sc, cams, P, beta_t=b)).sum())
    # render takes FP32 fields; perturb in float64 and pass float32-exact values
    g = oracle_lib.grad(sc, cams, P, rho, beta_t=beta_t.astype(np.float32)).ravel()
    bt32 = beta_t.astype(np.float32).astype(np.float64).ravel()
    fd = np.zeros_like(g)
    for v in range(sc.n_voxels):
        h = 2.0 ** -8
        bp, bm = bt32.copy(), bt32.copy()
        bp[v] += h
        bm[v] -= h
        fd[v] = (phi(bp.reshape(sc.beta_cloud.shape).astype(np.float32))
                 - phi(bm.reshape(sc.beta_cloud.shape).astype(np.float32))) / (2 * h)
    scale = np.abs(g).max()
    assert scale > 0
    assert np.abs(g - fd).max() < 1e-5 * scale, np.abs(g - fd).max() / scale
