"""Pins of the reflectometry oracle (Sec. 6.2) against what the paper and the
mathematics fix, independent of the oracle's own formulas:

- ray-sphere and nearest-surface hits against numpy's polynomial roots and
  plane intersections;
- the direction draw at the unknown sphere against the density the estimator
  divides by (chi-square on binned directions), and its mean continuation
  weight against the directional albedo by quadrature (Eq.
  brdf_conservation);
- the unknown sphere at kappa_s = 0 renders exactly like a diffuse sphere of
  albedo 1 (same draws, same weights);
- single-bounce images against the direct-illumination closed form of a point
  light (Eq. surface_rendering with one bounce), pixel by pixel, within the
  Monte Carlo error; two-bounce images of an empty box against quadrature of
  the once-reflected light (the second bounce is half of each pixel there);
- the gradient against central differences of the recycled loss on the same
  paths (Eq. gradient_simualtion_recycling is the exact derivative of Eq.
  forward_simualtion_recycling);
- the correction factor: r = 1 at theta_ref, E[r] = 1, and recycled images
  equal to freshly drawn ones within the Monte Carlo error (Sec. 5.2);
- path invariants: vertices on their surfaces, consecutive vertices mutually
  visible, early ends only at the unknown sphere.
"""
import numpy as np
import pytest

import inputs
import oracle.surface as S


def _rand_unit(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def test_sphere_hit_matches_polynomial_roots():
    rng = np.random.default_rng(3)
    hits = 0
    for _ in range(400):
        c = rng.uniform(0.3, 0.7, 3)
        r = rng.uniform(0.05, 0.2)
        p = rng.uniform(0.0, 1.0, 3)
        if np.linalg.norm(p - c) <= r:
            continue
        # half the rays aim near the sphere so that hits and misses both occur
        w = _rand_unit(rng) if rng.uniform() < 0.5 else c + rng.uniform(-1.5, 1.5, 3) * r - p
        w = w / np.linalg.norm(w)
        roots = np.roots([1.0, 2.0 * np.dot(p - c, w), np.dot(p - c, p - c) - r * r])
        real = [x.real for x in roots if abs(x.imag) < 1e-12 and x.real > 0]
        want = min(real) if real else np.inf
        got = S.sphere_hit(c, r, p, w)
        if np.isinf(want):
            assert np.isinf(got)
        else:
            hits += 1
            assert abs(got - want) <= 1e-10, (got, want)
    assert hits > 20


def test_nearest_surface_brute_force():
    scene = inputs.smallpaint()
    rng = np.random.default_rng(4)
    for _ in range(300):
        p = rng.uniform(0.01, 0.99, 3)
        if np.any(np.linalg.norm(scene.centers - p, axis=1) <= scene.radii):
            continue
        w = _rand_unit(rng)
        cands = []
        for a in range(3):
            for wall, plane in ((2 * a, 0.0), (2 * a + 1, 1.0)):
                if w[a] != 0:
                    t = (plane - p[a]) / w[a]
                    if t > 0:
                        cands.append((t, wall))
        for k, (c, r) in enumerate(zip(scene.centers, scene.radii)):
            roots = np.roots([1.0, 2.0 * np.dot(p - c, w), np.dot(p - c, p - c) - r * r])
            for x in roots:
                if abs(x.imag) < 1e-12 and x.real > 0:
                    cands.append((x.real, 6 + k))
        t_ref, id_ref = min(cands)
        sid, t = S.nearest(scene, p, w)
        assert sid == id_ref and abs(t - t_ref) <= 1e-9


def _frame(n):
    a = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(n, a)
    e1 /= np.linalg.norm(e1)
    return e1, np.cross(n, e1)


@pytest.mark.parametrize("kappa,gamma", [(0.7, 50.0), (0.3, 5.0)])
def test_phong_draws_follow_the_density_divided_by(kappa, gamma):
    """Directions drawn at the unknown sphere (oracle draw) binned in the
    mirror frame follow the mixture density that the estimator divides by
    (chi-square); lobe draws below the surface end the path, so the density
    is integrated over the bins including the part below the surface."""
    scene = inputs.surface_box([((0.5, 0.5, 0.5), 0.2, 0.0)], phong=0)
    rng = np.random.default_rng(5)
    x = np.array([0.5, 0.5 + 0.2, 0.5])          # top of the sphere, n = +y
    n = np.array([0.0, 1.0, 0.0])
    w_in = np.array([0.6, -0.8, 0.0])            # arriving obliquely
    wr = w_in - 2 * np.dot(w_in, n) * n
    e1, e2 = _frame(wr)
    nb_mu, nb_phi = 10, 8
    # bins in (cos to the mirror direction, azimuth about it), lobe region
    # mu in [mu_lo, 1]
    mu_lo = 0.5 if gamma > 10 else -1.0
    edges = np.linspace(mu_lo, 1.0, nb_mu + 1)
    counts = np.zeros((nb_mu, nb_phi))
    N = 40000
    for i in range(N):
        u = rng.uniform(0, 1, 3)
        ok, wo, _ = S.bounce(scene, 6, (kappa, gamma), x, w_in, u)
        if not ok:
            continue
        mu = float(np.dot(wo, wr))
        if mu < mu_lo:
            continue
        phi = np.arctan2(np.dot(wo, e2), np.dot(wo, e1)) % (2 * np.pi)
        counts[min(np.searchsorted(edges, mu) - 1, nb_mu - 1), int(phi / (2 * np.pi) * nb_phi) % nb_phi] += 1
    # expected: the density over each bin by midpoint quadrature on a fine grid
    expect = np.zeros_like(counts)
    sub = 24
    for a in range(nb_mu):
        mus = edges[a] + (np.arange(sub) + 0.5) / sub * (edges[a + 1] - edges[a])
        for b in range(nb_phi):
            phis = (b + (np.arange(sub) + 0.5) / sub) * 2 * np.pi / nb_phi
            acc = 0.0
            for m in mus:
                st = np.sqrt(max(0.0, 1 - m * m))
                for ph in phis:
                    d = m * wr + st * (np.cos(ph) * e1 + np.sin(ph) * e2)
                    nc = float(np.dot(n, d))
                    if nc > 0:
                        acc += S.phong_pdf(kappa, gamma, nc, m)
            expect[a, b] = acc * (edges[a + 1] - edges[a]) / sub * (2 * np.pi / nb_phi) / sub * N
    chi2 = float(((counts - expect) ** 2 / np.maximum(expect, 1e-9)).sum())
    dof = counts.size
    assert chi2 < dof + 6 * np.sqrt(2 * dof), (chi2, dof)


@pytest.mark.parametrize("kappa,gamma", [(0.7, 50.0), (0.4, 8.0)])
def test_mean_bounce_weight_is_directional_albedo(kappa, gamma):
    """E[f |n.w| / pdf] over the oracle's draws (0 for a draw that ends the
    path) equals the directional albedo integral of f |n.w| over the
    hemisphere (Eq. brdf_conservation), computed by quadrature in the
    normal's frame; it stays at most 1."""
    scene = inputs.surface_box([((0.5, 0.5, 0.5), 0.2, 0.0)], phong=0)
    x = np.array([0.5, 0.7, 0.5])
    n = np.array([0.0, 1.0, 0.0])
    w_in = np.array([0.5, -np.sqrt(0.75), 0.0])
    wr = w_in - 2 * np.dot(w_in, n) * n
    e1, e2 = _frame(n)
    # quadrature: mu = cos to n (Gauss-Legendre), phi uniform
    gl, gw = np.polynomial.legendre.leggauss(200)
    mus, mw = 0.5 * (gl + 1.0), 0.5 * gw
    phis = (np.arange(720) + 0.5) / 720 * 2 * np.pi
    alb = 0.0
    for m, wm in zip(mus, mw):
        st = np.sqrt(1 - m * m)
        d = m * n[:, None] + st * (np.cos(phis)[None, :] * e1[:, None] + np.sin(phis)[None, :] * e2[:, None])
        c = wr @ d
        lobe = np.where(c > 0, np.abs(c) ** gamma, 0.0)
        f = (1 - kappa) / np.pi + kappa * (gamma + 2) / (2 * np.pi) * lobe
        alb += wm * float((f * m).sum()) * (2 * np.pi / 720)
    rng = np.random.default_rng(6)
    N = 60000
    ws = np.zeros(N)
    for i in range(N):
        ok, _, wt = S.bounce(scene, 6, (kappa, gamma), x, w_in, rng.uniform(0, 1, 3))
        ws[i] = wt if ok else 0.0
    se = ws.std() / np.sqrt(N)
    assert abs(ws.mean() - alb) < 5 * se + 1e-4, (ws.mean(), alb, se)
    assert alb <= 1.0 + 1e-6


def test_phong_at_kappa_zero_is_a_white_diffuse_sphere():
    sph = [((0.5, 0.45, 0.55), 0.2, 1.0), ((0.25, 0.2, 0.3), 0.08, 0.6)]
    s_ph = inputs.surface_box(sph, phong=0, max_order=6)
    s_df = inputs.surface_box(sph, phong=-1, max_order=6)
    cam = inputs.cameras_at([[0.5, 0.5, 0.03]], [[0.5, 0.45, 0.55]], 12, 12, 10.0)
    pa = S.sample(s_ph, (0.0, 30.0), 11, 4000)
    pb = S.sample(s_df, (0.0, 30.0), 11, 4000)
    assert np.array_equal(pa.B, pb.B) and np.array_equal(pa.sid, pb.sid)
    assert np.array_equal(pa.pos, pb.pos)
    ia, ib = S.render(s_ph, cam, pa, (0.0, 30.0)), S.render(s_df, cam, pb, (0.0, 30.0))
    assert np.abs(ia - ib).max() <= 1e-12 * np.abs(ib).max()
    assert ib.max() > 0


def _pixel_rays(cams, sub):
    """Sub-pixel ray directions (world) and their exact solid angles."""
    f, W, H = float(cams.f_px[0]), cams.width, cams.height
    R = cams.rot[0]

    def F(x, y):
        return np.arctan(x * y / (f * np.sqrt(x * x + y * y + f * f)))

    out = []
    for r in range(H):
        for c in range(W):
            rays = []
            for i in range(sub):
                for j in range(sub):
                    x1, y1 = c - W / 2 + j / sub, r - H / 2 + i / sub
                    x2, y2 = x1 + 1 / sub, y1 + 1 / sub
                    om = F(x2, y2) - F(x1, y2) - F(x2, y1) + F(x1, y1)
                    d = R.T @ np.array([x1 + 0.5 / sub, y1 + 0.5 / sub, f])
                    rays.append((d / np.linalg.norm(d), om))
            out.append(rays)
    return out


def test_single_bounce_matches_point_light_closed_form():
    """max_order = 1: each pixel is the pixel-averaged radiance of the
    surfaces it sees, each lit directly by the point light:
    L = f(w_l -> w_v) I0 cos(theta_l) / d_l^2 (zero in the sphere's shadow),
    integrated over sub-pixels by their exact solid angles."""
    kappa, gamma = 0.6, 12.0
    scene = inputs.surface_box([((0.5, 0.45, 0.6), 0.2, 0.0)], phong=0, wall_albedo=[0.5, 0.6, 0.7, 0.8, 0.9, 0.65],
                               light=(0.3, 0.85, 0.4), max_order=1, intensity=2.0)
    cam = inputs.cameras_at([[0.5, 0.5, 0.03]], [[0.5, 0.45, 0.6]], 6, 6, 4.5)
    c0, r0 = scene.centers[0], scene.radii[0]
    ref = np.zeros(36)
    for p, rays in enumerate(_pixel_rays(cam, 24)):
        acc = om_tot = 0.0
        for d, om in rays:
            om_tot += om
            sid, t = S.nearest(scene, cam.pos[0], d)
            x = cam.pos[0] + t * d
            if sid < 6:
                n = np.zeros(3)
                n[sid // 2] = 1.0 if sid % 2 == 0 else -1.0
            else:
                n = (x - c0) / r0
            to_l = scene.light - x
            dl = np.linalg.norm(to_l)
            ul = to_l / dl
            cos_l = float(np.dot(n, ul))
            if cos_l <= 0:
                continue
            if sid < 6:
                # shadow of the sphere: does the segment x -> light cut it?
                q = x - c0
                b = np.dot(q, ul)
                disc = b * b - (np.dot(q, q) - r0 * r0)
                if disc > 0 and 0 < -b - np.sqrt(disc) < dl:
                    continue
                f = scene.wall_albedo[sid] / np.pi
            else:
                wl = -ul                                  # propagation direction of the light
                wr = wl - 2 * np.dot(wl, n) * n
                wv = -d
                cr = float(np.dot(wr, wv))
                f = (1 - kappa) / np.pi + kappa * (gamma + 2) / (2 * np.pi) * (max(cr, 0.0) ** gamma)
            acc += om * f * scene.intensity * cos_l / dl ** 2
        ref[p] = acc / om_tot
    # Monte Carlo: batches give the standard error of each pixel
    nb, per = 20, 100_000
    imgs = np.array([S.render(scene, cam, S.sample(scene, (kappa, gamma), 40 + k, per), (kappa, gamma)).ravel()
                     for k in range(nb)])
    mean, se = imgs.mean(0), imgs.std(0, ddof=1) / np.sqrt(nb)
    z = np.abs(mean - ref) / np.maximum(se, 1e-12)
    assert np.all(z < 5.0), (z.max(), mean, ref)
    assert np.abs(mean.sum() - ref.sum()) <= 0.01 * ref.sum()


def _loss(img, target):
    return 0.5 * float(((img - target) ** 2).sum())


def test_gradient_matches_central_differences_on_the_same_paths():
    scene = inputs.smallpaint(max_order=6)
    cam = inputs.smallpaint_camera(scene, 16)
    paths = S.sample(scene, (0.5, 20.0), 21, 20000)
    theta = np.array([0.55, 24.0])
    target = S.render(scene, cam, paths, (0.7, 40.0)) * 1.1
    img = S.render(scene, cam, paths, theta)
    g = S.grad(scene, cam, paths, img - target, theta)
    for k, h in ((0, 1e-5), (1, 1e-4)):
        e = np.zeros(2)
        e[k] = h
        fd = (_loss(S.render(scene, cam, paths, theta + e), target) -
              _loss(S.render(scene, cam, paths, theta - e), target)) / (2 * h)
        assert abs(g[k] - fd) <= 1e-6 * abs(fd) + 1e-12, (k, g[k], fd)


def test_correction_factor_and_recycled_images():
    scene = inputs.smallpaint(max_order=6)
    cam = inputs.smallpaint_camera(scene, 8)
    ref = (0.5, 20.0)
    paths = S.sample(scene, ref, 31, 200_000)
    lr = S.log_r(scene, paths, ref)
    assert np.all(lr == 0.0)
    mean_r, ess = S.reweight(scene, paths, ref)
    assert mean_r == 1.0 and abs(ess - paths.n) < 1e-6 * paths.n
    tt = (0.65, 30.0)
    r = np.exp(S.log_r(scene, paths, tt))
    assert abs(r.mean() - 1.0) < 5 * r.std() / np.sqrt(paths.n)
    # recycled F(theta_t | theta_ref) against fresh paths drawn at theta_t:
    # equal within their joint Monte Carlo error (batch estimates)
    nb = 10
    rec = np.array([S.render(scene, cam, S.sample(scene, ref, 100 + k, 40_000), tt).ravel() for k in range(nb)])
    fre = np.array([S.render(scene, cam, S.sample(scene, tt, 200 + k, 40_000), tt).ravel() for k in range(nb)])
    se = np.sqrt(rec.var(0, ddof=1) / nb + fre.var(0, ddof=1) / nb)
    z = np.abs(rec.mean(0) - fre.mean(0)) / np.maximum(se, 1e-12)
    assert np.all(z < 5.0), z.max()


def test_path_invariants():
    scene = inputs.smallpaint()
    paths = S.sample(scene, (0.7, 50.0), 41, 5000)
    M = scene.max_order
    assert np.all((paths.B >= 1) & (paths.B <= M))
    short = paths.B < M
    assert short.any()
    assert np.all(paths.sid[short, paths.B[short] - 1] == 6 + scene.phong)
    for i in range(0, paths.n, 17):
        prev = scene.light
        for b in range(paths.B[i]):
            x, sid = paths.pos[i, b], paths.sid[i, b]
            if sid < 6:
                assert x[sid // 2] == (0.0 if sid % 2 == 0 else 1.0)
            else:
                k = sid - 6
                assert abs(np.linalg.norm(x - scene.centers[k]) - scene.radii[k]) <= 1e-12
            d = x - prev
            L = np.linalg.norm(d)
            skip = -1 if b == 0 else paths.sid[i, b - 1]
            sid2, t = S.nearest(scene, prev, d / L, skip)
            assert sid2 == sid and abs(t - L) <= 1e-9 * max(L, 1.0)
            prev = x


def _wall_points(n):
    """Midpoints, inward normals, areas and wall ids of an n x n grid of
    patches on each wall of the unit box."""
    g = (np.arange(n) + 0.5) / n
    u, v = np.meshgrid(g, g, indexing="ij")
    u, v = u.ravel(), v.ravel()
    pts, nrm, ids = [], [], []
    for w in range(6):
        a = w // 2
        o = [k for k in range(3) if k != a]
        p = np.zeros((n * n, 3))
        p[:, a] = 0.0 if w % 2 == 0 else 1.0
        p[:, o[0]], p[:, o[1]] = u, v
        nn = np.zeros(3)
        nn[a] = 1.0 if w % 2 == 0 else -1.0
        pts.append(p)
        nrm.append(np.tile(nn, (n * n, 1)))
        ids.append(np.full(n * n, w))
    return np.concatenate(pts), np.concatenate(nrm), np.full(6 * n * n, 1.0 / (n * n)), np.concatenate(ids)


def test_two_bounces_match_quadrature():
    """max_order = 2 in an empty box: each pixel is the direct radiance of the
    wall it sees plus the once-reflected radiance, the integral over every
    other wall point y of (rho_x/pi) L1(y -> x) cos_x cos_y / |x - y|^2 with
    L1 = (rho_y/pi) I0 cos_l / d_l^2 (Eq. surface_rendering applied twice),
    by midpoint quadrature over 48 x 48 patches per wall and 4 x 4 rays per
    pixel; the oracle's path-traced image agrees within its Monte Carlo
    error plus a 0.5 % quadrature allowance."""
    rho = np.array([0.5, 0.6, 0.7, 0.8, 0.9, 0.65])
    scene = inputs.surface_box([], phong=-1, wall_albedo=rho, light=(0.3, 0.8, 0.45), max_order=2, intensity=1.0)
    # a narrow view of the back wall keeps every seen point 0.25 or more from
    # the other walls, where the reflected-light integrand is smooth
    cam = inputs.cameras_at([[0.5, 0.5, 0.05]], [[0.5, 0.45, 1.0]], 5, 5, 10.0)
    Y, NY, AY, WY = _wall_points(48)
    lt = scene.light
    dl = lt - Y
    r2l = (dl * dl).sum(1)
    L1 = rho[WY] / np.pi * scene.intensity * np.maximum((NY * dl).sum(1), 0) / r2l ** 1.5
    ref = np.zeros(25)
    for p, rays in enumerate(_pixel_rays(cam, 4)):
        acc = om_tot = 0.0
        for d, om in rays:
            om_tot += om
            sid, t = S.nearest(scene, cam.pos[0], d)
            x = cam.pos[0] + t * d
            n = np.zeros(3)
            n[sid // 2] = 1.0 if sid % 2 == 0 else -1.0
            to_l = lt - x
            direct = rho[sid] / np.pi * scene.intensity * max(float(n @ to_l), 0.0) / np.linalg.norm(to_l) ** 3
            dy = Y - x
            r2 = (dy * dy).sum(1)
            cx = (dy @ n) / np.sqrt(r2)
            cy = -(NY * dy).sum(1) / np.sqrt(r2)
            ok = (WY != sid) & (cx > 0) & (cy > 0)
            indirect = rho[sid] / np.pi * float((L1 * cx * cy / r2 * AY)[ok].sum())
            acc += om * (direct + indirect)
        ref[p] = acc / om_tot
    nb, per = 20, 100_000
    imgs = np.array([S.render(scene, cam, S.sample(scene, (0.5, 10.0), 60 + k, per), (0.5, 10.0)).ravel()
                     for k in range(nb)])
    mean, se = imgs.mean(0), imgs.std(0, ddof=1) / np.sqrt(nb)
    assert np.all(np.abs(mean - ref) <= 5 * se + 0.005 * ref), (mean / ref - 1, se / ref)
    assert abs(mean.sum() / ref.sum() - 1) < 0.005
