"""Pins of the oracle's space carving (Sec. 6.1, photo-hull initialisation):
in the orthographic limit the photo hull of silhouette images is the
intersection of the silhouettes' extrusions along the viewing directions (the
visual hull); a camera that sees no voxel removes nothing."""
import numpy as np

import inputs


def _far_cameras(n, voxel_km, dist_km=1000.0):
    """A camera far above the box looking down (image u along +x, v along +y)
    and one far on the -x side looking along +x (u along +z, v along +y),
    each framing the n^3 box with one pixel per voxel column; and a third
    looking away from the box."""
    L = n * voxel_km
    c = 0.5 * L
    f = 0.5 * n / (0.5 * L / dist_km)
    pos = [[c, c, c + dist_km], [c - dist_km, c, c], [c, c, c + dist_km]]
    tgt = [[c, c, c], [c, c, c], [c, c, c + 2 * dist_km]]
    return inputs.cameras_at(pos, tgt, n, n, f)


def test_orthographic_photo_hull_is_the_visual_hull(oracle_lib):
    n = 5
    sc = inputs.homogeneous((n, n, n), voxel_km=0.1, beta=1.0)
    cams = _far_cameras(n, sc.voxel_km)
    rng = np.random.default_rng(12)
    top = rng.integers(0, 2, (n, n))    # [row = iy][col = ix]
    side = rng.integers(0, 2, (n, n))   # [row = iy][col = iz]
    images = np.stack([top, side, np.zeros((n, n))]).astype(np.float64)
    mask = oracle_lib.space_carve(sc, cams, images, 0.5)
    iz, iy, ix = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    expect = (top[iy, ix] == 1) & (side[iy, iz] == 1)
    assert mask.dtype == np.uint8
    assert np.array_equal(mask.astype(bool), expect)
    assert 0 < expect.sum() < n ** 3
    # without the side view, the hull is the top silhouette extruded along z
    only_top = inputs.Cameras(1, n, n, cams.pos[:1], cams.rot[:1], cams.f_px[:1])
    m1 = oracle_lib.space_carve(sc, only_top, images[:1], 0.5)
    assert np.array_equal(m1.astype(bool), np.broadcast_to(top == 1, (n, n, n)))


def test_threshold_is_inclusive_and_per_camera(oracle_lib):
    n = 4
    sc = inputs.homogeneous((n, n, n), voxel_km=0.1, beta=1.0)
    cams = _far_cameras(n, sc.voxel_km)
    images = np.stack([np.full((n, n), 2.0), np.full((n, n), 3.0), np.zeros((n, n))])
    assert oracle_lib.space_carve(sc, cams, images, [1.0, 2.0, 0.0]).all()
    assert not oracle_lib.space_carve(sc, cams, images, [2.0, 2.0, 0.0]).any()
    assert not oracle_lib.space_carve(sc, cams, images, [1.0, 3.0, 0.0]).any()
