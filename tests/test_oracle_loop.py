"""Pins of the oracle's loop glue: the sort, the loss and Adam."""
import numpy as np
import torch


def test_sort_is_stable_by_path_size(oracle_lib):
    rng = np.random.default_rng(1)
    B = rng.integers(0, 21, 5000)
    perm = oracle_lib.sort_permutation(B)
    assert (np.diff(B[perm]) >= 0).all()
    for b in range(21):
        ids = perm[B[perm] == b]
        assert (np.diff(ids) > 0).all()


def test_loss_and_residual():
    import oracle
    img = np.arange(12.0).reshape(3, 2, 2)
    tgt = np.ones_like(img)
    L, res = oracle.loss_and_residual(img, tgt)
    assert np.array_equal(res, img - 1) and L == 0.5 * ((img - 1) ** 2).sum()


def test_adam_matches_torch_then_projects():
    """Kingma & Ba's update as implemented by torch.optim.Adam, then beta >= 0."""
    import oracle
    rng = np.random.default_rng(2)
    beta = rng.uniform(0.0, 1.0, 50)
    p = torch.tensor(beta.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=0.1, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(50)
    v = np.zeros(50)
    for t in range(1, 6):
        g = rng.standard_normal(50)
        p.grad = torch.tensor(g)
        opt.step()
        with torch.no_grad():
            p.clamp_(min=0.0)
        beta, m, v = oracle.adam_step(beta, g, m, v, t, 0.1)
        assert np.allclose(beta, p.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_volume_errors_by_hand():
    """Sec. 6 error measures on a hand-worked case: true (1, 2, 3), estimate
    (2, 2, 1): ||b* - b||_1 = 1 + 0 + 2 = 3, ||b*||_1 = 6, ||b||_1 = 5."""
    import oracle
    eps, delta = oracle.volume_errors([2.0, 2.0, 1.0], [1.0, 2.0, 3.0])
    assert eps == 0.5 and abs(delta - 1.0 / 6.0) < 1e-15
    assert oracle.volume_errors([1.0, 2.0, 3.0], [1.0, 2.0, 3.0]) == (0.0, 0.0)


def test_downsampled_render_equals_coarse_render(oracle_lib):
    """Every local estimate lands in one fine pixel and hence in the coarse
    pixel holding it, so down-sampling the fine images reproduces the render
    with the coarse cameras on the same paths (up to projections that fall
    on a pixel edge within rounding)."""
    import inputs
    sc = inputs.cloud8()
    cams = inputs.arc_cameras(sc, [-30.0, 0.0, 30.0], 32, 32)
    paths = oracle_lib.sample(sc, 1001, 4000)
    fine = oracle_lib.render(sc, cams, paths)
    for k in (2, 4):
        coarse = oracle_lib.render(sc, inputs.coarse_cameras(cams, k), paths)
        down = oracle_lib.downsample_images(cams, fine, k)
        assert down.shape == coarse.shape
        assert np.abs(down - coarse).max() <= 1e-12 * np.abs(coarse).max()


def test_downsample_of_uniform_radiance_is_uniform():
    """A constant radiance stays constant whatever the pixel solid angles."""
    import inputs
    import oracle
    sc = inputs.cloud8()
    cams = inputs.arc_cameras(sc, [0.0, 45.0], 12, 12)
    img = np.full((2, 12, 12), 3.5)
    for k in (2, 3, 4, 6):
        assert np.allclose(oracle.downsample_images(cams, img, k), 3.5, rtol=1e-15, atol=0)
