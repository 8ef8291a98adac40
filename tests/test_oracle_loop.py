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
