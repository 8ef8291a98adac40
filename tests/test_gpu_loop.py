"""GPU tests of the loop glue around the hot path (Alg. 2 and Sec. 6.1),
through the C ABI: down-sampled measurements, the Sec. 6 error measures and
space carving against the oracle, and short runs of the Alg. 2 driver with
its resampling policy and coarse-to-fine stages."""
import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2110_00085_amd import api, prt
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    prt.lib()
    return torch, prt, api


def test_downsample_and_volume_errors_match_oracle(env):
    torch, P, api = env
    ctx = api.Context(0)
    sc = inputs.cloud8()
    cams = inputs.arc_cameras(sc, [-30.0, 0.0, 30.0, 50.0], 48, 48)
    rng = np.random.default_rng(21)
    img = rng.uniform(0.0, 2.0, (cams.n, 48, 48))
    ch = P.CamerasHost(cams)
    img_d = torch.as_tensor(img).cuda()
    for k in (1, 2, 3, 4, 8, 16):
        say(f"downsample 48 -> {48 // k}")
        out = torch.empty((cams.n, 48 // k, 48 // k), dtype=torch.float64, device="cuda")
        P.prt_downsample_images(ctx.handle, ch, img_d, k, out)
        ref = oracle.downsample_images(cams, img, k)
        # solid angles from atan on each side (libm ulps) and a different summation order
        err = float(np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max())
        assert err <= 1e-12, err
    with pytest.raises(P.PrtError) as e:
        P.prt_downsample_images(ctx.handle, ch, img_d, 5, out)
    assert e.value.code == P.PRT_E_INVALID
    for n in (1, 1000, 4096 * 3 + 17):
        say(f"volume errors, n = {n}")
        est = rng.uniform(0.0, 5.0, n)
        tru = rng.uniform(0.0, 5.0, n).astype(np.float32)
        err = torch.zeros(2, dtype=torch.float64, device="cuda")
        est_d, tru_d = torch.as_tensor(est).cuda(), torch.as_tensor(tru).cuda()
        P.prt_volume_errors(ctx.handle, est_d, tru_d, err)
        e_ref, d_ref = oracle.volume_errors(est, tru)
        got = err.cpu().numpy()
        de, dd = float(abs(got[0] - e_ref) / abs(e_ref)), float(abs(got[1] - d_ref))
        assert de <= 1e-12 and dd <= 1e-12, (de, dd)


def test_space_carve_matches_oracle(env):
    """The photo hull of rendered images of a cloud, against the oracle's, for
    thresholds at several image levels."""
    torch, P, api = env
    ctx = api.Context(0)
    sc = inputs.cloud8()
    cams = inputs.cloud8_cameras(sc)
    paths = oracle.sample(sc, 1001, 20_000)
    img = oracle.render(sc, cams, paths)
    ch = P.CamerasHost(cams)
    img_d = torch.as_tensor(img).cuda()
    mask = torch.empty((sc.nz, sc.ny, sc.nx), dtype=torch.uint8, device="cuda")
    beta = torch.empty((sc.nz, sc.ny, sc.nx), dtype=torch.float32, device="cuda")
    dummy = torch.as_tensor(sc.beta_cloud).cuda()
    for q in (0.1, 0.3, 0.6):
        thr = [float(np.quantile(img[d], q)) for d in range(cams.n)]
        say(f"space carve, per-camera thresholds at the {q} quantile")
        P.prt_space_carve(ctx.handle, P.make_scene(sc, dummy), ch, img_d, thr, 7.5, mask, beta)
        ref = oracle.space_carve(sc, cams, img, thr)
        got = mask.cpu().numpy()
        same = bool(np.array_equal(got, ref))
        assert same, int((got != ref).sum())
        same = bool(np.array_equal(beta.cpu().numpy(), np.where(ref == 1, 7.5, 0.0).astype(np.float32)))
        assert same
        kept = int(ref.sum())
        assert 0 < kept < ref.size, kept


def test_alg2_loop_reduces_loss_and_mass_bias(env):
    """A short reconstruction of the 8^3 cloud from the true field scaled by
    0.6 (every voxel too thin): resampling every 5 iterations, two
    coarse-to-fine stages (4 x 4 and 16 x 16 pixels).  On the paths of each
    stage's first resampling window the loss is a deterministic function of
    beta, and it falls over the window; the mass bias |delta| falls over the
    run; the policy's resamples happen where it says; every record is finite.
    (Per-voxel epsilon is not asserted: at this N the per-voxel gradient noise
    moves Adam's normalised steps in both directions.)  The space-carved start
    of the same images is checked for sanity (it keeps part of the grid)."""
    torch, P, api = env
    from paper_2110_00085_amd.loop import Policy, Reconstruction, Stage, space_carved_start
    ctx = api.Context(0)
    sc = inputs.cloud8()
    cams = inputs.arc_cameras(sc, [-45.0, -15.0, 15.0, 45.0], 16, 16)
    truth = torch.as_tensor(sc.beta_cloud).cuda()
    st = api.PathStore.sample(ctx, sc, truth, 9001, 1_000_000)
    measured = api.render(ctx, sc, truth, P.CamerasHost(cams), st)
    st.close()
    thr = [0.05 * float(measured[d].max()) for d in range(cams.n)]
    mean_ext = float(sc.beta_cloud[sc.beta_cloud > 0].mean())
    carved, mask = space_carved_start(ctx, sc, cams, measured, thr, mean_ext)
    kept = int(mask.sum())
    say(f"space-carved start: {kept} of {mask.numel()} voxels kept, fill {mean_ext:.2f}")
    assert 0 < kept < mask.numel()
    assert bool(((carved == mean_ext) == (mask == 1)).all())
    beta0 = (0.6 * truth).contiguous()
    rec = Reconstruction(ctx, sc, cams, measured, beta0, lr=0.3, policy=Policy(period=5, drift=None), seed=500,
                         beta_true=truth)
    stages = [Stage(factor=4, n_paths=100_000, max_iters=12, window=100),
              Stage(factor=1, n_paths=200_000, max_iters=12, window=100)]
    records = rec.run(stages, callback=lambda r: say(
        f"  stage {r.stage} it {r.iteration}: loss {r.loss:.4e} eps {r.epsilon:.3f} delta {r.delta:+.3f} "
        f"mean r {r.mean_r:.3f} resampled {r.resampled}"))
    rec.close()
    assert len(records) == 24
    for r in records:
        assert np.isfinite([r.loss, r.mean_r, r.ess, r.epsilon, r.delta]).all()
    for k in (0, 1):
        rs = [r for r in records if r.stage == k]
        assert rs[0].resampled  # a stage starts from fresh paths
        assert [r.iteration for r in rs if r.resampled] == [rs[0].iteration + 5 * j for j in range(3)]
        assert not any(r.resampled for r in rs[1:5])
        assert rs[4].loss < rs[0].loss, (k, rs[0].loss, rs[4].loss)
    assert abs(records[-1].delta) < abs(records[0].delta)
