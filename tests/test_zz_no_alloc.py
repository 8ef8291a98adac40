"""The no-allocation variant of the correction-factor statistics
(prt_reweight_noalloc, for callers that cannot allocate device memory)
against prt_reweight on the same stores, through the C ABI: two calls in a
row, the second with a smaller input, in both precision modes; a grid whose
field beta_t - beta_ref exceeds the LDS (kept in the library's fixed scratch)
and one that fits the LDS; and the capacity error beyond the scratch."""
import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)


def _case(torch, api, P, ctx, scene, n, seed):
    beta = torch.as_tensor(scene.beta_cloud).cuda()
    st = api.PathStore.sample(ctx, scene, beta, seed, n)
    rng = np.random.default_rng(seed)
    bt = (scene.beta_cloud * (1 + 0.2 * rng.uniform(-1, 1, scene.beta_cloud.shape))).astype(np.float32)
    bt_d = torch.as_tensor(bt).cuda()  # kept alive: the scene holds only its address
    sc = P.make_scene(scene, bt_d)
    mr, ess = P.prt_reweight(ctx.handle, sc, st.handle)
    stats = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    P.prt_reweight_noalloc(ctx.handle, sc, st.handle, stats)
    torch.cuda.synchronize()
    got = stats.cpu().numpy()
    st.close()
    return (mr, ess), got


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_reweight_noalloc_equals_reweight(prec):
    import torch
    from paper_2110_00085_amd import api, prt as P
    assert torch.cuda.is_available()
    ctx = api.Context(0, P.PRT_ALL_FP64 if prec == "fp64" else P.PRT_TRAVERSAL_FP32)
    # 64^3 plume (its field exceeds the LDS: kept in the scratch array), then
    # the smaller 8^3 cloud (field in LDS) with fewer paths
    cases = [(inputs.plume64(max_order=12), 1 << 16, 4001), (inputs.cloud8(), 5_000, 4002)]
    for scene, n, seed in cases:
        say(f"noalloc reweight {prec}: grid {scene.nx}x{scene.ny}x{scene.nz}, {n} paths, seed {seed}")
        (mr, ess), got = _case(torch, api, P, ctx, scene, n, seed)
        say(f"  reweight ({mr:.15g}, {ess:.15g}) noalloc ({got[0]:.15g}, {got[1]:.15g})")
        assert np.isfinite(got).all()
        assert abs(got[0] - mr) <= 1e-15 * abs(mr)
        assert abs(got[1] - ess) <= 1e-15 * abs(ess)
    ctx.close()


def test_reweight_noalloc_rejects_grids_beyond_its_scratch():
    import torch
    from paper_2110_00085_amd import api, prt as P
    ctx = api.Context(0, P.PRT_ALL_FP64)
    scene = inputs.homogeneous((160, 160, 160), voxel_km=0.01, beta=1.0, max_order=2)  # 32.8 MB FP64 field
    beta = torch.as_tensor(scene.beta_cloud).cuda()
    st = api.PathStore.sample(ctx, scene, beta, 7, 1000)
    stats = torch.zeros(2, dtype=torch.float64, device="cuda")
    say("noalloc reweight: 160^3 FP64 field beyond the scratch -> capacity error")
    with pytest.raises(P.PrtError) as e:
        P.prt_reweight_noalloc(ctx.handle, P.make_scene(scene, beta), st.handle, stats)
    assert e.value.code == P.PRT_E_CAPACITY
    st.close()
    ctx.close()
