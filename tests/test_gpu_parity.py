"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs and, for render/grad/reweight, on identical stored paths
drawn by the oracle and imported into the library.

Tolerances: FP32 traversal mode -- images 1e-5, gradients 1e-4 relative (L2),
correction-factor statistics 1e-5; all-FP64 mode -- 1e-9 (only the
summation order of the FP64 atomics and libm ulps differ)."""
import dataclasses

import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

TOL = {"fp32": {"img": 1e-5, "grad": 1e-4, "rw": 1e-5}, "fp64": {"img": 1e-9, "grad": 1e-9, "rw": 1e-10}}


def say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2110_00085_amd import api, prt
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    prt.lib()  # fails loudly when the HIP library is missing
    return torch, prt, api


def _prec(P, name):
    return P.PRT_ALL_FP64 if name == "fp64" else P.PRT_TRAVERSAL_FP32


def _dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float32)).cuda()


def _rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _close(a, ref, tol, what=""):
    """Relative L2 error within tol, and every element within tol of the
    largest reference magnitude: max_i |a_i - ref_i| <= tol * max|ref|.  Also
    prints the largest per-element relative error with the denominator
    floored at 1e-6 max|ref|.  Returns the L2 error."""
    a, ref = np.asarray(a, float), np.asarray(ref, float)
    scale = float(np.abs(ref).max())
    assert scale > 0, what
    l2 = _rel(a, ref)
    emax = float(np.abs(a - ref).max()) / scale
    pix = float((np.abs(a - ref) / np.maximum(np.abs(ref), 1e-6 * scale)).max())
    say(f"  {what}: L2 {l2:.2e}, max element {emax:.2e} of max|ref|, floored per-element {pix:.2e}")
    assert l2 <= tol, (what, l2)
    assert emax <= tol, (what, emax)
    return l2


def _morton_cells(dims, off, vox, B):
    """Spatial tie-break key of the library's store order (a layout choice of
    the library, not of the method): Morton code of the coarse cell (8 per
    axis) holding each path's first vertex after the source (its first
    scatter, or its entry point when it has none)."""
    nx, ny, nz = dims
    off, B = np.asarray(off), np.asarray(B)
    v = np.asarray(vox, np.int64)[off[:-1] + (B > 0)]
    c = [(v % nx) * 8 // nx, (v // nx) % ny * 8 // ny, v // (nx * ny) * 8 // nz]
    m = np.zeros_like(v)
    for k in range(3):
        for a in range(3):
            m |= ((c[a] >> k) & 1) << (3 * k + a)
    return m


def _check_sort(perm, scene, off, vox, B):
    """The store order is a stable sort by size B (Alg. 2 'Sort', Sec. 5.3):
    a permutation of all ids whose sizes never decrease, equal to the
    oracle's stable sort by B wherever sizes differ; within a size the
    library orders paths by their spatial cell, then by id."""
    n = len(B)
    assert np.array_equal(np.sort(perm), np.arange(n))
    assert (np.diff(B[perm]) >= 0).all()
    ref = oracle.sort_permutation(B)
    assert np.array_equal(B[perm], B[ref])
    cells = _morton_cells((scene.nx, scene.ny, scene.nz), off, vox, B)
    assert np.array_equal(perm, np.lexsort((np.arange(n), cells, B)))


def _perturbed(scene, seed=5, amp=0.15):
    rng = np.random.default_rng(seed)
    return (scene.beta_cloud * (1 + amp * rng.uniform(-1, 1, scene.beta_cloud.shape))).astype(np.float32)


def _store(api, ctx, torch, scene, paths):
    return api.PathStore.from_host(ctx, scene, _dev(torch, scene.beta_cloud), paths.off, paths.xyz, paths.vox,
                                   paths.B, paths.beta_ref, paths.seed)


def _workload(name):
    if name == "cloud8":
        s = inputs.cloud8()
        return s, inputs.cloud8_cameras(s), 10_000, 1001
    if name == "cloud32mid":
        s = inputs.cloud32()
        return s, inputs.cloud32_cameras(s), (1 << 15) + 37, 1002
    if name == "slabs40":
        # 40 x 40 x 24 grid: the gradient tally runs in three z slabs of
        # 10, 10 and 4 layers (FP64 LDS, 12.8 KB per layer), one walk launch
        # per slab
        s = inputs.random_field((40, 40, 24), voxel_km=0.02, lo=0.0, hi=30.0, seed=40, albedo_cloud=0.99,
                                g=0.85, max_order=12)
        return s, inputs.arc_cameras(s, [-50.0, -20.0, 0.0, 25.0, 55.0], 32, 32), 20_011, 1040
    if name == "wide96":
        # 96 x 96 x 12 grid: one 72 KB z layer per slab would need 12 slabs, so
        # the tape-driven gradient bins its walks into 7 slabs of 14 y layers
        # (the last 12) and the recomputing one falls back to FP64 atomics on
        # the output
        s = inputs.random_field((96, 96, 12), voxel_km=0.02, lo=0.0, hi=25.0, seed=96, albedo_cloud=0.99,
                                g=0.85, max_order=10)
        return s, inputs.arc_cameras(s, [-40.0, 0.0, 40.0], 24, 24), 6_007, 1096
    if name == "sparse64":
        # 64 x 64 x 32 grid (512 KB, walked in global memory) holding four
        # cloud blobs in clear air: the render's connection walks cross the
        # cloud-free bricks of 8^3 voxels in one step each
        rng = np.random.default_rng(64)
        nx, ny, nz = 64, 64, 32
        z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
        inside = np.zeros((nz, ny, nx), bool)
        for _ in range(4):
            cx, cy, cz, r = rng.uniform(12, 52), rng.uniform(12, 52), rng.uniform(8, 24), rng.uniform(4, 9)
            inside |= ((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2) <= r * r
        beta = np.where(inside, rng.lognormal(3.0, 0.6, (nz, ny, nx)), 0.0).astype(np.float32)
        s = inputs.Scene(nx, ny, nz, 0.02, beta, albedo_cloud=0.99, g=0.85, max_order=12)
        return s, inputs.arc_cameras(s, [-45.0, 0.0, 30.0], 32, 32), 20_003, 1064
    if name == "ragged_z":
        # 64 x 48 x 13 grid (160 KB in FP32: sampled and rendered from the
        # z-tiled copy in global memory; 13 layers: the copy ends in a partial
        # tile of one layer) with the sun off the vertical so that free
        # flights and connections cross tile boundaries in both z directions
        s = inputs.random_field((64, 48, 13), voxel_km=0.02, lo=0.0, hi=35.0, seed=13, albedo_cloud=0.99, g=0.85,
                                max_order=10)
        s = dataclasses.replace(s, sun_zenith_deg=35.0, sun_azimuth_deg=20.0)
        return s, inputs.arc_cameras(s, [-50.0, -10.0, 35.0], 24, 20), 12_007, 1013
    if name == "manycams":
        # 20 cameras of 48 x 48: the FP32 image partials (184 KB) exceed the LDS,
        # so renders of fewer orders (no tape) fall back to FP64 atomics on the
        # output images; the all-orders render forms them from the tape
        s = inputs.cloud8()
        return s, inputs.arc_cameras(s, np.linspace(-60.0, 60.0, 20), 48, 48), 10_000, 1001
    if name == "incam":
        # one camera inside the grid box: its connections end at the camera,
        # not at the box boundary
        s = inputs.cloud8()
        outside = inputs.arc_cameras(s, [-30.0, 30.0], 16, 16)
        inside = inputs.cameras_at([[0.33, 0.07, 0.36]], [[0.2, 0.2, 0.2]], 16, 16, 6.0)
        cams = inputs.Cameras(3, 16, 16, np.concatenate([outside.pos, inside.pos]),
                              np.concatenate([outside.rot, inside.rot]), np.concatenate([outside.f_px, inside.f_px]))
        return s, cams, 10_000, 1003
    raise KeyError(name)


# ---------------------------------------------------------------- sampling

@pytest.mark.parametrize("name", ["cloud8", "ragged_z"])
def test_sample_fp64_matches_oracle(env, name):
    """All-FP64 draws reproduce the oracle's paths: on cloud8 from the grid in
    LDS, on ragged_z from the z-tiled copy in global memory."""
    torch, P, api = env
    scene, _, n, seed = _workload(name)
    say(f"sample fp64 {name} n={n}")
    ctx = api.Context(0, P.PRT_ALL_FP64)
    st = api.PathStore.sample(ctx, scene, _dev(torch, scene.beta_cloud), seed, n)
    off, xyz, vox, B, br = st.export()
    ref = oracle.sample(scene, seed, n)
    assert np.array_equal(br, scene.beta_cloud)
    same = B == ref.B
    assert same.mean() >= 0.9995, same.mean()
    for i in np.nonzero(same)[0][::7]:
        a, b = xyz[off[i]:off[i + 1]], ref.xyz[ref.off[i]:ref.off[i + 1]]
        assert a.shape == b.shape
        assert np.abs(a.astype(float) - b).max() <= 2e-6 * max(scene.nx, scene.ny, scene.nz), i
        assert np.array_equal(vox[off[i]:off[i + 1]], ref.vox[ref.off[i]:ref.off[i + 1]])
    _check_sort(P.prt_paths_permutation(ctx.handle, st.handle), scene, off, vox, B)


def test_resample_reuses_store(env):
    """prt_resample refills a store (growing and shrinking it) with exactly the
    paths prt_sample draws for the same seed and size."""
    torch, P, api = env
    say("resample grow/shrink")
    ctx = api.Context(0, P.PRT_ALL_FP64)
    s8 = inputs.cloud8()
    b8 = _dev(torch, s8.beta_cloud)
    st = api.PathStore.sample(ctx, s8, b8, 1001, 500)
    s32 = inputs.cloud32()
    b32 = _dev(torch, s32.beta_cloud)
    for sc, bd, seed, n in ((s8, b8, 7, 20_000), (s32, b32, 9, 3_000), (s8, b8, 1001, 10_000)):
        st.resample(sc, bd, seed, n)
        ref = api.PathStore.sample(ctx, sc, bd, seed, n)
        got, exp = st.export(), ref.export()
        for x, y in zip(got, exp):
            assert np.array_equal(x, y)
        assert st.info().n_paths == n and st.info().nx == sc.nx


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_two_pass_resample_equals_one_pass(env, prec):
    """A resample too large for the one-pass temporary draws every path twice
    (sizes first, then vertices straight into the store): the store it builds
    equals the one-pass store bit for bit, for a new store and a refill."""
    torch, P, api = env
    say(f"two-pass resample {prec}")
    for name in ("cloud8", "cloud32mid"):
        scene, _, n, seed = _workload(name)
        bd = _dev(torch, scene.beta_cloud)
        one = api.Context(0, _prec(P, prec))
        two = api.Context(0, _prec(P, prec))
        P.prt_set_sample_scratch_limit(two.handle, 0)
        a = api.PathStore.sample(one, scene, bd, seed, n)
        b = api.PathStore.sample(two, scene, bd, seed, n)
        for x, y in zip(a.export(), b.export()):
            assert np.array_equal(x, y), name
        assert np.array_equal(P.prt_paths_permutation(one.handle, a.handle),
                              P.prt_paths_permutation(two.handle, b.handle))
        b.resample(scene, bd, seed + 1, n // 2)
        a.resample(scene, bd, seed + 1, n // 2)
        for x, y in zip(a.export(), b.export()):
            assert np.array_equal(x, y), name


def _sample_launches(P, ctx):
    return P.prt_kernel_times(ctx.handle, reset=True)["sample"][1]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_compact_draw_equals_one_pass(env, prec):
    """With a temporary limit just under whole rows, a draw writes short rows
    plus chains of overflow segments in one sampler launch; the store equals
    the one-pass store bit for bit.  Where the pool runs out (a new store of
    long paths, or a refill sized from a draw in a field a thousand times
    thinner) the draw finishes with the second pass of the two-pass draw (two
    launches) and still gives the same store."""
    torch, P, api = env
    say(f"compact draw {prec}")
    thick = inputs.random_field((24, 24, 24), voxel_km=0.02, lo=20.0, hi=80.0, seed=24, albedo_cloud=0.99, g=0.85,
                                max_order=40)
    cases = [_workload("cloud8")[0::2] + (1,), _workload("cloud32mid")[0::2] + (1,),
             # 97% of the paths scatter, 15.5 times on average: six segments
             # for the longest, more than a new store's pool holds
             (thick, 20_000, 2)]
    for scene, n, first in cases:
        seed = 1001
        bd = _dev(torch, scene.beta_cloud)
        one = api.Context(0, _prec(P, prec))
        cmp_ = api.Context(0, _prec(P, prec))
        P.prt_set_sample_scratch_limit(cmp_.handle, n * (scene.max_order + 2) * 16 - 1)
        P.prt_enable_timing(cmp_.handle, True)
        a = api.PathStore.sample(one, scene, bd, seed, n)
        b = api.PathStore.sample(cmp_, scene, bd, seed, n)
        assert _sample_launches(P, cmp_) == first, scene.max_order
        for x, y in zip(a.export(), b.export()):
            assert np.array_equal(x, y)
        assert np.array_equal(P.prt_paths_permutation(one.handle, a.handle),
                              P.prt_paths_permutation(cmp_.handle, b.handle))
        # a larger refill, its pool sized from this store's draw
        a.resample(scene, bd, seed + 1, n + 5)
        b.resample(scene, bd, seed + 1, n + 5)
        assert _sample_launches(P, cmp_) == 1, scene.max_order
        for x, y in zip(a.export(), b.export()):
            assert np.array_equal(x, y)
        if scene.max_order == 10:
            # about 35% of cloud8's paths scatter
            thin = _dev(torch, scene.beta_cloud * 1e-3)
            a.resample(scene, thin, seed + 2, n)
            b.resample(scene, thin, seed + 2, n)
            _sample_launches(P, cmp_)
            a.resample(scene, bd, seed + 3, n)
            b.resample(scene, bd, seed + 3, n)
            assert _sample_launches(P, cmp_) == 2
            for x, y in zip(a.export(), b.export()):
                assert np.array_equal(x, y)


@pytest.mark.parametrize("name", ["cloud8", "cloud32mid", "ragged_z"])
def test_sample_fp32_close_to_oracle(env, name):
    torch, P, api = env
    scene, _, n, seed = _workload(name)
    say(f"sample fp32 {name} n={n}")
    ctx = api.Context(0, P.PRT_TRAVERSAL_FP32)
    st = api.PathStore.sample(ctx, scene, _dev(torch, scene.beta_cloud), seed, n)
    off, xyz, vox, B, _ = st.export()
    ref = oracle.sample(scene, seed, n)
    same = B == ref.B
    assert same.mean() >= 0.995, same.mean()
    dev = []
    for i in np.nonzero(same & (B > 0))[0][:3000]:
        a, b = xyz[off[i]:off[i + 1]].astype(float), ref.xyz[ref.off[i]:ref.off[i + 1]].astype(float)
        dev.append(np.abs(a - b).max())
    assert np.median(dev) < 1e-4, np.median(dev)
    _check_sort(P.prt_paths_permutation(ctx.handle, st.handle), scene, off, vox, B)


def test_sort_over_many_tiles(env):
    """The store order over many sort tiles with a ragged tail: 300 001 paths
    of cloud32 (74 tiles of 4096 keys; most paths leave without scattering,
    so a few cells hold most keys) are in the exact stable order by (B, cell,
    id), drawn and imported again in id order."""
    torch, P, api = env
    scene, n, seed = inputs.cloud32(), 300_001, 1234
    say(f"sort over many tiles: cloud32 n={n}")
    ctx = api.Context(0, P.PRT_TRAVERSAL_FP32)
    bt = _dev(torch, scene.beta_cloud)
    st = api.PathStore.sample(ctx, scene, bt, seed, n)
    off, xyz, vox, B, br = st.export()
    perm = P.prt_paths_permutation(ctx.handle, st.handle)
    _check_sort(perm, scene, off, vox, B)
    imp = api.PathStore.from_host(ctx, scene, bt, off, xyz, vox, B, br, seed)
    assert np.array_equal(P.prt_paths_permutation(ctx.handle, imp.handle), perm)


# ---------------------------------------------- render / grad / reweight

@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["cloud8", "cloud32mid", "slabs40", "wide96", "sparse64", "ragged_z", "manycams",
                                  "incam"])
def test_render_grad_reweight_match_oracle(env, prec, name):
    torch, P, api = env
    scene, cams, n, seed = _workload(name)
    say(f"render/grad/reweight {prec} {name} n={n}")
    paths = oracle.sample(scene, seed, n)
    beta_t = _perturbed(scene)
    ctx = api.Context(0, _prec(P, prec))
    st = _store(api, ctx, torch, scene, paths)
    ch = P.CamerasHost(cams)
    bt = _dev(torch, beta_t)
    tol = TOL[prec]
    for br in (scene.max_order, 1, 3):
        img = api.render(ctx, scene, bt, ch, st, br).cpu().numpy()
        ref = oracle.render(scene, cams, paths, beta_t=beta_t, max_order_render=br)
        _close(img, ref, tol["img"], f"images, orders <= {br}")
    rng = np.random.default_rng(3)
    res = rng.standard_normal(ref.shape) * np.abs(ref).mean()
    gref = oracle.grad(scene, cams, paths, res, beta_t=beta_t)
    assert np.abs(gref).max() > 0
    res_d = torch.as_tensor(res).cuda()
    # grad right after a render of all orders (reuses the render's transmittances)
    img = api.render(ctx, scene, bt, ch, st).cpu().numpy()
    _close(img, oracle.render(scene, cams, paths, beta_t=beta_t), tol["img"], "images, all orders")
    g = api.grad(ctx, scene, bt, ch, st, res_d).cpu().numpy()
    _close(g, gref, tol["grad"], "gradient after a full render")
    # grad after a partial-order render recomputes everything
    api.render(ctx, scene, bt, ch, st, 2)
    g = api.grad(ctx, scene, bt, ch, st, res_d).cpu().numpy()
    _close(g, gref, tol["grad"], "gradient recomputed")
    # grad at a field other than the last render's recomputes everything
    beta_u = _perturbed(scene, seed=11, amp=0.2)
    api.render(ctx, scene, bt, ch, st)
    g = api.grad(ctx, scene, _dev(torch, beta_u), ch, st, res_d).cpu().numpy()
    gref_u = oracle.grad(scene, cams, paths, res, beta_t=beta_u)
    _close(g, gref_u, tol["grad"], "gradient at another field")
    mr, ess = P.prt_reweight(ctx.handle, P.make_scene(scene, bt), st.handle)
    mr_ref, ess_ref = oracle.reweight(scene, paths, beta_t=beta_t)
    assert abs(mr - mr_ref) <= tol["rw"] * abs(mr_ref), (mr, mr_ref)
    assert abs(ess - ess_ref) <= tol["rw"] * abs(ess_ref), (ess, ess_ref)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["cloud8", "cloud32mid", "incam"])
def test_thread_per_path_kernels_match_oracle(env, prec, name):
    """The path-sorting ablation's thread-per-path render and gradient (Sec.
    5.3) in both path orders, against the oracle on the same stored paths."""
    torch, P, api = env
    scene, cams, n, seed = _workload(name)
    say(f"thread-per-path render/grad {prec} {name} n={n}")
    paths = oracle.sample(scene, seed, n)
    beta_t = _perturbed(scene)
    ctx = api.Context(0, _prec(P, prec))
    st = _store(api, ctx, torch, scene, paths)
    ch = P.CamerasHost(cams)
    bt = _dev(torch, beta_t)
    sc = P.make_scene(scene, bt)
    tol = TOL[prec]
    ref = oracle.render(scene, cams, paths, beta_t=beta_t)
    res = np.random.default_rng(3).standard_normal(ref.shape) * np.abs(ref).mean()
    gref = oracle.grad(scene, cams, paths, res, beta_t=beta_t)
    res_d = torch.as_tensor(res).cuda()
    img = torch.empty(ch.image_shape, dtype=torch.float64, device="cuda")
    g = torch.empty((scene.nz, scene.ny, scene.nx), dtype=torch.float64, device="cuda")
    for order in (P.PRT_ORDER_BY_SIZE, P.PRT_ORDER_BY_ID):
        for rep in range(2):  # the second call reuses the per-path copy
            P.prt_tpp_render(ctx.handle, sc, ch, st.handle, order, img)
            _close(img.cpu().numpy(), ref, tol["img"], f"thread-per-path images, order {order}, call {rep}")
            P.prt_tpp_grad(ctx.handle, sc, ch, st.handle, order, res_d, g)
            _close(g.cpu().numpy(), gref, tol["grad"], f"thread-per-path gradient, order {order}, call {rep}")
    with pytest.raises(P.PrtError) as e:
        P.prt_tpp_render(ctx.handle, sc, ch, st.handle, 2, img)
    assert e.value.code == P.PRT_E_INVALID


def test_counters_match_oracle(env):
    torch, P, api = env
    scene, cams, n, seed = _workload("cloud8")
    say("counters fp64 cloud8")
    paths = oracle.sample(scene, seed, n)
    ctx = api.Context(0, P.PRT_ALL_FP64)
    st = _store(api, ctx, torch, scene, paths)
    P.prt_counters(ctx.handle, reset=True)
    api.render(ctx, scene, _dev(torch, scene.beta_cloud), P.CamerasHost(cams), st)
    c = P.prt_counters(ctx.handle, reset=True)
    _, cref = oracle.render(scene, cams, paths, return_counters=True)
    assert c["local_estimates"] == cref[1]
    assert abs(c["voxel_segments"] - cref[0]) <= 1e-4 * cref[0], (c, cref)
    assert c["paths"] == n


def test_full_size_cloud32(env):
    """The benchmark workload (32^3, 9 x 64^2 cameras, 2^22 paths, 20 orders)
    in the launch configuration the bench times (FP32 traversal)."""
    torch, P, api = env
    scene, cams = inputs.cloud32(), None
    cams = inputs.cloud32_cameras(scene)
    n, seed = 1 << 22, 1002
    say(f"full size cloud32 n={n}: oracle sampling")
    paths = oracle.sample(scene, seed, n)
    beta_t = _perturbed(scene, seed=7, amp=0.1)
    ctx = api.Context(0, P.PRT_TRAVERSAL_FP32)
    st = _store(api, ctx, torch, scene, paths)
    ch = P.CamerasHost(cams)
    bt = _dev(torch, beta_t)
    say("full size: gpu render")
    img = api.render(ctx, scene, bt, ch, st).cpu().numpy()
    say("full size: oracle render")
    ref = oracle.render(scene, cams, paths, beta_t=beta_t)
    _close(img, ref, TOL["fp32"]["img"], "full size images")
    res = np.random.default_rng(4).standard_normal(ref.shape) * np.abs(ref).mean()
    say("full size: gpu grad")
    g = api.grad(ctx, scene, bt, ch, st, torch.as_tensor(res).cuda()).cpu().numpy()
    say("full size: oracle grad")
    gref = oracle.grad(scene, cams, paths, res, beta_t=beta_t)
    _close(g, gref, TOL["fp32"]["grad"], "full size gradient")
    mr, ess = P.prt_reweight(ctx.handle, P.make_scene(scene, bt), st.handle)
    mr_ref, ess_ref = oracle.reweight(scene, paths, beta_t=beta_t)
    assert abs(mr - mr_ref) <= 1e-5 * mr_ref and abs(ess - ess_ref) <= 1e-5 * ess_ref


@pytest.mark.parametrize("name", ["plume64", "field128"])
def test_full_size_large_workloads(env, name):
    """The 64^3 plume (9 x 128^2 cameras, 2^26 paths, 20 orders) and the
    128x128x64 cloud field (20 x 256^2 cameras, 2^28 paths, 30 orders) at
    full size in FP32 traversal (the oracle cannot render them whole):
    sampled paths of 2000 random ids against the oracle's; render, gradient
    and r sums of the full store against a split of the same paths into a
    store A (the first 50 000 ids) and a store B (the rest), each rendered on
    its own; and store A against the oracle."""
    torch, P, api = env
    if name == "plume64":
        scene = inputs.plume64()
        cams, n = inputs.plume64_cameras(scene), 1 << 26
    else:
        scene = inputs.field128()
        cams, n = inputs.field128_cameras(scene), 1 << 28
    seed, n_a = 1004, 50_000
    ch = P.CamerasHost(cams)
    ctx = api.Context(0, P.PRT_TRAVERSAL_FP32)
    say(f"full size {name} n={n}: sample")
    st = api.PathStore.sample(ctx, scene, _dev(torch, scene.beta_cloud), seed, n)
    beta_t = _perturbed(scene, seed=9, amp=0.1)
    bt = _dev(torch, beta_t)
    say(f"full size {name}: render, grad, reweight")
    img = api.render(ctx, scene, bt, ch, st).cpu().numpy()
    res = np.random.default_rng(5).standard_normal(img.shape) * np.abs(img).mean()
    res_d = torch.as_tensor(res).cuda()
    g = api.grad(ctx, scene, bt, ch, st, res_d).cpu().numpy()
    mr, ess = P.prt_reweight(ctx.handle, P.make_scene(scene, bt), st.handle)
    assert np.isfinite(img).all() and img.min() >= 0.0 and np.abs(img).max() > 0
    assert np.isfinite(g).all() and np.abs(g).max() > 0
    say(f"full size {name}: export")
    off, xyz, vox, B, br = st.export()
    st.close()
    ctx.close()
    # sampled paths, one by one
    ids = np.sort(np.random.default_rng(6).choice(n, 2000, replace=False))
    say(f"full size {name}: oracle sampling of {len(ids)} ids")
    ref = oracle.sample(scene, seed, ids=ids, n_total=n)
    same = B[ids] == ref.B
    assert same.mean() >= 0.995, same.mean()
    dev = [np.abs(xyz[off[i]:off[i + 1]].astype(float) - ref.xyz[ref.off[k]:ref.off[k + 1]]).max()
           for k, i in enumerate(ids) if same[k] and B[i] > 0]
    assert np.median(dev) < 1e-4, np.median(dev)
    # the same paths split into two stores
    ctx = api.Context(0, P.PRT_TRAVERSAL_FP32)
    e = int(off[n_a])
    parts = {"A": (off[:n_a + 1], xyz[:e], vox[:e], B[:n_a]),
             "B": (off[n_a:] - off[n_a], xyz[e:], vox[e:], B[n_a:])}
    out = {}
    for k, (o, x, v, b) in parts.items():
        say(f"full size {name}: store {k} ({len(b)} paths)")
        sk = api.PathStore.from_host(ctx, scene, _dev(torch, scene.beta_cloud), o, x, v, b, br, seed)
        out[k] = (api.render(ctx, scene, bt, ch, sk).cpu().numpy(), api.grad(ctx, scene, bt, ch, sk, res_d).cpu().numpy(),
                  P.prt_reweight(ctx.handle, P.make_scene(scene, bt), sk.handle), len(b))
        if k == "A":
            paths_a = oracle.Paths(o.copy(), x.astype(np.float32), v.copy(), b.astype(B.dtype), n_a, seed, br)
        sk.close()
    ctx.close()
    (img_a, g_a, (mr_a, ess_a), na), (img_b, g_b, (mr_b, ess_b), nb) = out["A"], out["B"]
    # images and r sums are FP64 sums of identical terms; the gradient weights
    # are stored in FP32 after the 1/N scaling, so they round differently
    _close(na * img_a + nb * img_b, n * img, 1e-10, "split-store images")
    _close(na * g_a + nb * g_b, n * g, 1e-6, "split-store gradient")
    assert abs(na * mr_a + nb * mr_b - n * mr) <= 1e-10 * n * mr
    r2 = lambda m, s_, k: (m * k) ** 2 / s_
    assert abs(r2(mr_a, ess_a, na) + r2(mr_b, ess_b, nb) - r2(mr, ess, n)) <= 1e-9 * r2(mr, ess, n)
    say(f"full size {name}: oracle on store A")
    ref_img = oracle.render(scene, cams, paths_a, beta_t=beta_t)
    _close(img_a, ref_img, TOL["fp32"]["img"], "store A images")
    ref_g = oracle.grad(scene, cams, paths_a, res, beta_t=beta_t)
    _close(g_a, ref_g, TOL["fp32"]["grad"], "store A gradient")
    mr_ref, ess_ref = oracle.reweight(scene, paths_a, beta_t=beta_t)
    assert abs(mr_a - mr_ref) <= 1e-5 * mr_ref and abs(ess_a - ess_ref) <= 1e-5 * ess_ref


def test_finite_differences_full_size_cloud32(env):
    """The differentiable step's check at its full size: the 32^3 field with
    2^22 stored paths in all-FP64 mode, L2 loss against images of a second
    seeded field rendered from fresh paths; prt_grad against differences of
    the loss at fixed paths on 64 random voxels (seed 33): central
    differences, or a one-sided three-point difference where beta < 2h."""
    torch, P, api = env
    scene = inputs.cloud32()
    cams = inputs.cloud32_cameras(scene)
    n = 1 << 22
    ch = P.CamerasHost(cams)
    ctx = api.Context(0, P.PRT_ALL_FP64)
    say("finite differences cloud32 n=2^22 fp64: target images")
    tgt_scene = scene.with_beta(inputs.gaussian_field_cloud(32, 3))
    st_t = api.PathStore.sample(ctx, tgt_scene, _dev(torch, tgt_scene.beta_cloud), 2003, n)
    tgt = api.render(ctx, tgt_scene, _dev(torch, tgt_scene.beta_cloud), ch, st_t)
    st_t.close()
    say("finite differences: sample, render, grad")
    b0 = _dev(torch, scene.beta_cloud)
    st = api.PathStore.sample(ctx, scene, b0, 1003, n)
    img = api.render(ctx, scene, b0, ch, st)
    g = api.grad(ctx, scene, b0, ch, st, (img - tgt).contiguous()).cpu().numpy().ravel()

    def L(b):
        im = api.render(ctx, scene, b, ch, st)
        return float(0.5 * ((im - tgt) ** 2).sum())

    h = 2.0 ** -6  # beta +- h is exact in FP32 for beta < 2^17
    flat = b0.view(-1)
    voxels = np.random.default_rng(33).choice(flat.numel(), 64, replace=False)
    say("finite differences: 64 voxels")
    for v in voxels:
        def at(k):
            b = flat.clone()
            b[v] += k * h
            return L(b.view_as(b0))
        if float(flat[v]) >= 2 * h:
            fd = (at(1) - at(-1)) / (2 * h)
        else:
            fd = (-3.0 * at(0) + 4.0 * at(1) - at(2)) / (2 * h)
        assert abs(fd - g[v]) <= 1e-5 * np.abs(g).max() + 1e-4 * abs(fd), (int(v), fd, g[v])
    st.close()


# ------------------------------------------------------------- loop glue

def test_loss_and_adam_match_oracle(env):
    torch, P, api = env
    say("loss + adam")
    ctx = api.Context(0, P.PRT_TRAVERSAL_FP32)
    rng = np.random.default_rng(8)
    n = 100_003
    img, tgt = rng.standard_normal(n), rng.standard_normal(n)
    res = torch.empty(n, dtype=torch.float64, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    P.prt_loss(ctx.handle, torch.as_tensor(img).cuda(), torch.as_tensor(tgt).cuda(), res, loss)
    L, r = oracle.loss_and_residual(img, tgt)
    assert np.array_equal(res.cpu().numpy(), r)
    assert abs(loss.item() - L) <= 1e-12 * L
    beta = rng.uniform(0, 1, 5000)
    b = torch.as_tensor(beta.copy()).cuda()
    b32 = torch.empty(5000, dtype=torch.float32, device="cuda")
    m = torch.zeros(5000, dtype=torch.float64, device="cuda")
    v = torch.zeros_like(m)
    mo, vo = np.zeros(5000), np.zeros(5000)
    for t in range(1, 4):
        g = rng.standard_normal(5000)
        P.prt_adam(ctx.handle, b, b32, torch.as_tensor(g).cuda(), m, v, t, 0.1)
        beta, mo, vo = oracle.adam_step(beta, g, mo, vo, t, 0.1)
    assert np.allclose(b.cpu().numpy(), beta, rtol=1e-13, atol=1e-15)
    assert np.array_equal(b32.cpu().numpy(), beta.astype(np.float32))


# ------------------------------------------------------------ edge cases

def test_edge_cases(env):
    torch, P, api = env
    say("edge cases")
    ctx = api.Context(0, P.PRT_TRAVERSAL_FP32)
    scene, cams, _, _ = _workload("cloud8")
    ch = P.CamerasHost(cams)
    # a single path
    paths = oracle.sample(scene, 1001, 1, ids=[37])
    st = _store(api, ctx, torch, scene, paths)
    bt = _dev(torch, scene.beta_cloud)
    img = api.render(ctx, scene, bt, ch, st).cpu().numpy()
    ref1 = oracle.render(scene, cams, paths)
    if np.abs(ref1).max() > 0:
        _close(img, ref1, 1e-5, "single path images")
    else:
        assert np.abs(img).max() == 0
    # an empty medium: no path scatters, images and gradient vanish, r = 1
    empty = scene.with_beta(np.zeros_like(scene.beta_cloud))
    empty.beta_air = 0.0
    z = _dev(torch, empty.beta_cloud)
    res = torch.ones(ch.image_shape, dtype=torch.float64, device="cuda")
    # 777 paths leave a partial last batch; 768 fill whole batches, so no batch scatters
    for n0 in (777, 768):
        st0 = api.PathStore.sample(ctx, empty, z, 5, n0)
        _, _, _, B, _ = st0.export(vertices=False)
        assert (B == 0).all()
        for _ in range(2):  # the second call finds the scratch of the first
            assert np.abs(api.render(ctx, empty, z, ch, st0).cpu().numpy()).max() == 0.0
            assert np.abs(api.grad(ctx, empty, z, ch, st0, res).cpu().numpy()).max() == 0.0
        mr, ess = P.prt_reweight(ctx.handle, P.make_scene(empty, z), st0.handle)
        assert mr == 1.0 and abs(ess - n0) < 1e-9
    # one scattering order only; capped paths
    s1 = inputs.cloud8()
    s1.max_order = 1
    p1 = oracle.sample(s1, 9, 3000)
    assert (p1.B <= 1).all() and (p1.B == 1).any()
    st1 = _store(api, ctx, torch, s1, p1)
    img1 = api.render(ctx, s1, _dev(torch, s1.beta_cloud), ch, st1).cpu().numpy()
    _close(img1, oracle.render(s1, cams, p1), 1e-5, "one order")
    # paths capped at 1 and 2 orders in a field 3x as thick (most scattering
    # paths end at the cap, without an exit vertex): render, gradient on the
    # tape and reweight at a perturbed field against the oracle
    for cap in (1, 2):
        sc = inputs.cloud8()
        sc.max_order = cap
        sc = sc.with_beta(3.0 * sc.beta_cloud)
        pc = oracle.sample(sc, 19, 4000)
        assert (pc.B == cap).mean() > 0.1, (pc.B == cap).mean()
        stc = _store(api, ctx, torch, sc, pc)
        beta_c = _perturbed(sc, seed=23, amp=0.1)
        btc = _dev(torch, beta_c)
        imgc = api.render(ctx, sc, btc, ch, stc).cpu().numpy()
        refc = oracle.render(sc, cams, pc, beta_t=beta_c)
        _close(imgc, refc, TOL["fp32"]["img"], f"capped at {cap}: images")
        resc = np.random.default_rng(29).standard_normal(refc.shape) * np.abs(refc).mean()
        gc = api.grad(ctx, sc, btc, ch, stc, torch.as_tensor(resc).cuda()).cpu().numpy()
        grefc = oracle.grad(sc, cams, pc, resc, beta_t=beta_c)
        _close(gc, grefc, TOL["fp32"]["grad"], f"capped at {cap}: gradient")
        mr, ess = P.prt_reweight(ctx.handle, P.make_scene(sc, btc), stc.handle)
        mr_ref, ess_ref = oracle.reweight(sc, pc, beta_t=beta_c)
        assert abs(mr - mr_ref) <= TOL["fp32"]["rw"] * abs(mr_ref), (cap, mr, mr_ref)
        assert abs(ess - ess_ref) <= TOL["fp32"]["rw"] * abs(ess_ref), (cap, ess, ess_ref)
    # cameras that see nothing
    far = inputs.cameras_at([[100.0, 100.0, 100.0]], [[200.0, 200.0, 200.0]], 8, 8, 10.0)
    assert np.abs(api.render(ctx, s1, _dev(torch, s1.beta_cloud), P.CamerasHost(far), st1).cpu().numpy()).max() == 0.0
    # repeated renders agree up to the rounding of the FP64 tally order (the
    # tape's FP64 LDS images, or FP64 atomics), for all orders and for fewer
    paths2 = oracle.sample(scene, 1001, 10_000)
    for prec in ("fp32", "fp64"):
        c2 = api.Context(0, _prec(P, prec))
        st2 = _store(api, c2, torch, scene, paths2)
        for br in (scene.max_order, 3):
            a = api.render(c2, scene, bt, ch, st2, br).cpu().numpy()
            b = api.render(c2, scene, bt, ch, st2, br).cpu().numpy()
            assert _rel(a, b) <= 1e-13, (prec, br, _rel(a, b))
            assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max(), (prec, br)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_no_air_and_a_zeroed_voxel(env, prec):
    """beta_air = 0 and beta_t = 0 in a voxel where stored paths scatter (as
    the projection of Adam onto beta >= 0 can leave it): those paths cannot
    occur under beta_t, so their correction factor is 0, not NaN; render,
    gradient and the r statistics match the oracle."""
    torch, P, api = env
    say(f"no air, zeroed voxel, {prec}")
    scene = inputs.cloud8()
    scene.beta_air = 0.0
    cams = inputs.cloud8_cameras(scene)
    paths = oracle.sample(scene, 77, 8000)
    # the voxel holding the most scatter vertices
    sc_vox = np.concatenate([paths.vox[paths.off[i] + 1:paths.off[i] + 1 + paths.B[i]] for i in range(paths.n)])
    v0 = int(np.bincount(sc_vox).argmax())
    beta_t = _perturbed(scene, seed=31, amp=0.1).ravel()
    beta_t[v0] = 0.0
    beta_t = beta_t.reshape(scene.beta_cloud.shape)
    lr = oracle.log_r(scene, paths, beta_t=beta_t)
    assert np.isneginf(lr).sum() > 50 and not np.isnan(lr).any()
    ctx = api.Context(0, _prec(P, prec))
    st = _store(api, ctx, torch, scene, paths)
    ch = P.CamerasHost(cams)
    bt = _dev(torch, beta_t)
    tol = TOL[prec]
    img = api.render(ctx, scene, bt, ch, st).cpu().numpy()
    ref = oracle.render(scene, cams, paths, beta_t=beta_t)
    _close(img, ref, tol["img"], "images")
    res = np.random.default_rng(37).standard_normal(ref.shape) * np.abs(ref).mean()
    g = api.grad(ctx, scene, bt, ch, st, torch.as_tensor(res).cuda()).cpu().numpy()
    _close(g, oracle.grad(scene, cams, paths, res, beta_t=beta_t), tol["grad"], "gradient")
    mr, ess = P.prt_reweight(ctx.handle, P.make_scene(scene, bt), st.handle)
    mr_ref, ess_ref = oracle.reweight(scene, paths, beta_t=beta_t)
    assert np.isfinite(mr) and np.isfinite(ess)
    assert abs(mr - mr_ref) <= tol["rw"] * abs(mr_ref), (mr, mr_ref)
    assert abs(ess - ess_ref) <= tol["rw"] * abs(ess_ref), (ess, ess_ref)


def test_store_outlives_its_context(env):
    """A store destroyed after the context that built it (the order of
    finalizers at interpreter exit is arbitrary): the store's destroy must not
    touch the context.  In this process, and in a child process that exits
    normally after destroying the context first."""
    import subprocess
    import sys
    torch, P, api = env
    say("store destroyed after its context")
    scene = inputs.cloud8()
    ctx = api.Context(0, P.PRT_TRAVERSAL_FP32)
    bt = _dev(torch, scene.beta_cloud)
    st = api.PathStore.sample(ctx, scene, bt, 3, 5000)
    n = st.info().n_paths
    ctx.close()
    assert st.info().n_paths == n
    st.close()
    code = ("import sys, numpy as np, torch; sys.path.insert(0, sys.argv[1]); import inputs; "
            "from paper_2110_00085_amd import api, prt; s = inputs.cloud8(); "
            "c = api.Context(0, prt.PRT_TRAVERSAL_FP32); b = torch.as_tensor(s.beta_cloud).cuda(); "
            "st = api.PathStore.sample(c, s, b, 3, 5000); prt.prt_destroy(c.handle); c.handle = None; "
            "st.close(); print('ok', flush=True)")
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code, root], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), (r.returncode, r.stdout[-500:], r.stderr[-2000:])


def test_argument_errors(env):
    torch, P, api = env
    say("argument errors")
    ctx = api.Context(0, P.PRT_TRAVERSAL_FP32)
    scene, cams, _, _ = _workload("cloud8")
    bt = _dev(torch, scene.beta_cloud)
    st = api.PathStore.sample(ctx, scene, bt, 1, 1000)
    ch = P.CamerasHost(cams)
    img = torch.empty(ch.image_shape, dtype=torch.float64, device="cuda")
    other = inputs.random_field((4, 4, 4))
    with pytest.raises(P.PrtError) as e:
        P.prt_render(ctx.handle, P.make_scene(other, _dev(torch, other.beta_cloud)), ch, st.handle, 10, img)
    assert e.value.code == P.PRT_E_MISMATCH
    bad = inputs.cloud8()
    bad.albedo_cloud = 1.5
    with pytest.raises(P.PrtError) as e:
        P.prt_render(ctx.handle, P.make_scene(bad, bt), ch, st.handle, 10, img)
    assert e.value.code == P.PRT_E_INVALID
    many = inputs.arc_cameras(scene, np.linspace(-60, 60, 25), 4, 4)
    with pytest.raises(P.PrtError) as e:
        P.prt_render(ctx.handle, P.make_scene(scene, bt), P.CamerasHost(many), st.handle, 10, img)
    assert e.value.code == P.PRT_E_CAPACITY
    bad2 = inputs.cloud8()
    bad2.max_order = 0
    with pytest.raises(P.PrtError) as e:
        P.prt_sample(ctx.handle, P.make_scene(bad2, bt), 1, 10)
    assert e.value.code == P.PRT_E_CAPACITY


# -------------------------------------------------------------- autograd

def test_autograd_function_and_finite_differences(env):
    """RenderFn.backward equals prt_grad, and (all-FP64) matches central finite
    differences of the rendered loss at fixed paths."""
    torch, P, api = env
    say("autograd + finite differences")
    sc = inputs.random_field((4, 4, 4), voxel_km=0.1, lo=0.5, hi=8.0, seed=21, albedo_cloud=0.9, g=0.85,
                             max_order=12)
    cams = inputs.arc_cameras(sc, [-40.0, 0.0, 35.0], 8, 8)
    ctx = api.Context(0, P.PRT_ALL_FP64)
    st = api.PathStore.sample(ctx, sc, _dev(torch, sc.beta_cloud), 404, 3000)
    ch = P.CamerasHost(cams)
    beta = torch.as_tensor(_perturbed(sc, 3, 0.2).astype(np.float64)).cuda().requires_grad_(True)
    tgt = torch.as_tensor(np.random.default_rng(2).uniform(0, 1, ch.image_shape)).cuda()
    img = api.RenderFn.apply(beta, ctx, sc, ch, st)
    loss = 0.5 * ((img - tgt) ** 2).sum()
    loss.backward()
    g = beta.grad.detach().cpu().numpy()
    g2 = api.grad(ctx, sc, beta.detach().float(), ch, st, (img - tgt).detach().contiguous()).cpu().numpy()
    assert np.allclose(g, g2, rtol=1e-12, atol=1e-14 * np.abs(g).max())

    def L(b64):
        with torch.no_grad():
            im = api.render(ctx, sc, b64.float().contiguous(), ch, st)
            return float(0.5 * ((im - tgt) ** 2).sum())

    b0 = beta.detach().float().double()
    h = 2.0 ** -8
    for v in [0, 13, 27, 42, 63]:
        e = torch.zeros_like(b0).view(-1)
        e[v] = h
        e = e.view_as(b0)
        fd = (L(b0 + e) - L(b0 - e)) / (2 * h)
        assert abs(fd - g.ravel()[v]) <= 1e-5 * np.abs(g).max() + 1e-9 * abs(fd), (v, fd, g.ravel()[v])
