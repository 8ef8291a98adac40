"""Host logic of the Alg. 2 driver: the resampling policy (every N_r
iterations and/or when the mean correction factor drifts) and the loss
saturation rule that ends a coarse-to-fine stage."""


def test_policy_and_saturation_rules():
    from paper_2110_00085_amd.loop import Policy, saturated
    p = Policy(period=3, drift=None)
    assert [p.resample(t, 0, 1.0) for t in range(5)] == [False, False, False, True, True]
    q = Policy(period=None, drift=0.2)
    assert not q.resample(10, 0, 1.19) and q.resample(10, 0, 1.21) and q.resample(10, 0, 0.79)
    assert q.resample(1, 0, float("nan")) and not q.resample(1, 0, None)
    e = Policy(period=None, drift=None, min_ess=0.1)
    assert not e.resample(50, 0, 1.0, 0.1) and e.resample(50, 0, 1.0, 0.099) and not e.resample(50, 0, 1.0, None)
    assert not saturated([10.0, 9.0, 8.0], 3, 1e-3)
    assert saturated([10.0, 10.0, 10.0, 9.9999], 3, 1e-3)
    assert not saturated([10.0, 9.0, 8.0, 7.0], 3, 1e-3)
