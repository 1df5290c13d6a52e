"""GPU SPHENIX viscosity switch (sphx_alpha_v_update) against the oracle on
seeded inputs that cover compression and expansion, no signal velocity, no
sound speed, alpha above and below its target, over a ragged size. FP32
against FP64: within 2e-6 of the larger of the two alphas (the update is
continuous across the jump rule, so a decision the two sides take
differently at the threshold changes the result by rounding only)."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def inputs_set(n, seed):
    rng = np.random.default_rng(seed)
    f = lambda a: np.asarray(a, np.float32)
    div_old = f(rng.normal(0.0, 1.0, n))
    div_new = f(div_old + rng.normal(0.0, 1.0, n) * (rng.random(n) < 0.8))
    c = f(10.0 ** rng.uniform(-2, 1, n) * (rng.random(n) > 0.02))
    h = f(10.0 ** rng.uniform(-3, -1, n))
    vs = f(10.0 ** rng.uniform(-3, 1, n) * (rng.random(n) > 0.02))
    alpha = f(rng.uniform(0.0, 2.0, n))
    return alpha, div_old, div_new, c, h, vs


@pytest.mark.parametrize("n,dt", [(100003, 1e-3), (4097, 0.3), (1, 1e-6)])
def test_switch_matches_oracle(n, dt):
    import torch
    from paper_2305_13380_amd import sphx
    alpha, dold, dnew, c, h, vs = inputs_set(n, n)
    ctx = sphx.Context(sphx.default_params(), 0)
    t = [torch.from_numpy(a).cuda() for a in (alpha, dold, dnew, c, h, vs)]
    sphx.alpha_v_update(ctx, t[0], t[1], t[2], t[3], t[4], t[5], dt)
    torch.cuda.synchronize()
    got = t[0].cpu().numpy().astype(np.float64)
    ref = oracle.alpha_v_update(alpha, dold, dnew, c, h, vs, dt, oracle.Params())
    err = np.abs(got - ref)
    assert np.all(err <= 2e-6 * np.maximum(np.abs(got), np.abs(ref)) + 1e-12), (
        "worst %.3g" % (err / (np.abs(ref) + 1e-30)).max())
    if n > 1000:
        # every branch was exercised
        jump = ref > alpha.astype(np.float64)
        assert jump.any() and (~jump).any() and np.any(c == 0) and np.any(vs == 0)


def test_switch_empty_and_invalid():
    import torch
    from paper_2305_13380_amd import sphx
    ctx = sphx.Context(sphx.default_params(), 0)
    e = torch.empty(0, dtype=torch.float32, device="cuda:0")
    sphx.alpha_v_update(ctx, e, e, e, e, e, e, 1e-3)
    a = torch.ones(8, dtype=torch.float32, device="cuda:0")
    for dt in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(sphx.SphxError):
            sphx.alpha_v_update(ctx, a, a, a, a, a, a, dt)
    torch.cuda.synchronize()
    assert torch.all(a == 1.0)
