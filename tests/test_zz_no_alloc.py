"""The frozen-policy sweep for callers that cannot allocate
(dpo_policy_eval_sweep_static, scratch in a static device array) against the
ordinary entry point (dpo_policy_eval_sweep), through the C ABI: two calls in
a row on different problems, the second smaller, each equal bit for bit in
value and residual; an empty free set; the size limit refused."""
import numpy as np
import pytest
import torch

from paper_2407_14675_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dpo():
    from paper_2407_14675_amd import dpo as mod
    mod.load()
    return mod


def _case(dpo, p, seed):
    ctx = dpo.Context(p)
    rng = np.random.default_rng(seed)
    n = p["n"]
    shape = (n[3], n[2], n[1], n[0])
    V = torch.from_numpy(inputs.random_value(p, seed=seed, frac_M=0.1).astype(np.float32)).cuda()
    ang = torch.from_numpy(rng.uniform(-np.pi, np.pi, size=shape).astype(np.float32)).cuda()
    thr = torch.from_numpy(rng.integers(0, 2, size=shape).astype(np.uint8)).cuda()
    return ctx, V, ang, thr


def _both(dpo, ctx, V, ang, thr):
    out_a, out_b = torch.full_like(V, -1.0), torch.full_like(V, -1.0)
    ra = torch.full((5,), -7.0, dtype=torch.float64, device="cuda")
    rb = torch.full((5,), -7.0, dtype=torch.float64, device="cuda")
    ctx.policy_eval_sweep(V, out_a, ang, thr, ra)
    ctx.policy_eval_sweep_static(V, out_b, ang, thr, rb)
    torch.cuda.synchronize()
    return out_a.cpu().numpy(), out_b.cpu().numpy(), ra.cpu().numpy(), rb.cpu().numpy()


def test_static_scratch_sweep_matches_the_allocating_one(dpo):
    print("static-scratch evaluation sweep", flush=True)
    # first a large grid (many workgroup partials, two-stage reduction), then a
    # smaller one: the second call's partials overwrite only part of the array
    for p, seed in ((inputs.with_grid(inputs.PI48, (48, 48, 48, 48)), 3), (inputs.with_grid(inputs.VI12, (9, 7, 6, 5)), 4)):
        ctx, V, ang, thr = _case(dpo, p, seed)
        a, b, ra, rb = _both(dpo, ctx, V, ang, thr)
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(ra, rb)
        assert ra[0] > 0 and np.isfinite(ra).all()
        # without a residual only the values are written
        c = torch.full_like(V, -1.0)
        ctx.policy_eval_sweep_static(V, c, ang, thr)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(c.cpu().numpy(), a)
        print("  grid", p["n"], "resid", ra[:3], flush=True)


def test_static_scratch_sweep_edges(dpo):
    print("static-scratch edges", flush=True)
    # every node fixed: the residual is written as zeros by a kernel
    p = inputs.with_grid(inputs.VI12, (4, 4, 4, 4))
    mask = torch.zeros((4, 4, 4, 4), dtype=torch.uint8, device="cuda")
    ctx = dpo.Context(p, mask=mask)
    assert ctx.n_free == 0
    V = ctx.init_value()
    ang, thr = ctx.empty_policy()
    out = V.clone()
    r = torch.full((5,), -7.0, dtype=torch.float64, device="cuda")
    ctx.policy_eval_sweep_static(V, out, ang, thr, r)
    torch.cuda.synchronize()
    assert np.all(r.cpu().numpy() == 0.0)
    assert torch.equal(out, V)
    # refused arguments
    with pytest.raises(dpo.DpoError):
        ctx.policy_eval_sweep_static(V, V, ang, thr)
    # beyond the static scratch: 256^3 x 5 = 83.9M free nodes (full-size
    # buffers, so that nothing could read out of bounds even if the host
    # check did not refuse the call)
    big = inputs.with_grid(inputs.VI12, (256, 256, 256, 5))
    cb = dpo.Context(big)
    assert cb.n_free > 67108864
    Vb = cb.init_value()
    ab, tb = cb.empty_policy()
    with pytest.raises(dpo.DpoError) as e:
        cb.policy_eval_sweep_static(Vb, Vb.clone(), ab, tb)
    assert e.value.code == dpo.DPO_EINVAL and "67,108,864" in str(e.value)
    del Vb, ab, tb
    cb.close()
