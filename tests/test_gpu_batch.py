"""Batched multi-problem solve (one launch per sweep for all problems,
hipGraph replays): parity with the sequential single-problem solves and with
the CPU oracle."""
import numpy as np
import pytest
import torch

from oracle.core import KIND_FREE, Oracle
from paper_2407_14675_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dpo():
    from paper_2407_14675_amd import dpo as mod
    mod.load()
    return mod


def small_batch(sides):
    """Config-3 style draws (target radius, thrust level) on small grids."""
    draws = inputs.batch_draws(len(sides), seed=3)
    return [inputs.orbit_problem((s,) * 4, target_radius=d["target_radius"], accel=d["accel"],
                                 name=f"batch_p{i}_{s}") for i, (d, s) in enumerate(zip(draws, sides))]


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def test_batch_equals_sequential_bit_for_bit(dpo):
    """Same kernels per node, so a fixed number of sweeps gives identical
    values and policies whatever the batching and workgroup size."""
    print("batch vs sequential", flush=True)
    probs = small_batch([9, 12, 7, 10, 13])
    b = dpo.Batch(probs)
    V1 = b.init_values()
    a1, t1 = b.empty_policies()
    rc, st, _ = b.solve_vi(V1, a1, t1, tol_rel=0.0, max_sweeps=24, sweeps_per_graph=8, block=128)
    assert rc == dpo.DPO_ENOCONV and all(s["sweeps"] == 24 for s in st)
    V2 = b.init_values()
    a2, t2 = b.empty_policies()
    b.solve_sequential(V2, a2, t2, tol_rel=0.0, max_sweeps=24, check_every=24)
    for p in range(len(probs)):
        np.testing.assert_array_equal(host(V1[p]), host(V2[p]))
        np.testing.assert_array_equal(host(a1[p]), host(a2[p]))
        np.testing.assert_array_equal(host(t1[p]), host(t2[p]))


def test_many_problems_stop_as_the_sequential_solves_do(dpo):
    """40 problems of 4..10 nodes per axis: the running set shrinks many
    times (each time the per-tile problem table is rebuilt), and with the
    stop test on the same sweeps (every 8) every problem stops on the same
    sweep as its sequential solve, with the same values bit for bit."""
    print("40 problems", flush=True)
    rng = np.random.default_rng(11)
    sides = [int(x) for x in rng.integers(4, 11, size=40)]
    probs = small_batch(sides)
    b = dpo.Batch(probs)
    V1 = b.init_values()
    a1, t1 = b.empty_policies()
    rc, st1, _ = b.solve_vi(V1, a1, t1, tol_rel=1e-6, max_sweeps=20000, sweeps_per_graph=8, block=64)
    assert rc == dpo.DPO_OK and all(s["converged"] for s in st1)
    V2 = b.init_values()
    a2, t2 = b.empty_policies()
    rc2, st2, _ = b.solve_sequential(V2, a2, t2, tol_rel=1e-6, max_sweeps=20000, check_every=8)
    assert rc2 == dpo.DPO_OK
    counts = [s["sweeps"] for s in st1]
    assert counts == [s["sweeps"] for s in st2]
    assert len(set(counts)) > 10  # the running set really shrinks step by step
    for p in range(len(probs)):
        np.testing.assert_array_equal(host(V1[p]), host(V2[p]))
        np.testing.assert_array_equal(host(a1[p]), host(a2[p]))


def test_batch_converges_to_oracle(dpo):
    print("batch vs oracle", flush=True)
    probs = small_batch([6, 8, 7])
    b = dpo.Batch(probs)
    Vs = b.init_values()
    angs, thrs = b.empty_policies()
    rc, st, sec = b.solve_vi(Vs, angs, thrs, tol_rel=1e-7, max_sweeps=20000, sweeps_per_graph=16, block=256)
    assert rc == dpo.DPO_OK and all(s["converged"] for s in st)
    for p, prob in enumerate(probs):
        o = Oracle(prob)
        ref = o.solve_vi(tol_abs=1e-9, max_sweeps=50000)
        assert ref["converged"]
        free = o.kind == KIND_FREE
        err = np.abs(host(Vs[p]) - ref["V"]) / np.maximum(1.0, np.abs(ref["V"]))
        assert err[free].max() <= 1e-4, (p, err.max())
        print("  problem", p, "sweeps", st[p]["sweeps"], "oracle sweeps", ref["sweeps"], flush=True)


def test_batch_problems_stop_independently(dpo):
    """A problem that converges early stops (its sweep count is smaller) while
    the others continue; stopped problems keep their converged values."""
    print("independent stop", flush=True)
    probs = small_batch([6, 11])
    probs[1] = dict(probs[1], dt=0.02)  # slower dynamics: needs more sweeps
    b = dpo.Batch(probs)
    Vs = b.init_values()
    rc, st, _ = b.solve_vi(Vs, tol_rel=1e-6, max_sweeps=40000, sweeps_per_graph=8, block=256)
    assert rc == dpo.DPO_OK
    assert st[0]["sweeps"] < st[1]["sweeps"]
    # each result equals its own single-problem solve to the stop tolerance
    for p in range(2):
        ctx = dpo.Context(probs[p])
        V = ctx.init_value()
        a, t = ctx.empty_policy()
        ctx.solve_vi(V, a, t, tol_rel=1e-6, max_sweeps=40000, check_every=1)
        err = np.abs(host(V) - host(Vs[p])) / np.maximum(1.0, np.abs(host(V)))
        assert err.max() <= 1e-4


def test_autotune_picks_a_valid_config(dpo, tmp_path):
    print("autotune", flush=True)
    from paper_2407_14675_amd import autotune
    b = dpo.Batch(small_batch([8, 10, 12]))
    cache = str(tmp_path / "cache.json")
    block, S = autotune.tune(b, cache_path=cache, replays=1)
    assert block in autotune.BLOCKS and S in autotune.SWEEPS_PER_GRAPH
    assert autotune.tune(b, cache_path=cache) == (block, S)  # served from the cache


def test_batch_rejects_bad_configs(dpo):
    b = dpo.Batch(small_batch([6, 7]))
    Vs = b.init_values()
    with pytest.raises(dpo.DpoError):
        b.solve_vi(Vs, sweeps_per_graph=7)
    with pytest.raises(dpo.DpoError):
        b.solve_vi(Vs, block=100)
