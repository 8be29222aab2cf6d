"""Benchmark of the semi-Lagrangian Bellman hot path on one MI355X.

Workload (the largest single-GPU configuration): the 96 x 96 x 96 x 64
planar orbit-transfer grid (56,623,104 nodes, 226.5 MB per float32 value
array), thrust acceleration 1e-3, dt = 0.02, running cost 1 + 0.1*thrust,
scan of 64 thrust angles + golden section (12 steps, 14 evaluations) + coast
per greedy step, 20 frozen-policy evaluation sweeps per policy update;
float32 values and policy, FP64 residual.  One step = one outer iteration of
modified policy iteration (greedy sweep, residual reduction and read-back,
20 evaluation sweeps), run by the library's own solver loop, from the state
value iteration to a relative residual of 1e-3 leaves (the schedule's first
phase, set-up).

Prints one JSON line: node-control evaluations per second of the timed
steps; the roofline of the dominant kernel (the evaluation sweep); the time
to a converged value function (value iteration to 1e-3, policy iteration to
1e-6, then on to the float32 floor, the accuracy that meets 1e-4 against the
oracle); network-seeded and walk-seeded against plain policy iteration on the
held-out thrust level; the CPU oracle timed on a bounded sample of the same
workload; and, as further keys, the 48^4 reduced-grid workload, the batched
solve, the paper's Example 1 and its variants.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks.  HBM3E 8 TB/s.  FP32 vector 157.3 TFLOP/s is the
# packed rate (256 CUs x 2.4 GHz x 256 flops per clock); the sweeps issue
# ordinary (unpacked) VALU instructions, one wave64 instruction per SIMD every
# four clocks: 256 x 4 x 2.4e9 / 4 = 6.14e11 wave instructions/s, 78.6
# TFLOP/s of FMA.  bench measures both ceilings on the device beside them.
HBM_PEAK_GBS = 8000.0
VALU_PEAK_TFLOPS = 157.3
VALU_UNPACKED_WAVE_INSTR_PER_S = 256 * 4 * 2.4e9 / 4

# Algorithmic HBM bytes of one frozen-policy evaluation per node: the value
# read (4), the value written (4), the stored control (4) and the node's
# index (4).  The descriptor the library streams instead of the control and
# the index is 8 bytes (cell code + the two cell coordinates, packed).
EVAL_ALGO_BYTES_PER_NODE = 16
# Greedy sweep: packed coordinates (4) + value read (4) + value, angle and
# throttle written (4 + 4 + 1) + the packed foot descriptor written (8).
GREEDY_BYTES_PER_NODE = 25
EVALS_PER_GREEDY_NODE = 1 + 64 + 2 + 12
# VALU wave instructions per wave of 64 nodes of the greedy sweep with foot
# descriptors, from the SQ_INSTS_VALU counter (profiles/k_sweep_fast_seeded_96x96x96x64.md)
GREEDY_VALU_PER_WAVE = 2208
# Gather bytes of one evaluation done naively: 16 float32 corners.
GATHER_BYTES_PER_EVAL = 64

# HBM traffic of the evaluation sweep measured with rocprofv3 counters, with
# the hash of the kernel sources it was measured on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_eval_brick_desc_96x96x96x64_traffic.json")
KERNEL_SOURCES = ["dpo_brick.hip", "dpo_kernels.hip", "dpo_device.h", "dpo_kernels.h", "dpo_search.h",
                  "dpo_api.hip"]  # the last holds the brick plan (tiles, planes per workgroup)


def kernel_source_hash():
    """Hash of the kernel sources with comments and blank space removed, so
    that only code changes invalidate a counter measurement."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2407_14675_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic():
    """Bytes per launch from the committed counter summary, or None when the
    kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except OSError:
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measure_ceilings(reps=10):
    """HBM and VALU ceilings measured on this GPU with the library's own probe
    kernels: a 16-byte streaming copy and read of 1 GiB buffers (far above the
    256 MiB last-level cache) and a plain FP32 FMA loop (eight independent
    chains per lane, no packed instructions) over 8192 workgroups of 256."""
    import torch

    from paper_2407_14675_amd import dpo

    n = 1 << 28  # floats: 1 GiB
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    sink = torch.zeros(1, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        ev0.record(stream)
        for _ in range(reps):
            fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) * 1e-3 / reps

    t_copy = timed(lambda: dpo.probe_copy(src, dst))
    t_read = timed(lambda: dpo.probe_read(src, sink))
    del src, dst
    blocks, iters = 8192, 4096
    t_fma = timed(lambda: dpo.probe_fma(blocks, iters, sink))
    fmas = blocks * 256 * iters * 8
    wave_instr = blocks * 4 * iters * 8
    return {
        "hbm_copy_GBs": 8.0 * n / t_copy / 1e9,
        "hbm_read_GBs": 4.0 * n / t_read / 1e9,
        "hbm_peak_GBs": HBM_PEAK_GBS,
        "fp32_fma_tflops": 2.0 * fmas / t_fma / 1e12,
        "valu_wave_instr_per_s": wave_instr / t_fma,
        "fp32_vector_peak_tflops_packed": VALU_PEAK_TFLOPS,
        "what": "1 GiB float4 copy (read + write bytes) and read; FP32 FMA loop, 8 chains per lane, "
                "8192 x 256 threads x 4096 iterations, plain v_fma_f32",
    }


def cpu_baseline(problem, V, seconds=12.0, seed=17):
    """The FP64 oracle on a bounded random sample of the workload's nodes: one
    greedy step (coast + 64 scan + 14 golden) and 20 frozen-policy evaluations
    per sampled node, at the value the timed steps start from, on one host
    thread."""
    import numpy as np

    from oracle.core import Oracle

    o = Oracle(problem)
    rng = np.random.default_rng(seed)
    evals_per_node = EVALS_PER_GREEDY_NODE + 20
    done_nodes = 0
    t0 = time.perf_counter()
    chunk = 2000
    while time.perf_counter() - t0 < seconds:
        nodes = np.sort(rng.choice(o.N, size=chunk, replace=False)).astype(np.int64)
        Vn, ang, thr, _ = o.bellman_nodes(V, nodes)
        for _ in range(20):
            o.q_many(V, nodes, thr, ang)
        done_nodes += chunk
    dt = time.perf_counter() - t0
    shape = "x".join(str(k) for k in problem["n"])
    return {
        "value": done_nodes * evals_per_node / dt,
        "unit": "node-control evals/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{done_nodes} random nodes of the {shape} grid x (1 coast + 64 scan + 14 golden + 20 policy "
                  f"evals), at the value the timed steps start from, FP64, single thread, {dt:.1f} s",
    }


def bench_batched(max_sweeps=20000, tol=1e-6, side_scale=1.0):
    """16 transfer problems (target radius, thrust level and grid side drawn
    with seed 3; sides 24..64, times side_scale) solved by value iteration,
    batched (one launch per sweep, hipGraph replays, autotuned) and one after
    another."""
    import torch

    from paper_2407_14675_amd import autotune, dpo, inputs

    probs = inputs.batch_problems(side_scale=side_scale)
    b = dpo.Batch(probs)
    t0 = time.perf_counter()
    block, S = autotune.tune(b, replays=2)
    tune_s = time.perf_counter() - t0
    Vs = b.init_values()
    angs, thrs = b.empty_policies()
    torch.cuda.synchronize()
    rc, st, sec = b.solve_vi(Vs, angs, thrs, tol_rel=tol, max_sweeps=max_sweeps, sweeps_per_graph=S, block=block)
    V2 = b.init_values()
    a2, t2 = b.empty_policies()
    torch.cuda.synchronize()
    rc2, st2, sec2 = b.solve_sequential(V2, a2, t2, tol_rel=tol, max_sweeps=max_sweeps, check_every=16)
    evals = sum(s["sweeps"] * nf * 17 for s, nf in zip(st, b.n_free))
    diff = max(float(((x - y).abs() / y.abs().clamp(min=1.0)).max()) for x, y in zip(Vs, V2))
    return {
        "problems": len(probs),
        "sides": [p["n"][0] for p in probs],
        "free_nodes": int(sum(b.n_free)),
        "block": block,
        "sweeps_per_graph": S,
        "autotune_seconds": tune_s,
        "batched_seconds": sec,
        "sequential_seconds": sec2,
        "speedup": sec2 / sec if sec > 0 else None,
        "batched_evals_per_s": evals / sec if sec > 0 else None,
        "sweeps": [s["sweeps"] for s in st],
        "all_converged": bool(all(s["converged"] for s in st)) and bool(all(s["converged"] for s in st2)),
        "max_rel_diff_batched_vs_sequential": diff,
        "tol_rel": tol,
    }


def greedy_vs_seeded(ctx, V, ang, reps=5):
    """The greedy step's two searches on the state the timed steps leave
    (policy iteration under way): the full search (coast + scan 64 + golden
    12) against the seeded local search (8 thrust evaluations around each
    node's previous angle, the paper's warm start) with its fallback to the
    full search where the result moves the node's value by more than 1e-5
    relative.  Device time per sweep (events; the seeded sweep includes its
    second pass over the deferred nodes) and the fraction that fell back."""
    import torch

    from paper_2407_14675_amd import inputs

    W = torch.empty_like(V)
    a2, t2 = ctx.empty_policy()
    r = torch.zeros(5, dtype=torch.float64, device="cuda")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(reps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / reps

    full_ms = timed(lambda: ctx.bellman_sweep(V, W, a2, t2, resid=r))
    resid = float(r[0])
    seed = ang.clone()
    ctx.set_search(inputs.SEEDED)
    seeded_ms = timed(lambda: ctx.bellman_sweep_seeded(V, W, a2, t2, seed, resid=r))
    fallback = float(r[4]) / max(1, ctx.n_free)
    ctx.set_search(ctx.problem["search"])
    del W, a2, t2, seed
    return {"full_search_ms": full_ms, "seeded_ms": seeded_ms, "seeded_over_full": seeded_ms / full_ms,
            "fallback_fraction": fallback, "resid_max_rel": resid,
            "what": "one greedy sweep of the 96^3 x 64 grid on the value the timed steps leave; seeds = the "
                    "previous greedy angles; kernels k_sweep_fast<1> and k_sweep_fast<2> + k_sweep_fallback"}


MLP_FLOPS_PER_SAMPLE = 6 * (4 * 128 + 128 * 128 + 128 * 3)  # forward 2 x MAC, backward 4 x MAC


def rel_diff(A, B, free):
    d = (A - B).abs() / B.abs().clamp(min=1.0)
    d[~free] = 0
    return float(d.max()), int((d > 1e-4).sum())


# Plain and network-seeded solves of the held-out thrust level, each solved
# this many times in alternation and compared at the median (the solves are
# deterministic, so the runs differ in timing only).
HELD_OUT_RUNS = 5

# Policy iteration from a 1e-6 stop on to the float32 floor: stop at a
# relative one-step residual of 3e-7 or on a stall.  The one-step residual
# understates the distance to the fixed point by the iteration's horizon: on
# the 24 x 24 x 24 x 16 version of the 96 x 96 x 96 x 64 problem the 1e-6 stop
# is 2.1e-4 away from the oracle's converged solution, 3e-7 is 1.8e-5 away.
FLOOR_TOL = 3e-7


def to_float32_floor(ctx, V, a, t, eval_sweeps, free, ref=None):
    """Policy iteration on, in place, from a 1e-6 stop to the float32 floor:
    the extra time and steps, the largest change it made, and (with ref) the
    distance of the result from the reference solution."""
    import torch

    from paper_2407_14675_amd import inputs

    V6 = V.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, st = ctx.solve_pi(V, a, t, tol_rel=FLOOR_TOL, eval_sweeps=eval_sweeps, max_outer=3000)
    torch.cuda.synchronize()
    out = {"extra_seconds": time.perf_counter() - t0, "extra_outer": st["sweeps"], "tol_rel": FLOOR_TOL,
           "converged": bool(st["converged"]), "stalled": bool(st["stalled"]), "resid_max_rel": st["resid_max_rel"],
           "V_x0": ctx.value_at(V, inputs.X0)}
    out["max_rel_change_from_1e-6_stop"], out["nodes_changed_over_1e-4"] = rel_diff(V6, V, free)
    if ref is not None:
        out["max_rel_diff_vs_reference"], out["nodes_over_1e-4"] = rel_diff(V, ref, free)
    del V6
    return out


def sweep_times(ctx, V, reps=5):
    """Event-timed average of one greedy sweep and one evaluation sweep (the
    descriptors of that greedy sweep) from the value V, in ms."""
    import torch

    W = torch.empty_like(V)
    ang, thr = ctx.empty_policy()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ctx.bellman_sweep(V, W, ang, thr)
    ev0.record(stream)
    for _ in range(reps):
        ctx.bellman_sweep(V, W, ang, thr)
    ev1.record(stream)
    torch.cuda.synchronize()
    greedy_ms = ev0.elapsed_time(ev1) / reps
    ctx.policy_eval_sweep_last(V, W)
    ev0.record(stream)
    for _ in range(reps):
        ctx.policy_eval_sweep_last(V, W)
    ev1.record(stream)
    torch.cuda.synchronize()
    return greedy_ms, ev0.elapsed_time(ev1) / reps


def one_gpu_share(p, full_greedy_ms, full_eval_ms, gpus=8):
    """The kernels on one GPU's share of the m-sharded grid at its real shape:
    the top 64/gpus mass planes plus the ghost plane below them (the plane a
    neighbour would send), after 200 value-iteration sweeps on the slab."""
    from paper_2407_14675_amd import dpo

    n = p["n"]
    planes = n[3] // gpus
    h_m = (p["hi"][3] - p["lo"][3]) / (n[3] - 1)
    first = n[3] - planes - 1
    q = dict(p, n=(n[0], n[1], n[2], planes + 1), lo=tuple(p["lo"][:3]) + (p["lo"][3] + first * h_m,),
             name=p["name"] + f"_slab{planes}+1")
    ctx = dpo.Context(q)
    V = ctx.init_value()
    a, t = ctx.empty_policy()
    ctx.solve_vi(V, a, t, tol_rel=0.0, max_sweeps=200, check_every=200)
    g, e = sweep_times(ctx, V)
    return {"gpus": gpus, "grid": list(q["n"]), "nodes": ctx.N, "greedy_ms": g, "eval_ms": e,
            "full_grid_greedy_ms_over_gpus": full_greedy_ms / gpus, "full_grid_eval_ms_over_gpus": full_eval_ms / gpus}


def solve_to_floor(ctx, V, a, t, schedule, seed=None, free=None, ref=None):
    """A timed solve from the value in V: `schedule` = "vi_pi" (value
    iteration to 1e-3, then policy iteration to 1e-6: the workload's
    schedule) or "pi" (policy iteration from V); with seed, the first policy
    iteration runs seeded (the context's search must be SEEDED and is reset
    to the full search after it).  Then policy iteration on with the full
    search to the float32 floor (3e-7 or a stall).  Returns the record with
    the times of both stops and, with ref, the distance from it."""
    import torch

    from paper_2407_14675_amd import inputs

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    vi = None
    if schedule == "vi_pi":
        rc, vi = ctx.solve_vi(V, a, t, tol_rel=1e-3, max_sweeps=20000, check_every=16)
        torch.cuda.synchronize()
    t1 = time.perf_counter()
    rc, st = ctx.solve_pi(V, a, t, tol_rel=1e-6, eval_sweeps=inputs.EVAL_SWEEPS, max_outer=3000, seed=seed)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    rec = {"vi_sweeps": vi["sweeps"] if vi else 0, "vi_seconds": t1 - t0, "pi_outer": st["sweeps"],
           "pi_eval_sweeps": st["eval_sweeps"], "pi_seconds": t2 - t1, "seconds_to_1e-6": t2 - t0,
           "evals": (vi["evals"] if vi else 0) + st["evals"], "converged": bool(st["converged"]),
           "resid_max_rel": st["resid_max_rel"]}
    if seed is not None:
        rec["verify_steps"] = st["verify_steps"]
        rec["fallback_nodes"] = st["fallback_nodes"]
        ctx.set_search(inputs.SCAN_GOLDEN)
    if ref is not None and free is not None:
        rec["max_rel_diff_vs_reference_at_1e-6"], _ = rel_diff(V, ref, free)
    fl = to_float32_floor(ctx, V, a, t, inputs.EVAL_SWEEPS, free, ref=ref)
    rec["to_float32_floor"] = fl
    rec["seconds_to_float32_floor"] = rec["seconds_to_1e-6"] + fl["extra_seconds"]
    rec["V_x0"] = ctx.value_at(V, inputs.X0)
    return rec


def train_network(ctx, V, a, t):
    """The control-proposal network trained on a converged solution: 2M
    (state, control) pairs from the free nodes with V < 0.98 M, 10 epochs of
    Adam (step 2e-3) in batches of 16384, on the device.  Returns the network
    and the record (seconds include drawing the pairs)."""
    import torch

    from paper_2407_14675_amd import dpo, inputs

    p = ctx.problem
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nodes = ctx.feasible_nodes(V, inputs.MLP_FEASIBLE_FRAC * p["M"])
    sel = inputs.mlp_pair_selection(nodes.numel())
    x, tgt = ctx.gather_pairs(nodes, sel, a, t)
    net = dpo.Mlp(inputs.mlp_params32())
    net.set_adam(lr=inputs.MLP_LR)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hist = None
    for order in inputs.mlp_epoch_orders(x.shape[0], batch=inputs.MLP_BATCH):
        hist = net.train_epoch(x, tgt, perm=order, batch=inputs.MLP_BATCH)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    samples = x.shape[0] * inputs.MLP_EPOCHS
    rec = {"pairs": int(x.shape[0]), "feasible_nodes": int(nodes.numel()), "epochs": inputs.MLP_EPOCHS,
           "batch": inputs.MLP_BATCH, "lr": inputs.MLP_LR, "seconds": t2 - t0, "pair_seconds": t1 - t0, "train_seconds": t2 - t1,
           "final_loss": float(hist.mean()), "tflops": samples * MLP_FLOPS_PER_SAMPLE / (t2 - t1) / 1e12,
           "mfma_bf16_peak_tflops": 2500.0}
    del x, tgt, nodes
    return net, rec


def bench_converge_and_learned(with_walk=True):
    """96 x 96 x 96 x 64, thrust 1e-3: the workload's schedule from V0 to
    1e-6 and on to the float32 floor (the reference), and plain policy
    iteration from V0 (to 1e-6 and the floor) against it; walk-seeded policy
    iteration (seeds = the previous greedy angles); the network trained on
    the reference; then the held-out thrust 5e-4: plain policy iteration
    from V0 against network-seeded policy iteration (proposal, seeded phase,
    full-search certification) to the floor, the seeded time counted with
    and without the training."""
    import torch

    from paper_2407_14675_amd import dpo, inputs

    out = {"grid": [96, 96, 96, 64]}
    p = inputs.large_problem(accel=1e-3)
    ctx = dpo.Context(p)
    free = ctx.kind() == 0
    V = ctx.init_value()
    a, t = ctx.empty_policy()
    ref = solve_to_floor(ctx, V, a, t, "vi_pi", free=free)
    out["reference_a1e-3"] = ref
    log(f"bench: 96^3 x 64 reference {ref}")
    Vp = ctx.init_value()
    ap, tp = ctx.empty_policy()
    out["plain_pi_a1e-3"] = plain = solve_to_floor(ctx, Vp, ap, tp, "pi", free=free, ref=V)
    log(f"bench: plain PI a=1e-3 {plain}")
    del Vp, ap, tp
    if with_walk:
        ctx.set_search(inputs.SEEDED)
        Vw = ctx.init_value()
        aw, tw = ctx.empty_policy()
        walk = solve_to_floor(ctx, Vw, aw, tw, "pi", seed=aw, free=free, ref=V)
        walk["speedup_vs_plain_pi_to_floor"] = plain["seconds_to_float32_floor"] / walk["seconds_to_float32_floor"]
        walk["speedup_vs_plain_pi_to_1e-6"] = plain["seconds_to_1e-6"] / walk["seconds_to_1e-6"]
        walk["eval_ratio_vs_plain_pi"] = plain["evals"] / max(1, walk["evals"])
        out["walk_seeded_pi_a1e-3"] = walk
        log(f"bench: walk-seeded PI a=1e-3 {walk}")
        del Vw, aw, tw
    net, out["mlp_training"] = train_network(ctx, V, a, t)
    log(f"bench: network {out['mlp_training']}")
    del V, a, t, free
    ctx.close()
    torch.cuda.empty_cache()

    # held-out thrust level: plain and network-seeded policy iteration, each
    # solved HELD_OUT_RUNS times in alternation, medians compared.  The
    # float32-floor stop is a stall test (32 steps without a new lowest
    # residual): deterministic for one solve, but its step count moves by
    # tens of steps with small changes of the state it starts from.
    import statistics

    q = inputs.large_problem(accel=5e-4)
    cq = dpo.Context(q)
    free = cq.kind() == 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seed = net.propose(cq)
    torch.cuda.synchronize()
    prop_s = time.perf_counter() - t0
    plains, seededs, Vref = [], [], None
    for r in range(HELD_OUT_RUNS):
        cq.set_search(inputs.SCAN_GOLDEN)
        Vq = cq.init_value()
        aq, tq = cq.empty_policy()
        plains.append(solve_to_floor(cq, Vq, aq, tq, "pi", free=free, ref=Vref))
        log(f"bench: plain PI a=5e-4, run {r} {plains[-1]}")
        if Vref is None:
            Vref = Vq
        del aq, tq
        cq.set_search(inputs.SEEDED)
        Vs = cq.init_value()
        as_, ts = cq.empty_policy()
        seededs.append(solve_to_floor(cq, Vs, as_, ts, "pi", seed=seed, free=free, ref=Vref))
        log(f"bench: network-seeded PI a=5e-4, run {r} {seededs[-1]}")
        del Vs, as_, ts
    med = lambda recs, k: statistics.median(x[k] for x in recs)
    plain, seeded = plains[0], seededs[0]
    for recs, rec in ((plains, plain), (seededs, seeded)):
        rec["runs"] = len(recs)
        rec["runs_seconds_to_1e-6"] = [x["seconds_to_1e-6"] for x in recs]
        rec["runs_seconds_to_float32_floor"] = [x["seconds_to_float32_floor"] for x in recs]
        rec["runs_floor_extra_outer"] = [x["to_float32_floor"]["extra_outer"] for x in recs]
        rec["median_seconds_to_1e-6"] = med(recs, "seconds_to_1e-6")
        rec["median_seconds_to_float32_floor"] = med(recs, "seconds_to_float32_floor")
    greedy_nodes = cq.n_free * max(1, seeded["pi_outer"] - 1 - seeded["verify_steps"])
    seeded["fallback_fraction"] = seeded["fallback_nodes"] / greedy_nodes
    seeded["propose_seconds"] = prop_s
    seeded["held_out"] = True
    train_s = out["mlp_training"]["seconds"]
    p_floor, s_floor = plain["median_seconds_to_float32_floor"], seeded["median_seconds_to_float32_floor"] + prop_s
    p_6, s_6 = plain["median_seconds_to_1e-6"], seeded["median_seconds_to_1e-6"] + prop_s
    seeded["speedup_vs_plain_pi_to_floor"] = p_floor / s_floor
    seeded["speedup_vs_plain_pi_to_floor_incl_training"] = p_floor / (s_floor + train_s)
    seeded["speedup_vs_plain_pi_to_1e-6"] = p_6 / s_6
    seeded["speedup_vs_plain_pi_to_1e-6_incl_training"] = p_6 / (s_6 + train_s)
    # held-out solves a trained network must serve before its training has
    # paid for itself, at the median times to the floor
    gain = p_floor - s_floor
    seeded["break_even_solves_floor"] = train_s / gain if gain > 0 else None
    seeded["eval_ratio_vs_plain_pi"] = plain["evals"] / max(1, seeded["evals"])
    out["plain_pi_a5e-4"] = plain
    out["nn_seeded_pi_a5e-4"] = seeded
    log(f"bench: network-seeded PI a=5e-4 {seeded}")
    del seed, Vref, free
    cq.close()
    torch.cuda.empty_cache()
    return out


def bench_variants(mask, V_euler):
    """The paper's own step and search variants on the headline's 48^4 masked
    grid, each solved by policy iteration to 1e-6 from V0:
      * table walk: the 73 controls (coast + 72 angles) searched in full on
        the first greedy step and by the walk from the previous optimum after
        it, against the exhaustive search of the same table;
      * Heun foot: scan 64 + golden 12 with the second-order Runge-Kutta foot
        (direct path; evaluation sweeps recompute the foot from the angle),
        against the Euler solve of the headline (V_euler)."""
    import numpy as np
    import torch

    from paper_2407_14675_amd import dpo, inputs

    def solve(problem):
        ctx = dpo.Context(problem, mask=mask)
        V = ctx.init_value()
        ang, thr = ctx.empty_policy()
        torch.cuda.synchronize()
        t = time.perf_counter()
        rc, st = ctx.solve_pi(V, ang, thr, tol_rel=1e-6, eval_sweeps=inputs.EVAL_SWEEPS, max_outer=3000)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t
        return ctx, V, {"seconds": sec, "outer_iterations": st["sweeps"], "converged": bool(st["converged"]),
                        "evals": st["evals"], "evals_per_s": st["evals"] / sec,
                        "V_x0": ctx.value_at(V, inputs.X0), "kernel_path": ctx.kernel_path()}

    out = {}
    table = dict(inputs.PI48, search=dict(mode="table", n_angles=72))
    ct, Vt, rt = solve(table)
    cw, Vw, rw = solve(dict(table, search=dict(mode="table_walk", n_angles=72)))
    free = torch.from_numpy(np.ascontiguousarray(ct.kind().cpu().numpy() == 0)).cuda()
    d = ((Vw - Vt).abs() / Vt.abs().clamp(min=1.0))[free]
    rw.update({"max_rel_diff_vs_table": float(d.max()), "frac_within_1e-4": float((d <= 1e-4).float().mean()),
               "min_diff_vs_table": float((Vw - Vt)[free].min()), "speedup_vs_table": rt["seconds"] / rw["seconds"],
               "evals_ratio_table_over_walk": rt["evals"] / rw["evals"]})
    out["table72_exhaustive"] = rt
    out["table72_walk"] = rw
    log(f"bench: table 72 {rt}")
    log(f"bench: walk 72 {rw}")
    ch, Vh, rh = solve(dict(inputs.PI48, integrator="heun"))
    dh = ((Vh - V_euler).abs() / V_euler.abs().clamp(min=1.0))[free]
    rh.update({"max_rel_diff_vs_euler": float(dh.max()), "median_rel_diff_vs_euler": float(dh.median())})
    out["heun_scan_golden"] = rh
    log(f"bench: heun {rh}")
    return out


def bench_example1(with_cpu=True):
    """The paper's Example 1 at its own size (crown grid 110 x 30 x 30 x 30,
    73 controls, Heun foot, dt = 10 s, discount 1e-3): policy iteration
    (20 evaluation sweeps per step) with the full table at every greedy step
    and with the walk from the previous optimum, policy iteration with the
    evaluation solved exactly by GMRES, and value iteration, each from V0 = M
    to a relative residual of 1e-6; the read-out at the start of the paper's
    orbit raise (circular orbit at 6978 km, theta = 0)."""
    import math

    import torch

    from paper_2407_14675_amd import dpo, inputs

    p = inputs.EX1
    x_start = (inputs.EX1_START_RADIUS, 0.0, math.sqrt(inputs.EX1_MU / inputs.EX1_START_RADIUS), 0.0)
    out = {"grid": list(p["n"]), "nodes": int(inputs.n_nodes(p)), "controls": p["search"]["n_angles"] + 1,
           "integrator": p["integrator"], "tol_rel": 1e-6}

    def run(problem, solver):
        ctx = dpo.Context(problem)
        V = ctx.init_value()
        ang, thr = ctx.empty_policy()
        torch.cuda.synchronize()
        t = time.perf_counter()
        if solver == "pi":
            rc, st = ctx.solve_pi(V, ang, thr, tol_rel=1e-6, eval_sweeps=inputs.EVAL_SWEEPS, max_outer=5000)
        elif solver == "pi_exact":
            rc, st = ctx.solve_pi(V, ang, thr, tol_rel=1e-6, eval_sweeps=-1, max_outer=500)
        else:
            rc, st = ctx.solve_vi(V, ang, thr, tol_rel=1e-6, max_sweeps=200000, check_every=16)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t
        res = {"seconds": sec, "sweeps": st["sweeps"], "eval_sweeps": st["eval_sweeps"],
               "converged": bool(st["converged"]), "stalled": bool(st["stalled"]),
               "resid_max_rel": st["resid_max_rel"], "evals": st["evals"], "evals_per_s": st["evals"] / sec,
               "V_start": ctx.value_at(V, x_start), "kernel_path": ctx.kernel_path()}
        return V, res

    Vt, out["pi_table"] = run(p, "pi")
    log(f"bench: example 1 PI {out['pi_table']}")
    Vw, out["pi_walk"] = run(dict(p, search=dict(mode="table_walk", n_angles=p["search"]["n_angles"])), "pi")
    d = (Vw - Vt).abs() / Vt.abs().clamp(min=1.0)
    out["pi_walk"]["max_rel_diff_vs_table"] = float(d.max())
    out["pi_walk"]["frac_within_1e-4"] = float((d <= 1e-4).float().mean())
    log(f"bench: example 1 PI walk {out['pi_walk']}")
    Ve, out["pi_exact_gmres"] = run(p, "pi_exact")
    out["pi_exact_gmres"]["max_rel_diff_vs_modified_pi"] = float(((Ve - Vt).abs() / Vt.abs().clamp(min=1.0)).max())
    log(f"bench: example 1 PI exact {out['pi_exact_gmres']}")
    Vv, out["vi"] = run(p, "vi")
    out["vi"]["max_rel_diff_vs_pi"] = float(((Vv - Vt).abs() / Vt.abs().clamp(min=1.0)).max())
    out["vi_over_pi_time"] = out["vi"]["seconds"] / out["pi_table"]["seconds"]
    log(f"bench: example 1 VI {out['vi']}")
    out["paper"] = {"pi_seconds": 18 * 60, "vi_seconds": 15 * 3600,
                    "hardware": "MacBook Air laptop, Mex-compiled Matlab (paper Section 4)"}
    out["orbit_raise"] = orbit_raise(p, Vt, x_start, cpu=with_cpu)
    log(f"bench: example 1 orbit raise {out['orbit_raise']}")
    # the second reading of the fuel weight's units: alpha per second of
    # thrust (u_bar read as the on/off throttle), solved and flown the same way
    q = inputs.crown_problem(fuel_reading="throttle")
    Vq, rec = run(q, "pi")
    rec["fuel_weight_per_thrust_second"] = q["w_fuel"]
    rec["orbit_raise"] = orbit_raise(q, Vq, x_start, cpu=False)
    rec["reading"] = "alpha * u_bar with u_bar = 1 while the thruster fires (2.04e-8 per second of thrust)"
    out["fuel_per_thrust_second"] = rec
    log(f"bench: example 1, fuel weight per second of thrust {rec}")
    return out


def orbit_raise(p, V, x_start, horizon_s=5e5, batch=4096, cpu=True):
    """The paper's closed-loop orbit raise on the Example 1 solution V: from
    the circular orbit at 6978 km, the feedback eq:feed with tau = dt and the
    model integrated by RK4, for horizon_s seconds.  Reports when the
    semi-major axis first comes within 1 km of the target, when the thruster
    fires for the last time, and the final errors (radius against the target
    ellipse at the final angle, semi-major axis, eccentricity vector); the
    same loop for `batch` perturbed starts at once (trajectory-steps/s); the
    single raise again with Example 2's drag on the simulated system (the
    feedback still from V of the model without it); and, as this section's
    CPU baseline, the oracle's run of the single trajectory on one host core
    (time, and where its throttle first differs)."""
    import math

    import numpy as np
    import torch

    from paper_2407_14675_amd import dpo, inputs

    mu = p["mu"]
    steps = int(round(horizon_s / p["dt"]))
    ctx = dpo.Context(p)

    def elements(x):
        r, vr, vt, th = x
        v2 = vr * vr + vt * vt
        a = -mu * r / (v2 * r - 2 * mu)
        h = r * vt
        ec, es = h * h / (mu * r) - 1, vr * h / mu
        return a, ec * math.cos(th) + es * math.sin(th), ec * math.sin(th) - es * math.cos(th)

    def raise_once(drag):
        torch.cuda.synchronize()
        t = time.perf_counter()
        final, traj, thr, _ = ctx.simulate(V, np.array([x_start]), tau=p["dt"], steps=steps, drag=drag)
        torch.cuda.synchronize()
        gpu_s = time.perf_counter() - t
        traj = traj.cpu().numpy()[:, 0]
        thr = thr.cpu().numpy()[:, 0]
        a_err = np.array([elements(x)[0] - p["el_a"] for x in traj[::10]])
        near = np.flatnonzero(np.abs(a_err) < 1.0)
        fired = np.flatnonzero(thr)
        xf = traj[-1]
        a, ex, ey = elements(xf)
        e_bar = (p["el_e"] * math.cos(p["el_omega"]), p["el_e"] * math.sin(p["el_omega"]))
        pp = p["el_a"] * (1 - p["el_e"] ** 2)
        r_target = pp / (1 + p["el_e"] * math.cos(xf[3] - p["el_omega"]))
        res = {"gpu_seconds": gpu_s,
               "t_within_1km_of_a_bar_s": float(near[0] * 10 * p["dt"]) if near.size else None,
               "max_abs_a_error_after_that_km": float(np.abs(a_err[near[0]:]).max()) if near.size else None,
               "last_thrust_s": float((fired[-1] + 1) * p["dt"]) if fired.size else None,
               "thrust_fraction": float(thr.mean()),
               "final_radius_error_km": float(abs(xf[0] - r_target)), "final_a_error_km": float(a - p["el_a"]),
               "final_e_error": float(math.hypot(ex - e_bar[0], ey - e_bar[1]))}
        return res, thr

    first, thr = raise_once(0.0)
    out = {"horizon_s": horizon_s, "steps": steps, "tau_s": p["dt"], **first,
           "paper": "target neighbourhood after ~1e5 s, thruster off after ~5e5 s, radius error ~1e-2 km"}
    dragged, _ = raise_once(inputs.EX2_DRAG)
    out["with_drag"] = {"drag_per_km": inputs.EX2_DRAG, **dragged,
                        "paper": "Example 2: close to the raise without drag, with later corrections"}
    # many perturbed starts at once
    rng = np.random.default_rng(5)
    starts = np.tile(np.array(x_start), (batch, 1))
    starts[:, 0] += rng.uniform(-20, 20, size=batch)
    starts[:, 3] = rng.uniform(0, 2 * math.pi, size=batch)
    bsteps = 2000
    torch.cuda.synchronize()
    t = time.perf_counter()
    ctx.simulate(V, starts, tau=p["dt"], steps=bsteps, history=False)
    torch.cuda.synchronize()
    bt = time.perf_counter() - t
    out["batch"] = {"trajectories": batch, "steps": bsteps, "seconds": bt,
                    "trajectory_steps_per_s": batch * bsteps / bt}
    if cpu:
        from oracle.core import Oracle
        o = Oracle(p)
        t = time.perf_counter()
        ofinal, otraj, othr, _ = o.simulate(V.cpu().numpy().astype(np.float64), np.array([x_start]), p["dt"], steps)
        sec = time.perf_counter() - t
        same = (othr[:, 0] == thr)
        out["cpu_baseline"] = {
            "kind": "oracle", "cores": 1, "seconds": sec, "unit": "trajectory-steps/s", "value": steps / sec,
            "sample": f"the same single trajectory, {steps} steps, FP64",
            "steps_before_first_different_throttle": int(np.argmin(same)) if not same.all() else steps,
            "final_radius_km": float(ofinal[0, 0]),
            "last_thrust_s": float((np.flatnonzero(othr[:, 0])[-1] + 1) * p["dt"]) if othr.any() else None}
    return out


def kernel_launch_ms(ctx, fn, stream, reps=20):
    """Average duration of one launch of fn (event-timed over reps
    back-to-back launches on the library's stream, after one untimed)."""
    import torch

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    ev0.record(stream)
    for _ in range(reps):
        fn()
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / reps


def bench_reduced_grid(steps, warmup, with_variants=True):
    """The 48^4 grid restricted to the reachability-masked active set (mask
    from a 12^4 pre-solve: the coarse value interpolated at a fine node below
    0.98*M, dilated by one cell per axis): timed policy-iteration steps, the
    time to a converged value (1e-6, then the float32 floor), and the paper's
    variants on the same grid.  At this size the working set sits in the
    last-level cache, so its sweeps are cache- and latency-bound, not HBM-bound."""
    import torch

    from paper_2407_14675_amd import dpo, inputs

    t_setup = time.perf_counter()
    c0 = dpo.Context(inputs.VI12)
    Vc = c0.init_value()
    a0, t0_ = c0.empty_policy()
    c0.solve_vi(Vc, a0, t0_, tol_rel=1e-7, max_sweeps=20000, check_every=16)
    p1 = inputs.PI48
    mask = c0.mask_from_coarse(Vc, p1, inputs.MASK_THRESHOLD_FRAC * p1["M"], inputs.MASK_DILATE)
    ctx = dpo.Context(p1, mask=mask)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    E = inputs.EVAL_SWEEPS
    V = ctx.init_value()
    ang, thr = ctx.empty_policy()
    if warmup > 0:
        ctx.solve_pi(V, ang, thr, tol_rel=0.0, eval_sweeps=E, max_outer=warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, st = ctx.solve_pi(V, ang, thr, tol_rel=0.0, eval_sweeps=E, max_outer=steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    W = V.clone()
    greedy_ms = kernel_launch_ms(ctx, lambda: ctx.bellman_sweep(V, W, ang, thr), stream)
    eval_ms = kernel_launch_ms(ctx, lambda: ctx.policy_eval_sweep_last(V, W), stream)
    n_free = ctx.n_free
    out = {"grid": list(p1["n"]), "active_free_nodes": int(n_free), "active_fraction": n_free / ctx.N,
           "setup_seconds": setup_s, "steps": st["sweeps"], "ms_per_step": elapsed * 1e3 / max(1, st["sweeps"]),
           "evals_per_s": st["evals"] / elapsed, "greedy_ms": greedy_ms, "eval_ms": eval_ms,
           "eval_bound": "last-level cache / latency (the working set fits the 256 MiB cache)",
           "eval_sweep_bytes": ctx.eval_sweep_bytes()}
    Vc1 = ctx.init_value()
    ac, tc = ctx.empty_policy()
    out["time_to_converge"] = conv = solve_to_floor(ctx, Vc1, ac, tc, "pi", free=ctx.kind() == 0)
    log(f"bench: 48^4 {out}")
    if with_variants:
        log("bench: paper variants (table walk, Heun foot)")
        out["paper_variants"] = bench_variants(mask, Vc1)
    del Vc1, ac, tc, V, W
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baselines")
    ap.add_argument("--only-headline", action="store_true",
                    help="only the timed steps and the kernel timings of the headline workload")
    ap.add_argument("--no-converge", action="store_true",
                    help="skip the 96^3 x 64 solves to convergence and the seeded comparisons")
    ap.add_argument("--no-reduced", action="store_true", help="skip the 48^4 reduced-grid workload")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched 16-problem measurement")
    ap.add_argument("--no-example1", action="store_true", help="skip the paper's Example 1 solves")
    ap.add_argument("--no-ceilings", action="store_true", help="skip the HBM and VALU ceiling probes")
    ap.add_argument("--sections", default="all",
                    help="comma list of the sections after the headline: converge, reduced, example1, batched, "
                         "ceilings, share, seeded (default all)")
    ap.add_argument("--eval-path", type=int, default=0, choices=(0, 1, 2),
                    help="kernels of the headline's evaluation sweeps: 0 automatic (LDS value bricks), "
                         "1 corner gathers from global memory, 2 bricks")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run one 1 GiB copy with the library's probe (reference for HBM byte counters)")
    args = ap.parse_args()
    known = {"converge", "reduced", "example1", "batched", "ceilings", "share", "seeded"}
    sections = known if args.sections == "all" else set(args.sections.split(","))
    if not sections <= known:
        ap.error(f"unknown sections {sorted(sections - known)}")
    if args.only_headline:
        sections = set()
    for flag, name in ((args.no_converge, "converge"), (args.no_reduced, "reduced"), (args.no_example1, "example1"),
                       (args.no_batched, "batched"), (args.no_ceilings, "ceilings")):
        if flag:
            sections.discard(name)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); sharding the grid along the mass "
              f"axis over several GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2407_14675_amd import dpo, inputs

    torch.cuda.set_device(0)
    if args.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dpo.probe_copy(src, dst)
        torch.cuda.synchronize()
        del src, dst
    log("bench: setup")

    # ---- headline workload: 96 x 96 x 96 x 64, thrust 1e-3
    t_setup = time.perf_counter()
    p = inputs.large_problem(accel=1e-3)
    ctx = dpo.Context(p)
    ctx.set_eval_path(args.eval_path)
    n_free = ctx.n_free
    V = ctx.init_value()
    ang, thr = ctx.empty_policy()
    rc, st_vi = ctx.solve_vi(V, ang, thr, tol_rel=1e-3, max_sweeps=20000, check_every=16)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    eval_path = ctx.eval_path()
    log(f"bench: set-up {setup_s:.2f} s (value iteration to 1e-3: {st_vi['sweeps']} sweeps), eval path {eval_path}")
    E = inputs.EVAL_SWEEPS
    if args.warmup > 0:
        ctx.solve_pi(V, ang, thr, tol_rel=0.0, eval_sweeps=E, max_outer=args.warmup)
    torch.cuda.synchronize()
    V_start = V.clone()

    # ---- timed region: K outer iterations of modified policy iteration
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, st = ctx.solve_pi(V, ang, thr, tol_rel=0.0, eval_sweeps=E, max_outer=args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    steps_done = st["sweeps"]
    value = st["evals"] / elapsed
    log(f"bench: {steps_done} steps in {elapsed:.4f}s, {value:.3e} evals/s")

    # ---- kernel durations inside the timed steps: the solver records HIP
    # events on its stream (torch's current stream) around every greedy sweep
    # and around every step's run of evaluation sweeps
    greedy_ms = st["greedy_seconds"] * 1e3 / max(1, steps_done)
    eval_ms = st["eval_seconds"] * 1e3 / max(1, st["eval_sweeps"])
    eval_algo_bytes = EVAL_ALGO_BYTES_PER_NODE * n_free
    eval_gbs = eval_algo_bytes / (eval_ms * 1e-3) / 1e9
    stream_bytes = ctx.eval_sweep_bytes()
    greedy_evals = n_free * EVALS_PER_GREEDY_NODE
    greedy_valu = GREEDY_VALU_PER_WAVE * ((n_free + 63) // 64) / (greedy_ms * 1e-3)
    log(f"bench: greedy sweep {greedy_ms:.4f} ms, eval sweep {eval_ms:.4f} ms ({eval_gbs:.0f} GB/s algorithmic)")
    # the counter record holds the brick kernel's bytes
    traffic = measured_traffic() if eval_path == 2 else None
    step_ms = elapsed * 1e3 / max(1, steps_done)

    one_share = None
    if "share" in sections:
        one_share = one_gpu_share(p, greedy_ms, eval_ms)
        log(f"bench: one GPU's share {one_share}")

    seeded_probe = None
    if "seeded" in sections:
        seeded_probe = greedy_vs_seeded(ctx, V, ang)
        log(f"bench: greedy full vs seeded {seeded_probe}")

    cpu = None
    if not args.no_cpu:
        log("bench: cpu baseline")
        cpu = cpu_baseline(p, V_start.cpu().numpy().astype("float64"))
        log(f"bench: cpu {cpu}")
    del V_start
    ctx.close()
    torch.cuda.empty_cache()

    ceilings = None
    if "ceilings" in sections:
        ceilings = measure_ceilings()
        log(f"bench: ceilings {ceilings}")

    converge = None
    if "converge" in sections:
        log("bench: 96^3 x 64 solves to convergence, walk- and network-seeded")
        converge = bench_converge_and_learned()

    reduced = None
    if "reduced" in sections:
        log("bench: 48^4 reduced grid")
        reduced = bench_reduced_grid(args.steps, args.warmup)

    example1 = None
    if "example1" in sections:
        log("bench: the paper's Example 1 (crown grid)")
        example1 = bench_example1(with_cpu=not args.no_cpu)

    batched = None
    if "batched" in sections:
        log("bench: batched 16-problem solve")
        batched = bench_batched()
        log(f"bench: batched {batched}")
        batched["small_grids"] = bench_batched(side_scale=0.25)
        log(f"bench: batched small {batched['small_grids']}")

    ttc = None
    if converge is not None:
        ref = converge["reference_a1e-3"]
        ttc = {"seconds_to_1e-4": ref["seconds_to_float32_floor"], "seconds_to_1e-6_stop": ref["seconds_to_1e-6"],
               "what": "value iteration to 1e-3, policy iteration to 1e-6, then on to the float32 floor "
                       "(3e-7 or a stall): the stop at which the value meets 1e-4 against the oracle",
               "nn_seeded_vs_plain_held_out_to_1e-4": converge["nn_seeded_pi_a5e-4"]["speedup_vs_plain_pi_to_floor"],
               "nn_seeded_vs_plain_held_out_to_1e-4_incl_training":
                   converge["nn_seeded_pi_a5e-4"]["speedup_vs_plain_pi_to_floor_incl_training"],
               "nn_seeded_vs_plain_held_out_to_1e-6_stop":
                   converge["nn_seeded_pi_a5e-4"]["speedup_vs_plain_pi_to_1e-6"],
               "held_out_runs": HELD_OUT_RUNS,
               "held_out_what": "medians over the runs; network trained once on the thrust-1e-3 solution, "
                                "proposal time counted, training time counted only in the _incl_training figure"}

    out = {
        "metric": "node-control Bellman evals/s (modified PI step on 96^3 x 64: greedy scan64+golden12+coast, "
                  "20 policy sweeps) + time-to-converged V at 1e-4 rel; NN-seeded vs plain",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": steps_done,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "policy iteration, 96 x 96 x 96 x 64 grid (56.6M nodes), thrust 1e-3, dt 0.02, "
                        "cost 1 + 0.1*thrust, scan 64 + golden 12 + coast, 20 evaluation sweeps per update, "
                        "from the value after value iteration to 1e-3",
            "grid": list(p["n"]),
            "free_nodes": int(n_free),
            "eval_sweeps": E,
            "steps_requested": args.steps,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_eval_brick_desc<true, true>" if eval_path == 2 else "k_policy_eval_d16<true, 3, 2>",
            "achieved": eval_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": eval_gbs / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes": eval_algo_bytes,
            "algorithmic_bytes_per_node": EVAL_ALGO_BYTES_PER_NODE,
            "stream_bytes_per_launch": stream_bytes,
            "nodes_per_launch": int(n_free),
            "avg_launch_ms": eval_ms,
            "launches_timed": st["eval_sweeps"],
            "launches_per_step": E,
            "share_of_step": E * eval_ms / step_ms,
            "timing": "HIP events recorded by the solver on its stream around each step's evaluation sweeps, "
                      "over the timed steps",
        },
        "greedy_sweep": {
            "kernel": "k_sweep_fast<1>",
            "bound": "alu",
            "avg_launch_ms": greedy_ms,
            "evals_per_launch": greedy_evals,
            "evals_per_s": greedy_evals / (greedy_ms * 1e-3),
            "hbm_bytes_per_node": GREEDY_BYTES_PER_NODE,
            "hbm_frac": GREEDY_BYTES_PER_NODE * n_free / (greedy_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "valu_wave_instr_per_wave": GREEDY_VALU_PER_WAVE,
            "valu_wave_instr_per_s": greedy_valu,
            "valu_peak_unpacked_wave_instr_per_s": VALU_UNPACKED_WAVE_INSTR_PER_S,
            "valu_frac_of_unpacked_peak": greedy_valu / VALU_UNPACKED_WAVE_INSTR_PER_S,
            "valu_frac_of_measured_fma_loop": (greedy_valu / ceilings["valu_wave_instr_per_s"]) if ceilings else None,
            "valu_note": "issue rate from the counted instructions per wave; above 1 because the sweep's moves, "
                         "selects and integer operations issue faster than the FP32 FMAs the peak counts",
        },
        "gather_roofline": {
            "naive_gather_bytes_per_eval": GATHER_BYTES_PER_EVAL,
            "naive_gather_frac": value * GATHER_BYTES_PER_EVAL / 1e9 / HBM_PEAK_GBS,
        },
        "setup": {"seconds": setup_s, "vi_sweeps": st_vi["sweeps"],
                  "what": "context creation and value iteration to 1e-3 (the schedule's first phase), "
                          "not in the timed steps"},
        "greedy_full_vs_seeded": seeded_probe,
        "time_to_converge": ttc,
        "converge_and_learned_96x96x96x64": converge,
        "one_gpu_share": one_share,
        "ceilings": ceilings,
        "reduced_grid_48x4": reduced,
        "paper_example1": example1,
        "batched": batched,
        "cpu_baseline": cpu,
        "host": {"nproc": os.cpu_count(), "cpu": platform.processor()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
