"""Host-side logic on the CPU: the network's epoch orders, the benchmark's
argument handling, and the guard that keeps a counter measurement from being
reported for kernel sources it was not taken on."""
import json
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

from paper_2407_14675_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("n,batch", [(1, 4096), (5, 3), (4096, 4096), (10000, 4096), (3 * 16384 + 7, 16384)])
def test_epoch_orders_are_permutations_of_cyclic_windows(n, batch):
    orders = list(inputs.mlp_epoch_orders(n, epochs=4, batch=batch, seed=9))
    assert len(orders) == 4
    nb = -(-n // batch)
    for o in orders:
        assert o.dtype == np.int32 and o.shape == (n,)
        np.testing.assert_array_equal(np.sort(o), np.arange(n))
        # runs of consecutive indices (cyclically): at most one break per window
        breaks = int(np.count_nonzero((o[1:] - o[:-1]) % n != 1)) if n > 1 else 0
        assert breaks <= nb
    if n > batch:
        assert any(not np.array_equal(orders[0], o) for o in orders[1:])
    again = list(inputs.mlp_epoch_orders(n, epochs=4, batch=batch, seed=9))
    for a, b in zip(orders, again):
        np.testing.assert_array_equal(a, b)


def test_pair_selection_is_random_order_without_repeats():
    sel = inputs.mlp_pair_selection(100000, n_pairs=5000, seed=4)
    assert sel.dtype == np.int32 and len(np.unique(sel)) == 5000
    assert sel.min() >= 0 and sel.max() < 100000
    assert not np.all(np.diff(sel) > 0)  # not sorted: the windows of an epoch mix the grid
    np.testing.assert_array_equal(inputs.mlp_pair_selection(100000, n_pairs=5000, seed=4), sel)
    assert len(inputs.mlp_pair_selection(300, n_pairs=5000)) == 300


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_bench_runs_on_one_gpu_only():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_bench_rejects_unknown_sections():
    r = run_bench("--sections", "converge,nonsense")
    assert r.returncode == 2 and "nonsense" in r.stderr


@pytest.fixture()
def bench_mod(tmp_path, monkeypatch):
    """bench imported with its kernel sources and counter record copied to a
    scratch tree."""
    sys.path.insert(0, ROOT)
    import bench

    csrc = tmp_path / "paper_2407_14675_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in bench.KERNEL_SOURCES:
        shutil.copy(os.path.join(ROOT, "paper_2407_14675_amd", "csrc", f), csrc / f)
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "profiles" / "traffic.json"))
    return bench, csrc


def test_source_hash_ignores_comments_and_space_only(bench_mod):
    bench, csrc = bench_mod
    h0 = bench.kernel_source_hash()
    f = csrc / bench.KERNEL_SOURCES[0]
    text = f.read_text()
    f.write_text("// a new comment line\n" + text.replace("\n", "\n\n", 3) + "\n/* block\ncomment */\n")
    assert bench.kernel_source_hash() == h0
    f.write_text(text + "\nstatic int unused_for_the_test = 1;\n")
    assert bench.kernel_source_hash() != h0


def test_traffic_reported_only_for_the_sources_it_was_measured_on(bench_mod):
    bench, csrc = bench_mod
    assert bench.measured_traffic() is None  # no record
    rec = {"bytes_per_launch": 1.5e9, "source_hash": bench.kernel_source_hash()}
    with open(bench.TRAFFIC_FILE, "w") as fh:
        json.dump(rec, fh)
    assert bench.measured_traffic() == 1.5e9
    f = csrc / bench.KERNEL_SOURCES[1]
    f.write_text(f.read_text() + "\nstatic int changed_for_the_test = 2;\n")
    assert bench.measured_traffic() is None


def test_committed_traffic_record_matches_the_sources():
    """The counter record in profiles/ was taken on the kernel sources as they
    are: otherwise bench reports no traffic and the record is stale."""
    sys.path.insert(0, ROOT)
    import bench

    with open(os.path.join(ROOT, "profiles", "k_eval_brick_desc_96x96x96x64_traffic.json")) as fh:
        rec = json.load(fh)
    assert rec["source_hash"] == bench.kernel_source_hash()
    assert rec["algorithmic_bytes_per_launch"] == 16 * 56592384
