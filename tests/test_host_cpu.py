"""Host-side logic on the CPU: the seeded input recipe, the counter-based
traffic summary, and the benchmark's roofline arithmetic."""
import csv
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2110_07131_amd import datagen, profiling  # noqa: E402


# --- seeded synthetic inputs -------------------------------------------------

def test_workload_is_deterministic_per_seed():
    a = datagen.workload(500, 200, 16, 0.5, 20, seed=3, k_choices=[1, 5])
    b = datagen.workload(500, 200, 16, 0.5, 20, seed=3, k_choices=[1, 5])
    c = datagen.workload(500, 200, 16, 0.5, 20, seed=4, k_choices=[1, 5])
    assert np.array_equal(a.Q, b.Q) and np.array_equal(a.P, b.P) and np.array_equal(a.qidx, b.qidx)
    assert not np.array_equal(a.Q, c.Q)
    assert a.Q.dtype == np.float32 and a.P.dtype == np.float32


def test_vectors_have_log_normal_norms():
    rng = np.random.default_rng(0)
    v = datagen.vectors(200_000, 8, 0.5, rng)
    r = np.log(np.linalg.norm(v.astype(np.float64), axis=1))
    assert abs(r.mean()) < 0.01 and abs(r.std() - 0.5) < 0.01
    # directions are isotropic: the mean unit vector is near zero
    u = v / np.linalg.norm(v, axis=1, keepdims=True)
    assert np.abs(u.mean(axis=0)).max() < 0.01


def test_queries_are_distinct_items_and_k_lists_expand():
    w = datagen.workload(300, 100, 8, 0.5, 40, seed=1, k_choices=[1, 5, 10])
    items = w.qidx[::3]
    assert len(np.unique(items)) == len(items) == 40
    assert np.all(w.qidx.reshape(-1, 3) == items[:, None])  # item-major cross product
    assert w.ks.tolist() == [1, 5, 10] * 40
    u = datagen.workload(300, 100, 8, 0.5, 40, seed=1, k_choices="uniform", k_max=7)
    assert u.ks.min() >= 1 and u.ks.max() <= 7


# --- traffic summary from counter runs ---------------------------------------

def _write_counters(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "pmc_counter_collection.csv"), "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writerows(rows)


def test_traffic_summary_from_counter_files(tmp_path):
    f, wdir = str(tmp_path / "f"), str(tmp_path / "w")
    # a 1 GiB copy reads half its bytes on FETCH_SIZE, all on WRITE_SIZE;
    # the kernel's per-dispatch values come in two dimensions to be summed
    _write_counters(f, [[1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 524288],
                        [2, "void rk::k_bfilter<false, 4>(...)", "FETCH_SIZE", 10000],
                        [2, "void rk::k_bfilter<false, 4>(...)", "FETCH_SIZE", 2000],
                        [3, "void rk::k_bfilter<false, 4>(...)", "FETCH_SIZE", 12000],
                        [4, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 3]])
    _write_counters(wdir, [[1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1048576],
                           [2, "void rk::k_bfilter<false, 4>(...)", "WRITE_SIZE", 500]])
    fr = profiling.read_counter(f, "FETCH_SIZE")
    wr = profiling.read_counter(wdir, "WRITE_SIZE")
    ff, fmeas = profiling.copy_factor(fr, 1 << 30)
    wf, _ = profiling.copy_factor(wr, 1 << 30)
    assert ff == pytest.approx(2.0) and fmeas == 524288 and wf == pytest.approx(1.0)
    avg, n = profiling.kernel_average(fr, "k_bfilter")
    assert n == 2 and avg == pytest.approx(12000.0)
    with pytest.raises(ValueError):
        profiling.kernel_average(fr, "k_bscan")
    # a phase: everything matching, per dispatch of the phase's first kernel
    rows = [("k_bscan<4, false>", 10.0), ("k_bscan<4, true>", 1.0), ("k_bdecide", 2.0),
            ("k_bscan<4, false>", 20.0), ("k_bscan<4, true>", 3.0), ("k_bdecide", 4.0)]
    tot, n = profiling.kernel_average(rows, "k_bscan|k_bdecide", r"k_bscan<\d+, false>")
    assert n == 2 and tot == pytest.approx(20.0)


def test_source_hash_is_stable_per_kernel():
    h = profiling.source_hash("k_bfilter")
    assert h == profiling.source_hash("k_bfilter") and len(h) == 16
    assert profiling.source_hash("k_bscan") != h  # its own source file
    assert profiling.source_hash("k_filter") != h


def test_source_hash_ignores_comments_only():
    a = 'int f(int x) { // twice\n  return 2 * x; /* not */\n}\nconst char* s = "//kept";\n'
    b = '/* header */\nint f(int x) { // once\n  return 2 * x; /* other */\n\n}\nconst char* s = "//kept";\n'
    sa = profiling.strip_comments(a)
    assert sa == profiling.strip_comments(b)
    assert '"//kept"' in sa and "twice" not in sa and "not" not in sa
    assert profiling.strip_comments("x = 1; // a") != profiling.strip_comments("x = 2; // a")


# --- benchmark roofline arithmetic -------------------------------------------

def test_dominant_roofline_arithmetic():
    import bench
    st = {"users_evaluated": 1_000_000, "scan_items": 0, "blocks_visited": 0, "blocks_pruned": 0}
    r = bench.dominant_roofline("batch_filter", (0.5, 1), st, 50, "fp32")
    # 2 d flops per evaluated pair in 0.5 ms
    assert r["achieved"] == pytest.approx(2 * 50 * 1e6 / 0.5e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3) and r["bound"] == "mfma"
    st["scan_items"] = 2_000_000
    r = bench.dominant_roofline("batch_pairs", (2.0, 2), st, 50, "bf16")
    assert r["kernel"] == "k_bscan" and r["peak"] == 157.3  # the scan runs float32 MFMA
    assert r["algorithmic_flops_per_launch"] == pytest.approx(2 * 50 * 2e6 / 2)
