"""The host CPU Simpfer (Algorithms 1-3 as the paper gives them, the
comparison baseline of the benchmark) returns exactly the oracle's result
sets: on the small evaluation workload, on integer vectors with many ties,
and at the edges (k > m, k > k_max with the paper's rebuild, zero users,
empty sets), for several block sizes and prefix lengths."""
import numpy as np
import pytest

import oracle
from cpu_simpfer import CpuSimpfer, set_threads, threads
from paper_2110_07131_amd import datagen


@pytest.fixture(scope="module")
def parity():
    return datagen.config_workload("parity")  # 2,000 x 1,000, d = 50, 20 queries


@pytest.mark.parametrize("lb,b", [(0, 0), (20, 64), (1000, 16), (10, 1)])
def test_equals_oracle_on_the_small_workload(parity, lb, b):
    w = parity
    s = CpuSimpfer(w.Q, w.P, 10, lb_items=lb, block_size=b)
    for qi in w.qidx:
        for k in (1, 5, 10):
            assert np.array_equal(s.query(w.P[qi], k), oracle.brute(w.Q, w.P, w.P[qi], k)), (qi, k)
    s.free()


def test_integer_ties():
    rng = np.random.default_rng(31)
    Q = datagen.small_int_vectors(300, 3, -3, 3, rng)
    P = datagen.small_int_vectors(80, 3, -3, 3, rng)
    Q[::17] = 0.0
    s = CpuSimpfer(Q, P, 6, lb_items=8, block_size=8)
    for j in range(0, 80, 3):
        for k in (1, 2, 6):
            assert np.array_equal(s.query(P[j], k), oracle.brute(Q, P, P[j], k)), (j, k)
    s.free()


def test_edges():
    rng = np.random.default_rng(5)
    w = datagen.workload(130, 7, 5, 0.7, 7, seed=5)
    s = CpuSimpfer(w.Q, w.P, 4)
    q = w.P[3]
    assert np.array_equal(s.query(q, 8), np.arange(130, dtype=np.int32))   # k > m: everyone
    assert np.array_equal(s.query(q, 6), oracle.brute(w.Q, w.P, q, 6))   # k > k_max: rebuild
    assert s.k_max == 6
    s.free()
    e = CpuSimpfer(np.zeros((0, 5), np.float32), w.P, 3)
    assert e.query(q, 2).size == 0
    z = CpuSimpfer(w.Q, np.zeros((0, 5), np.float32), 3)
    assert np.array_equal(z.query(q, 1), np.arange(130, dtype=np.int32))
    v = datagen.vectors(1, 5, 0.5, rng)[0]
    assert np.array_equal(CpuSimpfer(w.Q, w.P, 4).query(v, 2), oracle.brute(w.Q, w.P, v, 2))


def test_thread_count_does_not_change_results(parity):
    w = parity
    s = CpuSimpfer(w.Q, w.P, 10)
    t0 = threads()
    set_threads(1)
    one = [s.query(w.P[qi], 5) for qi in w.qidx[:6]]
    set_threads(t0)
    many = [s.query(w.P[qi], 5) for qi in w.qidx[:6]]
    assert all(np.array_equal(a, b) for a, b in zip(one, many))
    s.free()
