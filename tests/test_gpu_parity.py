"""GPU parity: the HIP path against the float64 CPU oracle, through the C ABI.

Result sets must be identical (no tolerance).  Index arrays are compared bit
for bit: the library computes every stored lower bound in float64 in the
oracle's summation order.
"""
import numpy as np
import pytest

import oracle
from paper_2110_07131_amd import datagen, rkmips
from paper_2110_07131_amd.rkmips import Index

pytestmark = pytest.mark.gpu

MODES = [(0, "fp32"), (0, "bf16"), (20, "fp32"), (20, "bf16")]  # (lb_items, precision)


def f32_down(x64):
    f = x64.astype(np.float32)
    over = f.astype(np.float64) > x64
    f[over] = np.nextafter(f[over], np.float32(-np.inf))
    return f


@pytest.fixture(scope="module")
def parity():
    return datagen.config_workload("parity")  # n=2000, m=1000, d=50, k_max=10, 20 queries


@pytest.mark.parametrize("lb,prec", MODES)
def test_index_build_matches_algorithm1(parity, lb, prec):
    w = parity
    kmax = 10
    idx = Index.build(w.Q, w.P, kmax, lb_items=lb, precision=prec)
    pre = oracle.preprocess(w.Q, w.P, kmax, lb if lb else w.P.shape[0], 64)
    assert np.array_equal(idx.export(rkmips.RK_F_PERM_Q), pre["permQ"])
    assert np.array_equal(idx.export(rkmips.RK_F_PERM_P), pre["permP"])
    assert np.array_equal(idx.export(rkmips.RK_F_SQNORM_Q), pre["s2Q"])
    assert np.array_equal(idx.export(rkmips.RK_F_SQNORM_P), pre["s2P"])
    L64 = idx.export(rkmips.RK_F_L64)
    assert np.array_equal(L64, pre["L"])
    L32 = idx.export(rkmips.RK_F_L32)
    assert np.array_equal(L32, f32_down(pre["L"]))
    LB = idx.export(rkmips.RK_F_LB)
    assert np.array_equal(LB, f32_down(pre["LB"]))
    nQ = idx.export(rkmips.RK_F_NORM_Q)
    nP = idx.export(rkmips.RK_F_NORM_P)
    # upward-rounded norms bound the exact norms of the float32 rows
    assert np.all(nQ.astype(np.float64) ** 2 >= pre["s2Q"][pre["permQ"]] * (1 + 1e-15))
    assert np.all(nP.astype(np.float64) ** 2 >= pre["s2P"][pre["permP"]] * (1 + 1e-15))
    assert np.all(np.diff(nQ) <= 0) and np.all(np.diff(nP) <= 0)
    assert np.array_equal(idx.export(rkmips.RK_F_BNORM), nQ[::64])
    idx.free()


@pytest.mark.parametrize("lb,prec", MODES)
def test_result_sets_equal_oracle(parity, lb, prec):
    w = parity
    idx = Index.build(w.Q, w.P, 10, lb_items=lb, precision=prec)
    for qi in w.qidx:
        q = w.P[qi]
        for k in (1, 2, 5, 10):
            got = idx.reverse_kmips(q, k)
            want = oracle.brute(w.Q, w.P, q, k)
            assert np.array_equal(got, want), (qi, k)
    idx.free()


@pytest.mark.parametrize("lb,prec", MODES)
def test_certified_decisions_are_sound(parity, lb, prec):
    w = parity
    idx = Index.build(w.Q, w.P, 10, lb_items=lb, precision=prec)
    idx.set_counting(True)
    yes_cls = {rkmips.RK_C_LEMMA2_YES, rkmips.RK_C_TABLE_YES, rkmips.RK_C_SCAN_YES, rkmips.RK_C_RECHECK_YES}
    for qi in w.qidx[:8]:
        for k in (1, 3, 10):
            cls, shat = idx.trace(w.P[qi], k)
            member = oracle.brute_mask(w.Q, w.P, w.P[qi], k)
            assert set(np.unique(cls)) <= set(range(8))
            assert np.array_equal(np.isin(cls, list(yes_cls)), member), (qi, k)
            # the bulk-precision u.q is within its certified margin of f(q,u)
            ev = ~np.isnan(shat)
            f = oracle.pair_dots(w.Q, w.P, np.nonzero(ev)[0], np.full(ev.sum(), qi))
            rel = np.abs(shat[ev] - f) / (np.linalg.norm(w.Q[ev].astype(np.float64), axis=1)
                                         * np.linalg.norm(w.P[qi].astype(np.float64)))
            assert rel.max() < (8e-3 if prec == "bf16" else 1e-5)
    st = idx.stats()
    assert st["blocks_visited"] > 0 and st["users_evaluated"] > 0
    if lb:
        assert st["survivors"] > 0 and st["scan_items"] > 0
    idx.free()


def test_batch_equals_single_queries(parity):
    w = parity
    idx = Index.build(w.Q, w.P, 10)
    ks = np.array([1, 3, 10, 2, 7] * 4, np.int32)[: len(w.qidx)]
    off, ids = idx.reverse_kmips_batch(w.queries, ks)
    for i, qi in enumerate(w.qidx):
        assert np.array_equal(ids[off[i]:off[i + 1]], oracle.brute(w.Q, w.P, w.P[qi], ks[i]))
    idx.free()


@pytest.mark.parametrize("n,m,d,kmax", [(130, 70, 3, 5), (64, 64, 1, 4), (65, 9, 7, 12), (1, 1, 2, 1),
                                         (200, 40, 512, 8), (300, 1500, 17, 6)])
@pytest.mark.parametrize("lb,prec", MODES)
def test_ragged_and_small_shapes(n, m, d, kmax, lb, prec):
    w = datagen.workload(n, m, d, 0.7, 5, seed=n + m + d)
    idx = Index.build(w.Q, w.P, kmax, lb_items=min(lb, m) if lb else 0, precision=prec)
    for qi in w.qidx:
        for k in sorted({1, min(kmax, 3), kmax}):
            assert np.array_equal(idx.reverse_kmips(w.P[qi], k), oracle.brute(w.Q, w.P, w.P[qi], k)), (qi, k)
    # a query that is not an item
    q = datagen.vectors(1, d, 0.7, np.random.default_rng(1))[0] * 2
    assert np.array_equal(idx.reverse_kmips(q, 1), oracle.brute(w.Q, w.P, q, 1))
    idx.free()


@pytest.mark.parametrize("lb,prec", MODES)
def test_integer_vectors_with_ties(lb, prec):
    # all products exact in every precision; many exact ties between q's
    # duplicate and other items, and zero users (always members)
    rng = np.random.default_rng(4)
    Q = datagen.small_int_vectors(300, 4, -3, 3, rng)
    P = datagen.small_int_vectors(90, 4, -3, 3, rng)
    Q[::17] = 0.0
    idx = Index.build(Q, P, 6, lb_items=lb, precision=prec)
    for j in range(0, 90, 7):
        for k in (1, 2, 6):
            assert np.array_equal(idx.reverse_kmips(P[j], k), oracle.brute(Q, P, P[j], k)), (j, k)
    idx.free()


def test_degenerate_sizes():
    rng = np.random.default_rng(0)
    Q = datagen.vectors(50, 8, 0.5, rng)
    P = datagen.vectors(6, 8, 0.5, rng)
    q = P[2]
    idx = Index.build(Q, P, 10)  # m < k_max
    assert np.array_equal(idx.reverse_kmips(q, 7), np.arange(50))  # k > m: everyone
    for k in range(1, 7):
        assert np.array_equal(idx.reverse_kmips(q, k), oracle.brute(Q, P, q, k))
    idx.free()
    idx = Index.build(Q, P[:0], 3)  # m = 0
    assert np.array_equal(idx.reverse_kmips(q, 1), np.arange(50))
    idx.free()
    idx = Index.build(Q[:0], P, 3)  # n = 0
    assert idx.reverse_kmips(q, 2).size == 0
    off, ids = idx.reverse_kmips_batch(np.stack([q, q]), [1, 2])
    assert off.tolist() == [0, 0, 0] and ids.size == 0
    idx.free()


def test_k_above_kmax_and_rebuild(parity):
    w = parity
    idx = Index.build(w.Q, w.P, 4)
    q = w.P[w.qidx[0]]
    with pytest.raises(rkmips.RkError) as e:
        idx.reverse_kmips(q, 5)
    assert e.value.status == rkmips.RK_E_KMAX
    with pytest.raises(rkmips.RkError) as e:
        idx.reverse_kmips(q, 0)
    assert e.value.status == rkmips.RK_E_INVAL
    idx.rebuild(8)
    assert np.array_equal(idx.reverse_kmips(q, 8), oracle.brute(w.Q, w.P, q, 8))
    idx.free()
    idx = Index.build(w.Q, w.P, 4, auto_rebuild=True)
    assert np.array_equal(idx.reverse_kmips(q, 9), oracle.brute(w.Q, w.P, q, 9))
    assert idx.stats()["rebuilds"] == 1 and idx.stats()["k_max"] == 9
    idx.free()


def test_truncation_reports_true_count(parity):
    w = parity
    idx = Index.build(w.Q, w.P, 10)
    q = w.P[w.qidx[0]]
    want = oracle.brute(w.Q, w.P, q, 10)
    L = rkmips.lib()
    import ctypes
    ids = np.empty(2, np.int32)
    cnt = ctypes.c_int64()
    st = L.rk_reverse_kmips(idx._h, q.ctypes.data, 10, ids.ctypes.data, 2, ctypes.byref(cnt))
    if len(want) > 2:
        assert st == rkmips.RK_E_TRUNC and cnt.value == len(want)
        assert ids.tolist() == want[:2].tolist()
    idx.free()


@pytest.mark.parametrize("cap", [0, 27])
def test_full_table_candidate_build(cap):
    # m > 1024 takes the MFMA candidate pass + float64 refine; a tiny
    # candidate capacity forces the exact overflow path for many users.
    w = datagen.workload(1500, 3000, 24, 0.5, 6, seed=5)
    kmax = 25
    idx = Index.build(w.Q, w.P, kmax, cand_cap=cap)
    st = idx.stats()
    pre = oracle.preprocess(w.Q, w.P, kmax, 3000, 64)
    assert np.array_equal(idx.export(rkmips.RK_F_L64), pre["L"])
    if cap:
        assert st["build_cand_overflow_users"] > 0
    else:
        assert st["build_cand_overflow_users"] == 0
    for qi in w.qidx:
        for k in (1, 25):
            assert np.array_equal(idx.reverse_kmips(w.P[qi], k), oracle.brute(w.Q, w.P, w.P[qi], k))
    idx.free()


def test_long_prefix_lower_bounds():
    # lb_items between the float64 seed prefix and m
    w = datagen.workload(700, 2600, 16, 0.5, 4, seed=9)
    idx = Index.build(w.Q, w.P, 12, lb_items=1800)
    pre = oracle.preprocess(w.Q, w.P, 12, 1800, 64)
    assert np.array_equal(idx.export(rkmips.RK_F_L64), pre["L"])
    for qi in w.qidx:
        assert np.array_equal(idx.reverse_kmips(w.P[qi], 5), oracle.brute(w.Q, w.P, w.P[qi], 5))
    idx.free()
