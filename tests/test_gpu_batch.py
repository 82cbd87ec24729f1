"""GPU parity of the batched path (many queries of mixed k per launch) against
the float64 CPU oracle, through the C ABI.  Every CSR row must equal the
oracle's result set exactly."""
import numpy as np
import pytest

import oracle
from paper_2110_07131_amd import datagen
from paper_2110_07131_amd.rkmips import Index

pytestmark = pytest.mark.gpu

MODES = [(0, "fp32"), (0, "bf16"), (20, "fp32"), (20, "bf16")]


def check_csr(w_Q, w_P, qs, ks, off, ids):
    assert off[0] == 0 and len(off) == len(ks) + 1
    assert np.all(np.diff(off) >= 0)
    for i in range(len(ks)):
        row = ids[off[i]:off[i + 1]]
        want = oracle.brute(w_Q, w_P, qs[i], int(ks[i]))
        assert np.array_equal(row, want), (i, int(ks[i]), row[:10], want[:10])


@pytest.mark.parametrize("lb,prec", MODES)
def test_batch_mixed_k_equals_oracle(lb, prec):
    w = datagen.config_workload("parity")
    rng = np.random.default_rng(3)
    qs = w.queries
    ks = rng.integers(1, 11, len(qs)).astype(np.int32)
    idx = Index.build(w.Q, w.P, 10, lb_items=lb, precision=prec)
    off, ids = idx.reverse_kmips_batch(qs, ks)
    check_csr(w.Q, w.P, qs, ks, off, ids)
    idx.free()


@pytest.mark.parametrize("lb,prec", MODES)
def test_small_batches_run_one_query_at_a_time(lb, prec):
    # batches of one and two queries take the one-query path (the batched
    # kernels' per-block cost does not pay for them); three take the
    # batched kernels: every row equals the oracle's, and the rows of the
    # same queries agree across the three forms
    w = datagen.config_workload("parity")
    rng = np.random.default_rng(9)
    qs = w.queries[:3]
    ks = rng.integers(1, 11, 3).astype(np.int32)
    idx = Index.build(w.Q, w.P, 10, lb_items=lb, precision=prec)
    idx.set_counting(True)
    rows = {}
    for nq in (1, 2, 3):
        before = idx.stats()["blocks_visited"]
        off, ids = idx.reverse_kmips_batch(qs[:nq], ks[:nq])
        check_csr(w.Q, w.P, qs[:nq], ks[:nq], off, ids)
        # the same Lemma 3 work either way: nq x (number of blocks)
        assert idx.stats()["blocks_visited"] - before == nq * idx.stats()["n_blocks"]
        for i in range(nq):
            rows.setdefault(i, []).append(ids[off[i]:off[i + 1]])
    for i, r in rows.items():
        assert all(np.array_equal(r[0], x) for x in r[1:]), i
    idx.free()


@pytest.mark.parametrize("lb,prec", MODES)
@pytest.mark.parametrize("n,m,d,kmax", [(130, 70, 3, 5), (65, 9, 7, 12), (1, 1, 2, 1), (200, 40, 160, 8)])
def test_batch_ragged_shapes_and_k_above_m(n, m, d, kmax, lb, prec):
    w = datagen.workload(n, m, d, 0.7, 12, seed=n * 7 + d)
    rng = np.random.default_rng(n)
    qs = np.vstack([w.queries, datagen.vectors(3, d, 0.7, rng) * 2])
    ks = rng.integers(1, kmax + 1, len(qs)).astype(np.int32)
    if m < kmax:
        ks[::3] = m + 1  # k > m: every user
    idx = Index.build(w.Q, w.P, kmax, lb_items=min(lb, m) if lb else 0, precision=prec)
    off, ids = idx.reverse_kmips_batch(qs, ks)
    check_csr(w.Q, w.P, qs, ks, off, ids)
    idx.free()


@pytest.mark.parametrize("lb,prec", [(0, "fp32"), (0, "bf16"), (20, "fp32")])
def test_batch_dense_results_over_several_assembly_rounds(lb, prec):
    # k close to m: most users are members, so bitmap words and lanes hold
    # many bits; 140,000 users take two rounds of the CSR assembly's loads
    # (16 groups of 64 lanes x 128 users each)
    w = datagen.workload(140_000, 40, 8, 0.5, 6, seed=11)
    ks = np.array([30, 25, 40, 20, 35, 39], np.int32)
    idx = Index.build(w.Q, w.P, 40, lb_items=lb, precision=prec)
    off, ids = idx.reverse_kmips_batch(w.queries, ks)
    assert off[-1] > 300_000  # dense rows
    check_csr(w.Q, w.P, w.queries, ks, off, ids)
    idx.free()


def test_batch_several_chunks():
    # more queries than one chunk (4096), small catalog
    w = datagen.workload(300, 150, 12, 0.6, 150, seed=12)
    rng = np.random.default_rng(12)
    pick = rng.integers(0, 150, 4500)
    qs = np.ascontiguousarray(w.P[pick])
    ks = rng.integers(1, 9, len(qs)).astype(np.int32)
    idx = Index.build(w.Q, w.P, 8)
    off, ids = idx.reverse_kmips_batch(qs, ks)
    # verify against the oracle on a sample, and exactly the CSR structure
    for i in list(range(0, 4500, 37)) + [4095, 4096, 4499]:
        assert np.array_equal(ids[off[i]:off[i + 1]], oracle.brute(w.Q, w.P, qs[i], int(ks[i]))), i
    idx.free()


@pytest.mark.parametrize("lb,prec", MODES)
@pytest.mark.parametrize("cap", [3, 100])
def test_pair_list_overflow_falls_back_to_float64(lb, prec, cap):
    # cap 3: the first reserved run of pair slots already crosses the end of
    # the list; cap 100: some runs fit, a later one crosses it
    w = datagen.workload(500, 200, 16, 0.5, 16, seed=4)
    rng = np.random.default_rng(4)
    ks = rng.integers(1, 9, len(w.qidx)).astype(np.int32)
    idx = Index.build(w.Q, w.P, 8, lb_items=lb, precision=prec, pair_cap=cap)
    off, ids = idx.reverse_kmips_batch(w.queries, ks)
    check_csr(w.Q, w.P, w.queries, ks, off, ids)
    idx.free()


def test_exact_pair_counter_beyond_int32():
    # margin_rel = 0.49 on nearly parallel and antiparallel vectors leaves
    # every (user, query) pair undecided (every block holds users of both
    # directions, so Lemma 3 prunes nothing): 4,096 queries x 540,000 users
    # reserve more than 2^31 pair slots in one query chunk.  The first ones
    # fit the list (float64 recheck), the filter decides the rest in float64
    # itself; the reserve counter must not wrap.
    rng = np.random.default_rng(90)
    n, m, d, nq = 540_000, 64, 4, 4096
    sign = np.where(rng.random(n) < 0.5, -1.0, 1.0)[:, None]
    Q = (sign * (1 + 0.01 * rng.standard_normal((n, d)))).astype(np.float32)
    P = (1 + 0.01 * rng.standard_normal((m, d))).astype(np.float32)
    qs = np.ascontiguousarray(P[rng.integers(0, m, nq)])
    ks = rng.integers(1, 3, nq).astype(np.int32)
    idx = Index.build(Q, P, 4, margin_rel=0.49)
    idx.set_counting(True)
    off, ids = idx.reverse_kmips_batch(qs, ks)
    st = idx.stats()
    assert st["blocks_pruned"] == 0 and st["lemma1_no"] == 0
    assert st["rechecks"] == nq * n > 2 ** 31
    # oracle on 3,000 users: the first and last norm-sorted blocks and a sample
    perm = oracle.sort_desc(oracle.sqnorms(Q))
    edge = np.concatenate([perm[:64], perm[(n - 1) // 64 * 64:]])
    us = np.union1d(edge, rng.choice(n, 3000 - edge.size, replace=False)).astype(np.int32)
    th = oracle.theta(np.ascontiguousarray(Q[us]), P, 4)
    assert off[0] == 0 and np.all(np.diff(off) >= 0)
    for i in range(nq):
        row = ids[off[i]:off[i + 1]]
        assert np.all(np.diff(row) > 0), i
        want = us[oracle.theta_query(th, np.ascontiguousarray(Q[us]), qs[i], int(ks[i]))]
        assert np.array_equal(row[np.isin(row, us, assume_unique=True)], want), i
    idx.free()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("bs", [64, 16])
def test_batch_query_tiles_split_over_workgroups(prec, bs):
    # 5,000 users (79 blocks, far fewer than the device's workgroup slots):
    # the exact table's filter splits each block's 32 query tiles over 8
    # workgroups of 4 tiles.  Every query is counted once per block, and
    # every result set equals the oracle's.
    rng = np.random.default_rng(123)
    w = datagen.workload(5000, 3000, 24, 0.6, 2000, seed=77)
    qs = np.vstack([w.queries, datagen.vectors(45, 24, 0.6, rng)])  # 2,045: a ragged last tile
    ks = rng.integers(1, 11, len(qs)).astype(np.int32)
    idx = Index.build(w.Q, w.P, 10, precision=prec, block_size=bs)
    idx.set_counting(True)
    off, ids = idx.reverse_kmips_batch(qs, ks)
    st = idx.stats()
    assert st["blocks_visited"] == len(ks) * st["n_blocks"]
    th = oracle.theta(w.Q, w.P, 10)
    assert off[0] == 0 and np.all(np.diff(off) >= 0)
    for i in range(len(ks)):
        want = oracle.theta_query(th, w.Q, qs[i], int(ks[i]))
        assert np.array_equal(ids[off[i]:off[i + 1]], want), i
    idx.free()


@pytest.mark.parametrize("lb,prec", MODES)
def test_batch_integer_ties(lb, prec):
    rng = np.random.default_rng(8)
    Q = datagen.small_int_vectors(260, 3, -3, 3, rng)
    P = datagen.small_int_vectors(70, 3, -3, 3, rng)
    Q[::13] = 0.0
    qs = np.ascontiguousarray(P[::3])
    ks = rng.integers(1, 7, len(qs)).astype(np.int32)
    idx = Index.build(Q, P, 6, lb_items=lb, precision=prec)
    off, ids = idx.reverse_kmips_batch(qs, ks)
    check_csr(Q, P, qs, ks, off, ids)
    idx.free()


def test_batch_counters_and_device_api():
    import torch
    w = datagen.config_workload("parity")
    ks = np.full(len(w.qidx), 3, np.int32)
    idx = Index.build(w.Q, w.P, 10)
    idx.set_counting(True)
    qs = torch.from_numpy(w.queries).cuda()
    off = torch.empty(len(ks) + 1, dtype=torch.int64, device="cuda")
    ids = torch.empty(len(ks) * 2000, dtype=torch.int32, device="cuda")
    idx.reverse_kmips_batch_dev(qs, ks, off, ids)
    torch.cuda.synchronize()
    off_h, ids_h = off.cpu().numpy(), ids.cpu().numpy()
    check_csr(w.Q, w.P, w.queries, ks, off_h, ids_h)
    st = idx.stats()
    assert st["blocks_visited"] == len(ks) * st["n_blocks"]
    assert st["users_evaluated"] + 0 >= st["lemma1_no"] + st["table_yes"]
    idx.free()


# --- grouped linear scan (bounded table) -----------------------------------

@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_grouped_scan_long_pass(prec):
    # m = 1000 items (16 tiles): members need scans well past the short pass
    w = datagen.config_workload("parity")
    rng = np.random.default_rng(21)
    qs = np.ascontiguousarray(np.vstack([w.queries, w.P[rng.integers(0, len(w.P), 40)]]))
    ks = rng.integers(1, 11, len(qs)).astype(np.int32)
    ks[:5] = 10
    idx = Index.build(w.Q, w.P, 10, lb_items=20, precision=prec)
    idx.set_counting(True)
    off, ids = idx.reverse_kmips_batch(qs, ks)
    check_csr(w.Q, w.P, qs, ks, off, ids)
    st = idx.stats()
    # the scan evaluated products beyond the 256 items of the short pass
    assert st["scan_items"] > 256 * 64
    assert st["results"] == off[-1]
    idx.free()


@pytest.mark.parametrize("cap", [256, 700, 256 * 30])
def test_grouped_scan_chunk_pool_partly_full(cap):
    # pairs beyond the chunk pool are decided in float64 by the filter; the
    # chunks that fit go through the grouped scan
    w = datagen.workload(700, 400, 16, 0.5, 30, seed=5)
    rng = np.random.default_rng(5)
    ks = rng.integers(1, 9, len(w.qidx)).astype(np.int32)
    idx = Index.build(w.Q, w.P, 8, lb_items=16, pair_cap=cap)
    off, ids = idx.reverse_kmips_batch(w.queries, ks)
    check_csr(w.Q, w.P, w.queries, ks, off, ids)
    idx.free()


def test_grouped_scan_several_chunks_bounded():
    # the per-block chunk lists are emptied between query chunks
    w = datagen.workload(300, 150, 12, 0.6, 150, seed=13)
    rng = np.random.default_rng(13)
    pick = rng.integers(0, 150, 4300)
    qs = np.ascontiguousarray(w.P[pick])
    ks = rng.integers(1, 9, len(qs)).astype(np.int32)
    idx = Index.build(w.Q, w.P, 8, lb_items=10)
    off, ids = idx.reverse_kmips_batch(qs, ks)
    for i in list(range(0, 4300, 41)) + [4095, 4096, 4299]:
        assert np.array_equal(ids[off[i]:off[i + 1]], oracle.brute(w.Q, w.P, qs[i], int(ks[i]))), i
    idx.free()


@pytest.mark.parametrize("m", [30, 256, 257])
def test_grouped_scan_short_catalog(m):
    # catalogs within or just past the short pass
    w = datagen.workload(400, m, 9, 0.8, 20, seed=m)
    rng = np.random.default_rng(m)
    qs = np.vstack([w.queries, datagen.vectors(5, 9, 0.8, rng)])
    ks = rng.integers(1, 7, len(qs)).astype(np.int32)
    idx = Index.build(w.Q, w.P, 6, lb_items=7)
    off, ids = idx.reverse_kmips_batch(qs, ks)
    check_csr(w.Q, w.P, qs, ks, off, ids)
    idx.free()


@pytest.mark.parametrize("nq", [10, 30])
def test_grouped_scan_many_flagged_pairs(nq):
    # Users along +x; 600 large items along -x (they never beat q, but their
    # norms put every pair's Corollary 1 limit past the short pass) and 20
    # small random items: every pair is flagged for the long pass, more than
    # the workgroup's list of flagged pairs holds when nq = 30 (64 x 30).
    rng = np.random.default_rng(40 + nq)
    Q = np.column_stack([1 + 0.1 * rng.random(64), 0.2 * rng.standard_normal(64)]).astype(np.float32)
    big = np.column_stack([-3 - rng.random(600), 0.3 * rng.standard_normal(600)])
    small = 0.6 * rng.standard_normal((20, 2))
    P = np.vstack([big, small]).astype(np.float32)
    qs = np.column_stack([0.4 + 0.2 * rng.random(nq), 0.1 * rng.standard_normal(nq)]).astype(np.float32)
    ks = rng.integers(1, 6, nq).astype(np.int32)
    idx = Index.build(Q, P, 5, lb_items=8)
    idx.set_counting(True)
    off, ids = idx.reverse_kmips_batch(qs, ks)
    check_csr(Q, P, qs, ks, off, ids)
    st = idx.stats()
    assert st["scan_long"] >= 64 * nq * 0.9
    idx.free()


def away_case(rng, n_users, n_away, n_rest, n_q, d=8):
    """Users along +x; the n_away largest items point away from them (never
    above q, but their norms put every Corollary 1 limit past the first pass
    over the item prefix), the other n_rest are random, and the queries are
    drawn from those: the long pass runs for every user."""
    Q = np.column_stack([1 + 0.2 * rng.random(n_users), 0.3 * rng.standard_normal((n_users, d - 1))])
    away = np.column_stack([-5 - rng.random(n_away), 0.2 * rng.standard_normal((n_away, d - 1))])
    rest = rng.standard_normal((n_rest, d))
    rest *= (1 + 2 * rng.random((n_rest, 1))) / np.linalg.norm(rest, axis=1, keepdims=True)
    P = np.vstack([away, rest]).astype(np.float32)
    qs = np.ascontiguousarray(P[rng.integers(n_away, n_away + n_rest, n_q)])
    ks = rng.integers(1, 9, n_q).astype(np.int32)
    return Q.astype(np.float32), P, qs, ks


def test_grouped_scan_lists_carried_across_chunks():
    # 4,400 queries (two query chunks) on the away-pointing catalog: the long
    # pass runs, and the second chunk starts from the first chunk's per-user
    # lists and scanned lengths
    w_Q, w_P, qs, ks = away_case(np.random.default_rng(14), 400, 900, 2100, 4400)
    idx = Index.build(w_Q, w_P, 8, lb_items=10)
    idx.set_counting(True)
    off, ids = idx.reverse_kmips_batch(qs, ks)
    st = idx.stats()
    assert st["scan_long"] > 0
    for i in list(range(0, 4400, 23)) + [4095, 4096, 4399]:
        assert np.array_equal(ids[off[i]:off[i + 1]], oracle.brute(w_Q, w_P, qs[i], int(ks[i]))), i
    # the same queries one chunk at a time give the same rows
    off2, ids2 = idx.reverse_kmips_batch(qs[4096:], ks[4096:])
    assert np.array_equal(off2, off[4096:] - off[4096])
    assert np.array_equal(ids2, ids[off[4096]:])
    idx.free()


def early_exit_case(rng):
    # Users along +x.  The 300 largest items point along -x (never above q,
    # but their norms put every limit past the short pass); the next 1,500
    # are large and random, so the flagged pairs of the small queries meet k
    # items above q within the first tiles of the long pass and stop there;
    # the large queries are members for most users, settled before the long
    # pass.
    d = 6
    Q = np.column_stack([1 + 0.2 * rng.random(128), 0.3 * rng.standard_normal((128, d - 1))])
    away = np.column_stack([-5 - rng.random(300), 0.2 * rng.standard_normal((300, d - 1))])
    mid = rng.standard_normal((1500, d))
    mid *= (3 + rng.random((1500, 1))) / np.linalg.norm(mid, axis=1, keepdims=True)
    small = 0.5 * rng.standard_normal((30, d))
    P = np.vstack([away, mid, small]).astype(np.float32)
    qs = np.column_stack([np.r_[0.5 + 0.3 * rng.random(40), 6.5 + 0.5 * rng.random(8)],
                          0.2 * rng.standard_normal((48, d - 1))]).astype(np.float32)
    ks = rng.integers(1, 7, len(qs)).astype(np.int32)
    return Q.astype(np.float32), P, qs, ks


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_grouped_scan_early_exit(prec):
    Q, P, qs, ks = early_exit_case(np.random.default_rng(60))
    idx = Index.build(Q, P, 6, lb_items=8, precision=prec)
    idx.set_counting(True)
    off, ids = idx.reverse_kmips_batch(qs, ks)
    check_csr(Q, P, qs, ks, off, ids)
    st = idx.stats()
    assert st["scan_long"] > 0
    # without the early exit every flagged user would scan nearly all of P
    assert st["scan_items"] < 0.4 * len(Q) * len(P)
    idx.free()


def handoff_case(rng, n_mid=40000):
    # 32 users along +x and 224 along +y, mixed in every block (similar
    # norms); 8 large items along +y (the lower-bound prefix: the y users'
    # pairs end at Lemma 1), 40,000 items of norm about 3 nearly orthogonal
    # to x and y, and 40 small ones.  Queries along +x beat almost every item
    # for the x users, whose scans run to the small items: each block has at
    # most 8 users scanning, with most of the catalog ahead.
    d = 16
    nx, ny = 32, 224
    Q = 0.05 * rng.standard_normal((nx + ny, d))
    Q[:nx, 0] += 1 + 0.1 * rng.random(nx)
    Q[nx:, 1] += 1 + 0.1 * rng.random(ny)
    Q = Q[rng.permutation(nx + ny)]
    top = 0.05 * rng.standard_normal((8, d))
    top[:, 1] += 5
    mid = rng.standard_normal((n_mid, d))
    mid[:, :2] *= 0.02
    mid *= (2.5 + rng.random((n_mid, 1))) / np.linalg.norm(mid, axis=1, keepdims=True)
    small = 0.3 * rng.standard_normal((40, d))
    P = np.vstack([top, mid, small]).astype(np.float32)
    qs = 0.05 * rng.standard_normal((20, d))
    qs[:, 0] += 0.9 + 0.2 * rng.random(20)
    ks = rng.integers(1, 9, 20).astype(np.int32)
    return Q.astype(np.float32), P, qs.astype(np.float32), ks


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_grouped_scan_handoff_to_group_passes(prec):
    # the last users of a block still scanning with most of a 625-tile
    # catalog ahead are handed to group passes of users from several blocks,
    # and their pairs decided from the final lists
    Q, P, qs, ks = handoff_case(np.random.default_rng(21))
    idx = Index.build(Q, P, 8, lb_items=8, precision=prec)
    idx.set_counting(True)
    off, ids = idx.reverse_kmips_batch(qs, ks)
    st = idx.stats()
    check_csr(Q, P, qs, ks, off, ids)
    assert st["scan_handoff"] > 0
    # every scanned (user, item) product comes from an MFMA quarter (32 x 32)
    # or a vector-ALU tile (at most 8 users x 64 items)
    assert st["scan_quarters"] > 0
    assert st["scan_items"] <= 1024 * st["scan_quarters"] + 512 * st["scan_valu_tiles"]
    idx.free()


def test_grouped_scan_handoff_with_lists_carried_across_chunks():
    # 4,200 queries (two query chunks) on the hand-off catalog: users handed
    # to group passes in the first chunk start the second from the lists and
    # coverage the group passes stored
    Q, P, qs0, _ = handoff_case(np.random.default_rng(22))
    rng = np.random.default_rng(23)
    qs = np.ascontiguousarray(qs0[rng.integers(0, len(qs0), 4200)] +
                              0.01 * rng.standard_normal((4200, qs0.shape[1])).astype(np.float32))
    ks = rng.integers(1, 9, 4200).astype(np.int32)
    idx = Index.build(Q, P, 8, lb_items=8)
    idx.set_counting(True)
    off, ids = idx.reverse_kmips_batch(qs, ks)
    st = idx.stats()
    assert st["scan_handoff"] > 0
    for i in list(range(0, 4200, 97)) + [4095, 4096, 4199]:
        assert np.array_equal(ids[off[i]:off[i + 1]], oracle.brute(Q, P, qs[i], int(ks[i]))), i
    idx.free()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_grouped_scan_handoff_on_short_catalogs(prec):
    # handoff_tiles = 1: blocks hand over their last users (and group passes
    # theirs, to the second pass) with any tile left, on a random workload
    w = datagen.workload(900, 2500, 12, 0.7, 60, seed=31)
    rng = np.random.default_rng(31)
    ks = rng.integers(1, 9, len(w.qidx)).astype(np.int32)
    idx = Index.build(w.Q, w.P, 8, lb_items=10, precision=prec, handoff_tiles=1)
    idx.set_counting(True)
    off, ids = idx.reverse_kmips_batch(w.queries, ks)
    st = idx.stats()
    check_csr(w.Q, w.P, w.queries, ks, off, ids)
    assert st["scan_handoff"] > 0
    idx.free()


def test_grouped_scan_handoff_on_short_catalogs_several_chunks():
    # 4,300 queries (two chunks) on the hand-off catalog cut to 2,048 items
    # (32 tiles), handoff_tiles = 1
    Q, P, qs0, _ = handoff_case(np.random.default_rng(32), n_mid=2000)
    rng = np.random.default_rng(33)
    qs = np.ascontiguousarray(qs0[rng.integers(0, len(qs0), 4300)] +
                              0.01 * rng.standard_normal((4300, qs0.shape[1])).astype(np.float32))
    ks = rng.integers(1, 9, 4300).astype(np.int32)
    idx = Index.build(Q, P, 8, lb_items=8, handoff_tiles=1)
    idx.set_counting(True)
    off, ids = idx.reverse_kmips_batch(qs, ks)
    assert idx.stats()["scan_handoff"] > 0
    for i in list(range(0, 4300, 29)) + [4095, 4096, 4299]:
        assert np.array_equal(ids[off[i]:off[i + 1]], oracle.brute(Q, P, qs[i], int(ks[i]))), i
    idx.free()


@pytest.mark.parametrize("d,prec,handoff", [(100, "fp32", 0), (99, "fp32", 1), (100, "bf16", 1),
                                              (66, "fp32", 1)])
def test_grouped_scan_shared_tile_region(d, prec, handoff):
    # 65 <= d <= 128: the scan's candidates and pair slots share the item
    # tile's region (odd d: its zero row is restored after every tile)
    w = datagen.workload(700, 1500, d, 0.6, 40, seed=d)
    rng = np.random.default_rng(d)
    ks = rng.integers(1, 9, len(w.qidx)).astype(np.int32)
    idx = Index.build(w.Q, w.P, 8, lb_items=10, precision=prec, handoff_tiles=handoff)
    idx.set_counting(True)
    off, ids = idx.reverse_kmips_batch(w.queries, ks)
    check_csr(w.Q, w.P, w.queries, ks, off, ids)
    assert idx.stats()["scan_long"] > 0
    idx.free()


@pytest.mark.parametrize("d", [200, 255])
def test_grouped_scan_shared_region_wide_tiles(d):
    # k_max = 50 at d = 200 or 255: separate candidate buffers would not fit
    # the CU's LDS (the batch would go one query at a time); with the shared
    # region the grouped scan runs
    w = datagen.workload(500, 1200, d, 0.8, 30, seed=d)
    rng = np.random.default_rng(d)
    ks = rng.integers(1, 51, len(w.qidx)).astype(np.int32)
    idx = Index.build(w.Q, w.P, 50, lb_items=60, handoff_tiles=1)
    idx.set_counting(True)
    off, ids = idx.reverse_kmips_batch(w.queries, ks)
    check_csr(w.Q, w.P, w.queries, ks, off, ids)
    assert idx.stats()["scan_long"] > 0
    idx.free()


# --- limits: largest k_max, widest d ----------------------------------------

@pytest.mark.parametrize("lb,prec", [(0, "fp32"), (130, "fp32"), (130, "bf16")])
def test_batch_kmax_128(lb, prec):
    # k_max = 128 (the limit): the scan's per-user lists exceed one wave
    w = datagen.workload(700, 400, 20, 0.6, 40, seed=77)
    rng = np.random.default_rng(77)
    ks = rng.integers(1, 129, len(w.qidx)).astype(np.int32)
    ks[:4] = 128
    idx = Index.build(w.Q, w.P, 128, lb_items=lb, precision=prec)
    off, ids = idx.reverse_kmips_batch(w.queries, ks)
    check_csr(w.Q, w.P, w.queries, ks, off, ids)
    idx.free()


@pytest.mark.parametrize("d,lb", [(512, 0), (512, 16), (257, 0), (257, 16)])
def test_batch_widest_dimensions(d, lb):
    # d = 512 (the limit) and an odd d: tiles too wide for the batched filter
    # go through the one-query path inside the batch call
    w = datagen.workload(300, 150, d, 0.5, 12, seed=d)
    rng = np.random.default_rng(d)
    ks = rng.integers(1, 9, len(w.qidx)).astype(np.int32)
    idx = Index.build(w.Q, w.P, 8, lb_items=lb)
    off, ids = idx.reverse_kmips_batch(w.queries, ks)
    check_csr(w.Q, w.P, w.queries, ks, off, ids)
    for qi, k in zip(w.qidx[:4], ks[:4]):
        assert np.array_equal(idx.reverse_kmips(w.P[qi], int(k)), oracle.brute(w.Q, w.P, w.P[qi], int(k)))
    idx.free()
