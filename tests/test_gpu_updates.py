"""GPU parity of catalog updates (Section 4.1: adding items keeps every lower
bound valid; adding users needs their rows and new blocks), through the C
ABI.  An exact table after rk_index_add_items, and any index after
rk_index_add_users, must equal an index built from scratch on the grown
catalog field by field; a bounded table keeps rows that stay below the
grown catalog's exact k-th values (oracle).  Every result set after the
updates equals the float64 oracle's on the grown catalog."""
import numpy as np
import pytest

import oracle
from paper_2110_07131_amd import datagen, rkmips
from paper_2110_07131_amd.rkmips import Index, RkError

pytestmark = pytest.mark.gpu

FIELDS = [rkmips.RK_F_PERM_Q, rkmips.RK_F_PERM_P, rkmips.RK_F_SQNORM_Q, rkmips.RK_F_SQNORM_P,
          rkmips.RK_F_NORM_Q, rkmips.RK_F_NORM_P, rkmips.RK_F_L64, rkmips.RK_F_L32, rkmips.RK_F_LB,
          rkmips.RK_F_BNORM]


def same_index(a, b, fields=FIELDS):
    for f in fields:
        x, y = a.export(f), b.export(f)
        assert x.shape == y.shape, f
        assert np.array_equal(x, y), f


def check_results(idx, Q, P, qs, ks):
    off, ids = idx.reverse_kmips_batch(qs, ks)
    kmax = int(ks.max())
    th = oracle.theta(Q, P, kmax)
    for i in range(len(ks)):
        if ks[i] > P.shape[0]:
            want = np.arange(Q.shape[0], dtype=np.int32)
        else:
            want = oracle.theta_query(th, Q, qs[i], int(ks[i]))
        assert np.array_equal(ids[off[i]:off[i + 1]], want), ("batch", i)
    for i in range(0, len(ks), 7):
        assert np.array_equal(idx.reverse_kmips(qs[i], int(ks[i])), ids[off[i]:off[i + 1]]), ("one", i)


def split(n_old, n_new, m_old, m_new, d, seed):
    w = datagen.workload(n_old + n_new, m_old + m_new, d, 0.6, 40, seed=seed)
    return w.Q[:n_old], w.Q[n_old:], w.P[:m_old], w.P[m_old:], w


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_add_items_exact_table_equals_fresh_build(prec):
    Q, _, P0, P1, w = split(3000, 0, 900, 333, 20, seed=61)
    P = np.vstack([P0, P1])
    idx = Index.build(Q, P0, 10, precision=prec)
    idx.add_items(P1)
    ref = Index.build(Q, P, 10, precision=prec)
    same_index(idx, ref)
    st = idx.stats()
    assert (st["m"], st["lb_items"], st["updates"]) == (P.shape[0], P.shape[0], 1)
    rng = np.random.default_rng(1)
    qs = np.vstack([P1[:30], P0[:10], datagen.vectors(10, 20, 0.6, rng)])
    ks = rng.integers(1, 11, len(qs)).astype(np.int32)
    check_results(idx, Q, P, qs, ks)
    idx.free()
    ref.free()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_add_items_bounded_table_keeps_valid_bounds(prec):
    Q, _, P0, P1, w = split(2500, 0, 700, 500, 16, seed=62)
    # the new items include the largest norms: the sorted prefix changes
    P1 = P1 * 1.7
    P = np.vstack([P0, P1])
    idx = Index.build(Q, P0, 8, lb_items=20, precision=prec)
    L_before = idx.export(rkmips.RK_F_L64)
    perm_before = idx.export(rkmips.RK_F_PERM_Q)
    idx.add_items(P1)
    # the rows are kept (same users, same order) and stay below the grown
    # catalog's exact k-th values
    assert np.array_equal(idx.export(rkmips.RK_F_PERM_Q), perm_before)
    L = idx.export(rkmips.RK_F_L64)
    assert np.array_equal(L, L_before)
    th = oracle.theta(Q, P, 8)  # original user order
    assert np.all(L <= th[perm_before].T)
    same_index(idx, Index.build(Q, P, 8, lb_items=20, precision=prec),
               [rkmips.RK_F_PERM_P, rkmips.RK_F_SQNORM_P, rkmips.RK_F_NORM_P])
    rng = np.random.default_rng(2)
    qs = np.vstack([P1[:25], P0[:15]])
    ks = rng.integers(1, 9, len(qs)).astype(np.int32)
    check_results(idx, Q, P, qs, ks)
    idx.free()


@pytest.mark.parametrize("lb,prec", [(0, "fp32"), (0, "bf16"), (20, "fp32"), (1100, "fp32")])
@pytest.mark.parametrize("bs", [64, 16])
def test_add_users_equals_fresh_build(lb, prec, bs):
    # lb = 1100 (> 1,024 items of the float64 seed): the candidate build path
    Q0, Q1, P, _, w = split(2100, 777, 1500, 0, 12, seed=63 + lb)
    Q = np.vstack([Q0, Q1])
    idx = Index.build(Q0, P, 9, lb_items=lb, precision=prec, block_size=bs)
    idx.add_users(Q1)
    ref = Index.build(Q, P, 9, lb_items=lb, precision=prec, block_size=bs)
    same_index(idx, ref)
    st = idx.stats()
    assert (st["n"], st["n_blocks"]) == (Q.shape[0], ref.stats()["n_blocks"])
    rng = np.random.default_rng(3)
    qs = np.ascontiguousarray(P[rng.integers(0, P.shape[0], 35)])
    ks = rng.integers(1, 10, len(qs)).astype(np.int32)
    check_results(idx, Q, P, qs, ks)
    idx.free()
    ref.free()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_updates_in_sequence_from_tiny_catalogs(prec):
    # from 40 users and 4 items (k_max = 6 > m: the table's lower rows are
    # empty, every k > m query returns every user) to 2,540 users x 904 items
    rng = np.random.default_rng(64)
    d = 10
    Q = datagen.vectors(40, d, 0.5, rng)
    P = datagen.vectors(4, d, 0.5, rng)
    idx = Index.build(Q, P, 6, precision=prec)
    for step in range(3):
        P_new = datagen.vectors(300, d, 0.5, rng)
        Q_new = datagen.vectors(833, d, 0.5, rng)
        idx.add_items(P_new)
        P = np.vstack([P, P_new])
        idx.add_users(Q_new)
        Q = np.vstack([Q, Q_new])
        qs = np.vstack([P_new[:12], datagen.vectors(8, d, 0.5, rng)])
        ks = rng.integers(1, 7, len(qs)).astype(np.int32)
        check_results(idx, Q, P, qs, ks)
    same_index(idx, Index.build(Q, P, 6, precision=prec))
    assert idx.stats()["updates"] == 6
    idx.free()


def test_updates_of_empty_catalogs_and_errors():
    rng = np.random.default_rng(65)
    d = 7
    Q = datagen.vectors(300, d, 0.5, rng)
    P = datagen.vectors(200, d, 0.5, rng)
    idx = Index.build(np.zeros((0, d), np.float32), np.zeros((0, d), np.float32), 5)
    idx.add_items(P)
    idx.add_users(Q)
    same_index(idx, Index.build(Q, P, 5))
    qs = np.ascontiguousarray(P[:20])
    ks = rng.integers(1, 6, len(qs)).astype(np.int32)
    check_results(idx, Q, P, qs, ks)
    idx.add_items(np.zeros((0, d), np.float32))  # no-op
    bad = P[:3].copy()
    bad[1, 2] = np.nan
    with pytest.raises(RkError):
        idx.add_items(bad)
    with pytest.raises(RkError):
        idx.add_users(bad)
    assert idx.stats()["m"] == 200 and idx.stats()["n"] == 300  # unchanged by the rejected calls
    assert rkmips.lib().rk_index_add_items(idx._h, None, 5) == rkmips.RK_E_INVAL
    assert rkmips.lib().rk_index_add_users(idx._h, None, -1) == rkmips.RK_E_INVAL
    check_results(idx, Q, P, qs, ks)
    idx.free()


def test_update_of_a_served_index_is_refused():
    rng = np.random.default_rng(66)
    Q = datagen.vectors(500, 8, 0.5, rng)
    P = datagen.vectors(100, 8, 0.5, rng)
    idx = Index.build(Q, P, 4)
    srv = rkmips.Server(max_batch=64)
    srv.add(idx)
    with pytest.raises(RkError):
        idx.add_items(P[:5])
    with pytest.raises(RkError):
        idx.rebuild(6)
    srv.close()
    idx.add_items(P[:5])  # the server is gone
    assert idx.stats()["m"] == 105
    idx.free()


def test_device_entry_points_after_updates():
    # the device batch calls (own workspace, and the static one of the entry
    # point that allocates nothing) size their work by the grown catalog
    import torch
    rng = np.random.default_rng(67)
    d = 16
    Q = datagen.vectors(1500, d, 0.5, rng)
    P = datagen.vectors(400, d, 0.5, rng)
    idx = Index.build(Q, P, 8)
    Q1, P1 = datagen.vectors(2600, d, 0.5, rng), datagen.vectors(350, d, 0.5, rng)
    idx.add_users(Q1)
    idx.add_items(P1)
    Q, P = np.vstack([Q, Q1]), np.vstack([P, P1])
    qs_np = np.vstack([P1[:40], datagen.vectors(24, d, 0.5, rng)])
    ks = rng.integers(1, 9, len(qs_np)).astype(np.int32)
    th = oracle.theta(Q, P, 8)
    qs = torch.from_numpy(np.ascontiguousarray(qs_np)).cuda()
    stream = torch.cuda.Stream()
    outs = []
    for f in (idx.reverse_kmips_batch_dev, idx.reverse_kmips_batch_dev_noalloc):
        off = torch.empty(len(ks) + 1, dtype=torch.int64, device="cuda")
        ids = torch.empty(len(ks) * Q.shape[0], dtype=torch.int32, device="cuda")
        f(qs, ks, off, ids, stream.cuda_stream)
        torch.cuda.synchronize()
        off_h = off.cpu().numpy()
        outs.append((off_h, ids[:int(off_h[-1])].cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    off_h, ids_h = outs[0]
    for i in range(len(ks)):
        want = oracle.theta_query(th, Q, qs_np[i], int(ks[i]))
        assert np.array_equal(ids_h[off_h[i]:off_h[i + 1]], want), i
    idx.free()
