"""GPU tests of the serving runtime (rk_server_*): continuous batching over
several resident catalogs, admission by device-memory footprint, and result
sets equal to the float64 oracle per request, through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_2110_07131_amd import datagen
from paper_2110_07131_amd.rkmips import (RK_E_INVAL, RK_E_KMAX, RK_E_NOMEM, Index, RkError,
                                         Server)

pytestmark = pytest.mark.gpu

CATS = [  # n, m, d, k_max, sigma
    (3000, 800, 24, 8, 0.5),
    (1500, 300, 50, 10, 0.7),
    (700, 1200, 12, 6, 0.4),
]


def catalogs(lb=0, prec="fp32"):
    out = []
    for i, (n, m, d, kmax, sg) in enumerate(CATS):
        w = datagen.workload(n, m, d, sg, min(m, 60), seed=100 + i)
        idx = Index.build(w.Q, w.P, kmax, lb_items=min(lb, m) if lb else 0, precision=prec)
        out.append((w, kmax, idx))
    return out


def requests(cats, n_req, seed, only=None):
    rng = np.random.default_rng(seed)
    reqs = []
    for tag in range(n_req):
        c = int(rng.integers(len(cats))) if only is None else only
        w, kmax, _ = cats[c]
        if rng.random() < 0.7:
            q = w.P[int(rng.integers(len(w.P)))]
        else:
            q = datagen.vectors(1, w.P.shape[1], 0.6, rng)[0]
        reqs.append((tag, c, np.ascontiguousarray(q), int(rng.integers(1, kmax + 1))))
    return reqs


def serve(srv, cat_ids, reqs):
    for tag, c, q, k in reqs:
        srv.submit(cat_ids[c], q, k, tag)
    got = {}
    while len(got) < len(reqs):
        for tag, cat, status, ids, t0, t1 in srv.poll(wait_us=20000):
            assert tag not in got
            assert status == 0 and t1 >= t0
            got[tag] = (cat, ids)
    assert srv.inflight() == 0
    return got


def check(cats, cat_ids, reqs, got):
    for tag, c, q, k in reqs:
        cat, ids = got[tag]
        assert cat == cat_ids[c]
        w = cats[c][0]
        assert np.array_equal(ids, oracle.brute(w.Q, w.P, q, k)), (tag, c, k)


@pytest.mark.parametrize("lb,prec,wait", [(0, "fp32", 0), (0, "bf16", 0), (20, "fp32", 0),
                                          (0, "fp32", 3000)])
def test_server_results_equal_oracle(lb, prec, wait):
    cats = catalogs(lb, prec)
    srv = Server(max_batch=64, max_wait_us=wait)
    cat_ids = [srv.add(idx) for _, _, idx in cats]
    assert cat_ids == [0, 1, 2]
    reqs = requests(cats, 400, seed=7)
    got = serve(srv, cat_ids, reqs)
    check(cats, cat_ids, reqs, got)
    srv.close()
    for _, _, idx in cats:
        idx.free()


def test_alone_vs_mix():
    cats = catalogs()
    srv = Server(max_batch=32)
    cat_ids = [srv.add(idx) for _, _, idx in cats]
    alone = requests(cats, 120, seed=11, only=1)
    got_alone = serve(srv, cat_ids, alone)
    mixed = requests(cats, 300, seed=12)
    tagged = [(t + 1000, c, q, k) for t, c, q, k in mixed] + alone
    rng = np.random.default_rng(5)
    order = rng.permutation(len(tagged))
    got_mix = serve(srv, cat_ids, [tagged[i] for i in order])
    for tag, _, _, _ in alone:
        assert np.array_equal(got_alone[tag][1], got_mix[tag][1]), tag
    check(cats, cat_ids, alone, got_alone)
    check(cats, cat_ids, [(t + 1000, c, q, k) for t, c, q, k in mixed], got_mix)
    srv.close()


def test_admission_by_footprint():
    cats = catalogs()
    first = cats[0][2].stats()["footprint_bytes"]
    probe = Server(max_batch=16)
    probe.add(cats[0][2])
    need_first = probe.used_bytes()  # index + batch workspace + server buffers
    probe.close()
    assert need_first >= first
    # room for the first catalog, not for the second one's index alone
    second = cats[1][2].stats()["footprint_bytes"]
    srv = Server(max_batch=16, hbm_budget=need_first + second // 2)
    assert srv.add(cats[0][2]) == 0
    used = srv.used_bytes()
    assert used <= need_first
    with pytest.raises(RkError) as e:
        srv.add(cats[1][2])
    assert e.value.status == RK_E_NOMEM
    assert srv.used_bytes() == used
    # the admitted catalog still serves
    reqs = requests(cats, 30, seed=3, only=0)
    check(cats, [0, None, None], reqs, serve(srv, [0, None, None], reqs))
    srv.close()


def test_submit_validation():
    cats = catalogs()
    srv = Server(max_batch=8)
    srv.add(cats[0][2])
    w, kmax, _ = cats[0]
    q = w.P[0]
    for cat, qq, k, status in [(1, q, 1, RK_E_INVAL), (0, q, 0, RK_E_INVAL),
                               (0, q, kmax + 1, RK_E_KMAX),
                               (0, np.full_like(q, np.nan), 1, RK_E_INVAL)]:
        with pytest.raises(RkError) as e:
            srv.submit(cat, qq, k, 0)
        assert e.value.status == status
    assert srv.inflight() == 0
    srv.close()


def test_large_results_grow_buffers():
    # ~n k / m members per query: more ids than the initial buffers hold, and
    # single results larger than the binding's first poll buffer (65,536 ids)
    w = datagen.workload(120_000, 20, 8, 0.3, 20, seed=9)
    idx = Index.build(w.Q, w.P, 15)
    srv = Server(max_batch=16)
    srv.add(idx)
    reqs = [(t, 0, np.ascontiguousarray(w.P[t % 20]), 12 + t % 4) for t in range(40)]
    got = serve(srv, [0], reqs)
    sizes = [len(got[t][1]) for t in range(40)]
    assert max(sizes) > 65536
    check([(w, 15, idx)], [0], reqs, got)
    srv.close()
    idx.free()
