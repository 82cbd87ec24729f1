"""GPU test of rk_reverse_kmips_batch_dev_noalloc (the batch entry point that
allocates nothing, with the library's static per-GPU workspace), through the
C ABI: its CSR output must equal rk_reverse_kmips_batch_dev's element by
element, on two calls in a row, the second one smaller (and on another
index, so the static workspace is laid out differently and holds the first
call's contents)."""
import numpy as np
import pytest

import oracle
from paper_2110_07131_amd import datagen
from paper_2110_07131_amd.rkmips import RK_E_INVAL, RK_E_KMAX, Index, RkError

pytestmark = pytest.mark.gpu


def run(idx, qs_np, ks, noalloc, cap_per_query=512):
    import torch
    qs = torch.from_numpy(np.ascontiguousarray(qs_np)).cuda()
    off = torch.full((len(ks) + 1,), -7, dtype=torch.int64, device="cuda")
    ids = torch.full((max(1, len(ks) * cap_per_query),), -7, dtype=torch.int32, device="cuda")
    stream = torch.cuda.Stream()
    f = idx.reverse_kmips_batch_dev_noalloc if noalloc else idx.reverse_kmips_batch_dev
    f(qs, ks, off, ids, stream.cuda_stream)
    torch.cuda.synchronize()
    off_h = off.cpu().numpy()
    assert off_h[0] == 0 and off_h[-1] <= ids.numel()
    return off_h, ids[:int(off_h[-1])].cpu().numpy()


def case(n, m, d, nq, seed, prec):
    w = datagen.workload(n, m, d, 0.5, nq, seed=seed, k_choices="uniform", k_max=25)
    idx = Index.build(w.Q, w.P, 25, precision=prec)
    return w, idx


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_noalloc_equals_batch_dev_on_two_calls(prec):
    # call 1: 400,000 users (50 KB bitmap rows: the 2,500 queries run in
    # chunks of 1,250 to fit the static workspace); call 2: a smaller call
    # on another index (100,000 users, 700 queries, one chunk)
    w1, i1 = case(400_000, 20_000, 50, 2500, 81, prec)
    w2, i2 = case(100_000, 10_000, 64, 700, 82, prec)
    calls = [(w1, i1), (w2, i2)]
    got = [run(idx, w.queries, w.ks, True) for w, idx in calls]
    for (w, idx), (off, ids) in zip(calls, got):
        ref_off, ref_ids = run(idx, w.queries, w.ks, False)
        assert np.array_equal(off, ref_off)
        assert np.array_equal(ids, ref_ids)
        # and a few rows against the oracle on the whole catalog
        for i in (0, len(w.ks) // 2, len(w.ks) - 1):
            want = oracle.brute(w.Q, w.P, w.queries[i], int(w.ks[i]))
            assert np.array_equal(ids[off[i]:off[i + 1]], want), i
    # the first index again after the second: same output
    off, ids = run(i1, w1.queries, w1.ks, True)
    assert np.array_equal(off, got[0][0]) and np.array_equal(ids, got[0][1])
    i1.free()
    i2.free()


def test_noalloc_rejects_what_it_cannot_run():
    import torch
    w = datagen.workload(3000, 500, 16, 0.5, 10, seed=83)
    bounded = Index.build(w.Q, w.P, 8, lb_items=16)
    exact = Index.build(w.Q, w.P, 8)
    qs = torch.from_numpy(w.queries).cuda()
    off = torch.empty(len(w.qidx) + 1, dtype=torch.int64, device="cuda")
    ids = torch.empty(len(w.qidx) * 3000, dtype=torch.int32, device="cuda")
    with pytest.raises(RkError) as e:
        bounded.reverse_kmips_batch_dev_noalloc(qs, np.full(len(w.qidx), 3, np.int32), off, ids)
    assert e.value.status == RK_E_INVAL
    with pytest.raises(RkError) as e:
        exact.reverse_kmips_batch_dev_noalloc(qs, np.full(len(w.qidx), 9, np.int32), off, ids)
    assert e.value.status == RK_E_KMAX
    # k > m (every user) and an empty batch are fine
    ks = np.full(len(w.qidx), 501, np.int32)
    exact.reverse_kmips_batch_dev_noalloc(qs, ks, off, ids)
    torch.cuda.synchronize()
    assert np.array_equal(off.cpu().numpy(), np.arange(len(w.qidx) + 1) * 3000)
    exact.reverse_kmips_batch_dev_noalloc(qs[:0], ks[:0], off[:1], ids)
    torch.cuda.synchronize()
    assert int(off[0].item()) == 0
    bounded.free()
    exact.free()
