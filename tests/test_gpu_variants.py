"""GPU parity of the index variants (the paper's Section 5.2 ablation and the
free constants of Definition 5): Lemma 3 blocks of 16, 32 or 64 users, and no
blocks at all ("Simpfer without blocks").  Result sets do not depend on the
variant: every one must equal the float64 oracle exactly, through the
one-query and the batched entry points; the block minima must equal the
oracle's Equation (1) over blocks of that size."""
import numpy as np
import pytest

import oracle
from paper_2110_07131_amd import datagen, rkmips
from paper_2110_07131_amd.rkmips import Index

pytestmark = pytest.mark.gpu

VARIANTS = [dict(block_size=16), dict(block_size=32), dict(block_size=64), dict(no_blocks=True),
            dict(block_size=16, no_blocks=True)]
TABLES = [(0, "fp32"), (0, "bf16"), (20, "fp32"), (20, "bf16")]


def f32_down(x64):
    f = x64.astype(np.float32)
    over = f.astype(np.float64) > x64
    f[over] = np.nextafter(f[over], np.float32(-np.inf))
    return f


@pytest.fixture(scope="module")
def wl():
    # 2,000 users (31 full tiles of 64 and one of 16: blocks of 16 and 32
    # are partial or empty at the end), 1,000 items
    return datagen.workload(2000, 1000, 50, 0.5, 24, seed=41)


@pytest.mark.parametrize("b", [16, 32])
def test_block_minima_of_smaller_blocks(wl, b):
    idx = Index.build(wl.Q, wl.P, 10, block_size=b)
    pre = oracle.preprocess(wl.Q, wl.P, 10, wl.P.shape[0], b)
    nB = -(-2000 // 64) * 64 // b   # blocks over the padded user range
    LB = idx.export(rkmips.RK_F_LB)
    assert LB.shape == (10, nB)
    real = pre["LB"].shape[1]       # blocks holding real users
    assert np.array_equal(LB[:, :real], f32_down(pre["LB"]))
    assert np.all(np.isinf(LB[:, real:]))
    nQ = idx.export(rkmips.RK_F_NORM_Q)
    assert np.array_equal(idx.export(rkmips.RK_F_BNORM)[:real], nQ[::b])
    st = idx.stats()
    assert (st["block_size"], st["n_blocks"]) == (b, nB)
    idx.free()


@pytest.mark.parametrize("lb,prec", TABLES)
@pytest.mark.parametrize("var", VARIANTS, ids=lambda v: "-".join(f"{k}{v[k]}" for k in v))
def test_variant_results_equal_oracle(wl, var, lb, prec):
    rng = np.random.default_rng(42)
    qs = wl.queries
    ks = rng.integers(1, 11, len(qs)).astype(np.int32)
    idx = Index.build(wl.Q, wl.P, 10, lb_items=lb, precision=prec, **var)
    idx.set_counting(True)
    off, ids = idx.reverse_kmips_batch(qs, ks)
    for i in range(len(ks)):
        want = oracle.brute(wl.Q, wl.P, qs[i], int(ks[i]))
        assert np.array_equal(ids[off[i]:off[i + 1]], want), ("batch", i)
    st = idx.stats()
    assert st["blocks_visited"] == len(ks) * st["n_blocks"]
    if var.get("no_blocks"):
        assert st["blocks_pruned"] == 0
    for i in range(0, len(ks), 5):
        assert np.array_equal(idx.reverse_kmips(qs[i], int(ks[i])),
                              oracle.brute(wl.Q, wl.P, qs[i], int(ks[i]))), ("one", i)
    idx.free()


def test_smaller_blocks_prune_at_least_as_much(wl):
    # a block of 16 users is a subset of its block of 64: its minimum lower
    # bound is at least as large and its first norm at most as large, so
    # every pair Lemma 3 prunes with 64-user blocks it also prunes with 16
    qs = wl.queries
    ks = np.full(len(qs), 5, np.int32)
    evaluated = {}
    for var in (dict(block_size=64), dict(block_size=32), dict(block_size=16), dict(no_blocks=True)):
        idx = Index.build(wl.Q, wl.P, 10, **var)
        idx.set_counting(True)
        idx.reverse_kmips_batch(qs, ks)
        evaluated[str(var)] = idx.stats()["users_evaluated"]
        idx.free()
    e = list(evaluated.values())
    assert e[2] <= e[1] <= e[0] <= e[3], evaluated
    assert e[3] == len(ks) * 2000
