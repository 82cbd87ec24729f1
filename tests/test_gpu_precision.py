"""Precision forms (float32, and bfloat16 inputs with float32 accumulation):
the bulk products that the certified tests rely on stay within the rigorous
error bound the library uses, measured against f in float64 (the oracle) on a
d = 100 workload, and the fraction of users sent to the float64 recheck is
reported.  The measured figures are printed (pytest -s)."""
import numpy as np
import pytest

import oracle
from paper_2110_07131_amd import datagen
from paper_2110_07131_amd.rkmips import Index

pytestmark = pytest.mark.gpu


def gamma(k, u):
    return k * u / (1 - k * u)


def eps_bound(prec, d):
    # the library's certified relative bounds (float32 any order; bf16 inputs)
    slack = gamma(d, 2.0 ** -53) + 16 * 2.0 ** -24
    if prec == "fp32":
        return gamma(d + 2, 2.0 ** -24) + slack
    return (1 + 2.0 ** -8) ** 2 * (1 + gamma(d + 2, 2.0 ** -24)) - 1 + slack


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_bulk_error_within_certified_bound(prec):
    n, m, d = 200_000, 20_000, 100
    w = datagen.workload(n, m, d, 0.5, 10, seed=31)
    idx = Index.build(w.Q, w.P, 25, precision=prec)
    idx.set_counting(True)
    nu = np.linalg.norm(w.Q.astype(np.float64), axis=1)
    # theta_25 of every tenth user, from the oracle's exact table: a fixed
    # margin of 1e-3 |u||q| (instead of the certified bound) decides these
    # users' pairs, and its wrong and undecided decisions are counted
    th = np.full(n, np.nan)
    th[::10] = oracle.theta(w.Q[::10], w.P, 25)[:, 24]
    worst, pairs = 0.0, 0
    wrong, undecided, sampled = 0, 0, 0
    for q in w.queries:
        cls, shat = idx.trace(q, 25)
        users = np.nonzero(~np.isnan(shat))[0]
        if users.size == 0:  # every block pruned by Lemma 3
            continue
        s64 = oracle.pair_dots(w.Q, q[None, :], users, np.zeros(len(users), np.int64))
        nq = np.linalg.norm(q.astype(np.float64))
        sh = shat[users].astype(np.float64)
        rel = np.abs(sh - s64) / np.maximum(nu[users] * nq, 1e-300)
        worst = max(worst, float(rel.max()))
        pairs += len(users)
        t = users % 10 == 0
        tu, s64t, sht = th[users[t]], s64[t], sh[t]
        member = s64t >= tu
        mg = 1e-3 * nu[users[t]] * nq
        no, yes = sht + mg < tu, sht - mg >= tu
        wrong += int(np.count_nonzero(no & member) + np.count_nonzero(yes & ~member))
        undecided += int(np.count_nonzero(~no & ~yes))
        sampled += int(t.sum())
    st = idx.stats()
    borderline = st["rechecks"] / max(st["users_evaluated"], 1)
    bound = eps_bound(prec, d)
    print(f"\n[precision] {prec}: max |s^-f|/(|u||q|) = {worst:.3e} over {pairs} pairs; "
          f"certified bound {bound:.3e}; float64 rechecks {st['rechecks']} of "
          f"{st['users_evaluated']} evaluated users ({borderline:.2e}); a fixed 1e-3 margin "
          f"decides {wrong} of {sampled} sampled pairs wrongly and leaves {undecided} "
          f"({undecided / max(sampled, 1):.2e}) to float64")
    assert pairs > 500_000
    assert worst < bound
    idx.free()
