"""Pins of the oracle's inner stopping rule (Sec. 5.1: a local solve stops once
|p^(k+1) - p^(k)|_2 / |p^(k+1)|_2 falls below a tolerance).

The reference for the rule is computed outside the oracle: fixed-count runs of
k - 1 and k local steps are exported, the relative change of each subdomain's
block of p is taken with numpy, and the first k below the tolerance must be
the count the adaptive run reports, with the adaptive state equal to the k-step
state."""
import numpy as np
import pytest

import oracle

RC, CC = [0, 5, 12, 20], [0, 9, 17]


def make(f, **kw):
    return oracle.Oracle(oracle.Problem(np.asarray(f, dtype=np.float64), 6.0, np.asarray(RC), np.asarray(CC), **kw))


def sub_blocks(o, p):
    """Slices of the concatenated p per subdomain (row-major)."""
    out, off = [], 0
    for r, c, ra, rb, ca, cb in o.subdomains():
        h, w = rb - ra, cb - ca
        n = (h + 1) * w + h * (w + 1)
        out.append(p[off:off + n])
        off += n
    return out


def fixed_state(f, k):
    o = make(f, n_inner=k)
    o.run(1)
    return o, o.export()


@pytest.mark.parametrize("tol", [3e-2, 1e-2, 2e-3])
def test_first_outer_step_count_matches_relative_change(tol):
    rng = np.random.default_rng(5)
    f = rng.uniform(size=(20, 17))
    cap = 60
    a = make(f, n_inner=cap, inner_tol=tol)
    a.run(1)
    counts = a.inner_counts()
    assert a.inner_margin() > 1e-6
    # per subdomain, the first k with |p_k - p_{k-1}| < tol |p_k| (fixed-count runs)
    prev = None
    expect = [None] * len(counts)
    states = {}
    for k in range(1, cap + 1):
        o, e = fixed_state(f, k)
        blocks = sub_blocks(o, e["p"])
        states[k] = blocks
        if prev is not None:
            for s, (bk, bp) in enumerate(zip(blocks, prev)):
                if expect[s] is None and np.linalg.norm(bk - bp) < tol * np.linalg.norm(bk):
                    expect[s] = k
        prev = blocks
        if all(x is not None for x in expect):
            break
    expect = [cap if x is None else x for x in expect]
    assert list(counts[:, 0]) == expect and list(counts[:, 1]) == expect
    got = sub_blocks(a, a.export()["p"])
    for s, k in enumerate(expect):
        assert np.array_equal(got[s], states[k][s]), s


def test_huge_tolerance_takes_one_step():
    rng = np.random.default_rng(6)
    f = rng.uniform(size=(20, 17))
    a = make(f, n_inner=9, inner_tol=1e30)
    b = make(f, n_inner=1)
    a.run(4)
    b.run(4)
    assert np.array_equal(a.export()["p"], b.export()["p"])
    assert np.all(a.inner_counts() == [4, 1])


def test_tiny_tolerance_is_the_fixed_count():
    rng = np.random.default_rng(7)
    f = rng.uniform(size=(20, 17))
    a = make(f, n_inner=12, inner_tol=1e-300)
    b = make(f, n_inner=12)
    a.run(5)
    b.run(5)
    assert np.array_equal(a.export()["p"], b.export()["p"])
    assert np.all(a.inner_counts() == [60, 12])


def test_constant_image_stops_at_the_fixed_point():
    """One subdomain and constant f: p = 0 is the solution and the first step
    changes nothing, so every local solve stops after one step.  (On a
    decomposed grid the one-sided differences at the interfaces move p off 0.)"""
    f = np.full((20, 17), 0.3)
    a = oracle.Oracle(oracle.Problem(f, 6.0, np.array([0, 20]), np.array([0, 17]), n_inner=30, inner_tol=1e-6))
    a.run(3)
    assert np.all(a.inner_counts() == [3, 1])
    assert not a.export()["p"].any()


def test_counts_accumulate_over_outer_steps():
    rng = np.random.default_rng(8)
    f = rng.uniform(size=(20, 17))
    a = make(f, n_inner=40, inner_tol=1e-3)
    tot = np.zeros(6, dtype=np.int64)
    mx = np.zeros(6, dtype=np.int64)
    for n in range(5):
        before = a.inner_counts()[:, 0].copy()
        a.run(1)
        step = a.inner_counts()[:, 0] - before
        assert np.all((step >= 1) & (step <= 40))
        tot += step
        mx = np.maximum(mx, step)
    assert np.array_equal(a.inner_counts()[:, 0], tot)
    assert np.array_equal(a.inner_counts()[:, 1], mx)
