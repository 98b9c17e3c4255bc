"""Pins of the oracle's inner stopping rule (Sec. 5.1: a local solve stops once
|p^(k+1) - p^(k)|_2 / |p^(k+1)|_2 falls below a tolerance), for the local
FISTA solver (ROF) and for the local accelerated primal-dual solver (TV-L1 with
an inpainting mask, convex Chan-Vese), whose state then also holds u^(k).

The reference for the rule is computed outside the oracle: fixed-count runs of
k - 1 and k local steps are exported, the relative change of each subdomain's
block of p is taken with numpy, and the first k below the tolerance must be
the count the adaptive run reports, with the adaptive state equal to the k-step
state."""
import numpy as np
import pytest

import oracle

RC, CC = [0, 5, 12, 20], [0, 9, 17]
_MASK = (np.random.default_rng(50).uniform(size=(20, 17)) > 0.15).astype(np.uint8)
SOLVERS = {
    "fista": dict(),
    "cp2_l1_mask": dict(inner="CP2", fidelity="L1", mask=_MASK, gamma=1.0 / 400.0),
    "cp2_cv": dict(inner="CP2", fidelity="CV", tau=1.0, sigma=0.5, gamma=1.0 / 8.0),
}
ALPHA = {"fista": 6.0, "cp2_l1_mask": 1.5, "cp2_cv": 10.0}


def make(f, solver="fista", **kw):
    args = dict(SOLVERS[solver])
    args.update(kw)
    return oracle.Oracle(oracle.Problem(np.asarray(f, dtype=np.float64), ALPHA[solver], np.asarray(RC),
                                        np.asarray(CC), **args))


def sub_blocks(o, p):
    """Slices of the concatenated p per subdomain (row-major)."""
    out, off = [], 0
    for r, c, ra, rb, ca, cb in o.subdomains():
        h, w = rb - ra, cb - ca
        n = (h + 1) * w + h * (w + 1)
        out.append(p[off:off + n])
        off += n
    return out


def fixed_state(f, k, solver="fista"):
    o = make(f, solver, n_inner=k)
    o.run(1)
    return o, o.export()


def _uprime(e, o):
    """u of every subdomain's pixels, in the subdomain order of sub_blocks."""
    return [e["u"][ra:rb, ca:cb] for r, c, ra, rb, ca, cb in o.subdomains()]


@pytest.mark.parametrize("solver,tol", [(s, t) for s in SOLVERS for t in (3e-2, 1e-2, 2e-3)
                                        if not (s == "cp2_l1_mask" and t == 2e-3)] + [("cp2_l1_mask", 5e-3)])
def test_first_outer_step_count_matches_relative_change(tol, solver):
    rng = np.random.default_rng(5)
    f = rng.uniform(size=(20, 17))
    cap = 60
    a = make(f, solver, n_inner=cap, inner_tol=tol)
    a.run(1)
    counts = a.inner_counts()
    assert a.inner_margin() > 1e-6
    # per subdomain, the first k with |p_k - p_{k-1}| < tol |p_k| (fixed-count runs)
    prev = None
    expect = [None] * len(counts)
    states = {}
    for k in range(1, cap + 1):
        o, e = fixed_state(f, k, solver)
        blocks = sub_blocks(o, e["p"])
        states[k] = (blocks, _uprime(e, o))
        if prev is not None:
            for s, (bk, bp) in enumerate(zip(blocks, prev)):
                if expect[s] is None and np.linalg.norm(bk - bp) < tol * np.linalg.norm(bk):
                    expect[s] = k
        prev = blocks
        if all(x is not None for x in expect):
            break
    expect = [cap if x is None else x for x in expect]
    assert list(counts[:, 0]) == expect and list(counts[:, 1]) == expect
    assert len(set(expect)) > 1          # the subdomains stop at different steps
    ea = a.export()
    got, gotu = sub_blocks(a, ea["p"]), _uprime(ea, a)
    for s, k in enumerate(expect):
        assert np.array_equal(got[s], states[k][0][s]), s
        assert np.array_equal(gotu[s], states[k][1][s]), s    # u^(k) with p^(k) (CP2: u is state)


@pytest.mark.parametrize("solver", list(SOLVERS))
def test_huge_tolerance_takes_one_step(solver):
    rng = np.random.default_rng(6)
    f = rng.uniform(size=(20, 17))
    a = make(f, solver, n_inner=9, inner_tol=1e30)
    b = make(f, solver, n_inner=1)
    a.run(4)
    b.run(4)
    assert np.array_equal(a.export()["p"], b.export()["p"])
    assert np.array_equal(a.export()["u"], b.export()["u"])
    assert np.all(a.inner_counts() == [4, 1])


@pytest.mark.parametrize("solver", list(SOLVERS))
def test_tiny_tolerance_is_the_fixed_count(solver):
    rng = np.random.default_rng(7)
    f = rng.uniform(size=(20, 17))
    a = make(f, solver, n_inner=12, inner_tol=1e-300)
    b = make(f, solver, n_inner=12)
    a.run(5)
    b.run(5)
    assert np.array_equal(a.export()["p"], b.export()["p"])
    assert np.array_equal(a.export()["u"], b.export()["u"])
    assert np.all(a.inner_counts() == [60, 12])


@pytest.mark.parametrize("solver", list(SOLVERS))
def test_constant_image_stops_at_the_fixed_point(solver):
    """One subdomain and constant f: p = 0 is the solution and the first step
    changes nothing (div^* of a constant u is 0 on interior edges), so every
    local solve stops after one step.  (On a decomposed grid the one-sided
    differences at the interfaces move p off 0.)"""
    f = np.full((20, 17), 0.3)
    args = dict(SOLVERS[solver])
    args.pop("mask", None)
    a = oracle.Oracle(oracle.Problem(f, ALPHA[solver], np.array([0, 20]), np.array([0, 17]), n_inner=30,
                                     inner_tol=1e-6, **args))
    a.run(3)
    assert np.all(a.inner_counts() == [3, 1])
    assert not a.export()["p"].any()


@pytest.mark.parametrize("solver", list(SOLVERS))
def test_counts_accumulate_over_outer_steps(solver):
    rng = np.random.default_rng(8)
    f = rng.uniform(size=(20, 17))
    a = make(f, solver, n_inner=40, inner_tol=1e-3)
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
