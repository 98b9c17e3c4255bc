"""Pins of the oracle's reverse pass (dl/df, dl/dalpha of the unrolled solve,
FISTA local solver) against central finite differences of the oracle's own
forward map, which is itself pinned in test_oracle_pins.py."""
import numpy as np
import pytest

import oracle
from paper_1901_00682_amd import synth


def _loss(f, g, alpha, rc, cc, n_outer, K):
    o = oracle.Oracle(oracle.Problem(f, alpha, rc, cc, n_inner=K))
    o.run(n_outer)
    u = o.export()["u"]
    return float(((u - g) ** 2).sum()), u


CASES = [
    (24, 24, [0, 8, 16, 24], [0, 8, 16, 24], 8.0, 12, 5),
    (20, 27, [0, 7, 20], [0, 1, 13, 27], 5.0, 9, 4),
    (16, 16, [0, 16], [0, 16], 10.0, 6, 3),
    (1, 30, [0, 1], [0, 11, 30], 6.0, 10, 5),
]


@pytest.mark.parametrize("H,W,rc,cc,alpha,n_outer,K", CASES)
def test_reverse_matches_central_differences(H, W, rc, cc, alpha, n_outer, K):
    rng = np.random.default_rng(H * 1000 + W)
    g = synth.shapes(H, W, rng)
    f = g + synth.gaussian((H, W), 0.1, rng)
    rc, cc = np.array(rc), np.array(cc)
    _, u = _loss(f, g, alpha, rc, cc, n_outer, K)
    o = oracle.Oracle(oracle.Problem(f, alpha, rc, cc, n_inner=K))
    fbar, abar = o.backward(n_outer, 2.0 * (u - g))
    d = rng.standard_normal((H, W))
    d /= np.linalg.norm(d)
    eps = 1e-5
    fd = (_loss(f + eps * d, g, alpha, rc, cc, n_outer, K)[0] - _loss(f - eps * d, g, alpha, rc, cc, n_outer, K)[0]) / (2 * eps)
    fda = (_loss(f, g, alpha + eps, rc, cc, n_outer, K)[0] - _loss(f, g, alpha - eps, rc, cc, n_outer, K)[0]) / (2 * eps)
    assert abs(fd - float((fbar * d).sum())) <= 1e-7 * max(abs(fd), 1e-3)
    assert abs(fda - abar) <= 1e-7 * max(abs(fda), 1e-3)


def test_reverse_with_configured_step():
    """The configured finite-difference step (eps = 1e-3) agrees to 1e-3."""
    c = synth.config5(n_images=1, size=64, grid=4, n_outer=20)[0]
    f = c.f.astype(np.float64)
    g = c.clean.astype(np.float64)
    _, u = _loss(f, g, c.alpha, c.row_cuts, c.col_cuts, c.n_outer, c.n_inner)
    o = oracle.Oracle(oracle.Problem(f, c.alpha, c.row_cuts, c.col_cuts, n_inner=c.n_inner))
    fbar, abar = o.backward(c.n_outer, 2.0 * (u - g))
    rng = synth.rng_for(5, synth.DIRECTION)
    d = rng.standard_normal(f.shape)
    d /= np.linalg.norm(d)
    eps = 1e-3
    lp = _loss(f + eps * d, g, c.alpha, c.row_cuts, c.col_cuts, c.n_outer, c.n_inner)[0]
    lm = _loss(f - eps * d, g, c.alpha, c.row_cuts, c.col_cuts, c.n_outer, c.n_inner)[0]
    fd = (lp - lm) / (2 * eps)
    assert abs(fd - float((fbar * d).sum())) <= 1e-3 * abs(fd)


def test_reverse_of_linear_regime_is_transpose():
    """With a tiny image contrast and a large alpha no constraint is active, the
    unrolled map f -> u is linear, and the reverse pass is its exact
    transpose: <J d1, d2> = <d1, J^T d2>."""
    H, W = 12, 10
    rc, cc = np.array([0, 5, 12]), np.array([0, 4, 10])
    rng = np.random.default_rng(3)
    f0 = 1e-3 * rng.standard_normal((H, W))
    alpha, n_outer, K = 50.0, 6, 4

    def u_of(f):
        o = oracle.Oracle(oracle.Problem(f, alpha, rc, cc, n_inner=K))
        o.run(n_outer)
        e = o.export()
        assert np.abs(e["p"]).max() < 1.0   # no active box constraint
        return e["u"]

    d1, d2 = rng.standard_normal((H, W)), rng.standard_normal((H, W))
    Jd1 = u_of(f0 + d1 * 1e-3) - u_of(f0)   # linear map (u(0) = 0 here): exact up to rounding
    Jd1 /= 1e-3
    o = oracle.Oracle(oracle.Problem(f0, alpha, rc, cc, n_inner=K))
    JTd2, _ = o.backward(n_outer, d2)
    assert abs(float((Jd1 * d2).sum()) - float((d1 * JTd2).sum())) <= 1e-9 * abs(float((Jd1 * d2).sum()))


def test_reverse_rejects_cp2():
    f = np.zeros((8, 8))
    o = oracle.Oracle(oracle.Problem(f, 1.0, np.array([0, 8]), np.array([0, 8]), inner="CP2", fidelity="L1"))
    with pytest.raises(ValueError):
        o.backward(2, np.zeros((8, 8)))
