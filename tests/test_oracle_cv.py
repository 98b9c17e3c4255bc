"""Pins of the oracle's convex Chan-Vese fidelity (Sec. 3, eq. CCV; the
segmentation experiment of Sec. 5.3 with its outer parameters tau = 1,
tau sigma = 1/2).

The references are independent of the oracle's decomposed code: the prox by
brute-force minimisation, the textbook primal-dual method on global arrays,
the exact minimum as a linear program, and the binary problem by enumeration
(by the coarea formula the convex model and the binary one have the same
minimum, and thresholding a minimiser at any level in (0, 1) gives a binary
minimiser).
"""
import numpy as np
import pytest

import oracle
from oracle import textbook as tb

C1, C2 = 0.6, 0.1     # the intensities used for the segmentation experiment
CV = dict(fidelity="CV", inner="CP2", tau=1.0, sigma=0.5, gamma=1.0 / 8.0, c1=C1, c2=C2)


def make(f, alpha, rc, cc, **kw):
    args = dict(CV)
    args.update(kw)
    return oracle.Oracle(oracle.Problem(np.asarray(f, dtype=np.float64), alpha, np.asarray(rc),
                                        np.asarray(cc), **args))


def binary_energy(S, f, alpha):
    return alpha * float((S * tb.cv_g(f, C1, C2)).sum()) + tb.tv_aniso(S)


def test_prox_cv_minimises_linear_term_on_unit_interval():
    rng = np.random.default_rng(21)
    z, f = rng.normal(0.5, 0.8, 300), rng.uniform(size=300)
    a = 0.3
    u = oracle.prox("CV", z, f, a, c1=C1, c2=C2)
    g = (f - C1) ** 2 - (f - C2) ** 2
    grid = np.linspace(0.0, 1.0, 200001)
    for k in range(0, 300, 13):
        obj = a * g[k] * grid + 0.5 * (grid - z[k]) ** 2
        assert abs(grid[np.argmin(obj)] - u[k]) <= 1e-5
    assert u.min() >= 0.0 and u.max() <= 1.0


def test_one_subdomain_cp2_is_textbook_cp2():
    rng = np.random.default_rng(22)
    f = rng.uniform(size=(18, 23))
    o = make(f, 10.0, [0, 18], [0, 23], n_inner=40, no_prox_term=True, gamma=0.0)
    o.run(1)
    e = o.export()
    q1, q2, u = tb.cp2_full(f, 10.0, 40, 10.0, 1 / 80, 0.0, fidelity="CV", c1=C1, c2=C2)
    P1, P2 = o.to_torn(e["p"])
    assert np.abs(P1[1:18] - q1).max() <= 1e-13
    assert np.abs(P2[:, 1:23] - q2).max() <= 1e-13
    assert np.abs(e["u"] - u).max() <= 1e-13


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_lp_minimum_equals_binary_minimum(seed):
    """Coarea: the convex relaxation is exact (pins the LP reference itself)."""
    rng = np.random.default_rng(100 + seed)
    f = rng.uniform(size=(3, 4))
    J, u = tb.cv_exact_energy(f, 4.0, C1, C2)
    Jb, S = tb.cv_binary_min(f, 4.0, C1, C2)
    assert abs(J - Jb) <= 1e-9 * max(1.0, abs(Jb))
    assert abs(binary_energy(S, f, 4.0) - Jb) <= 1e-12


@pytest.mark.parametrize("rc,cc", [([0, 2, 4], [0, 2, 4]), ([0, 1, 4], [0, 3, 4]), ([0, 4], [0, 4])])
def test_dd_converges_to_exact_minimum(rc, cc):
    rng = np.random.default_rng(31)
    f = np.clip(np.kron([[0.6, 0.1], [0.1, 0.6]], np.ones((2, 2))) + rng.normal(0, 0.1, (4, 4)), 0, 1)
    alpha = 6.0
    J, _ = tb.cv_exact_energy(f, alpha, C1, C2)
    Jb, S = tb.cv_binary_min(f, alpha, C1, C2)
    assert abs(J - Jb) <= 1e-9 * abs(Jb) and abs(Jb) > 0.1 and 0 < S.sum() < 16   # a non-trivial segmentation
    o = make(f, alpha, rc, cc, n_inner=200)
    o.run(3000)
    u = o.export()["u"]
    assert u.min() >= 0.0 and u.max() <= 1.0
    assert abs(o.energy(u) - J) <= 1e-6 * abs(J)
    # thresholding at 1/2 (the paper's binarisation) gives a binary minimiser
    assert abs(binary_energy((u > 0.5).astype(float), f, alpha) - Jb) <= 1e-6 * abs(Jb)


def test_duality_gap_is_nonnegative_and_closes():
    """Weak duality at random states, strong duality at the solution: pins the
    dual value D(p) = sum min(0, alpha g - div p) of the Chan-Vese model."""
    rng = np.random.default_rng(41)
    f = rng.uniform(size=(6, 7))
    alpha = 2.5
    o = make(f, alpha, [0, 3, 6], [0, 4, 7], n_inner=50)
    st = o.export()
    for _ in range(20):
        st = dict(st)
        st["p"] = rng.uniform(-1, 1, o.n_p)
        st["u"] = rng.uniform(0, 1, (6, 7))
        o.import_state(st)
        J, D, gap, _ = o.diagnostics()
        assert gap >= -1e-12 and np.isfinite(D)
    o2 = make(f, alpha, [0, 3, 6], [0, 4, 7], n_inner=200)
    rows = o2.run(4000, diag_every=1000)
    Jstar, _ = tb.cv_exact_energy(f, alpha, C1, C2)
    J, D, gap, nb = rows[-1, 1:]
    assert abs(J - Jstar) <= 1e-6 * abs(Jstar)
    assert abs(D - Jstar) <= 1e-5 * abs(Jstar)
    assert nb <= 1e-5


@pytest.mark.parametrize("level,expect", [(0.2, 0.0), (0.5, 1.0)])
def test_constant_image_segments_to_the_nearer_intensity(level, expect):
    """g > 0 everywhere (f nearer c2) gives u = 0, g < 0 (f nearer c1) gives u = 1."""
    f = np.full((9, 10), level)
    o = make(f, 10.0, [0, 4, 9], [0, 5, 10], n_inner=20)
    o.run(300)
    u = o.export()["u"]
    assert np.abs(u - expect).max() <= 1e-12


def test_rejects_cv_with_fista_or_mask():
    f = np.zeros((8, 8))
    with pytest.raises(ValueError):
        make(f, 1.0, [0, 8], [0, 8], inner="FISTA")
    with pytest.raises(ValueError):
        make(f, 1.0, [0, 8], [0, 8], mask=np.ones((8, 8), np.uint8))
