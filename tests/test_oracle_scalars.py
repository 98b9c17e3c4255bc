"""Pins of the scalars of Algorithm 1 (Sec. 4): the step sigma of the
multiplier update, the step tau of the anchor phat = p~^n - tau B^* lambda^(n+1)
and the proximal weight 1/tau of the local problems eq. (DD_local_dual) /
eq. (DD_local).

The fixed point of (DD) does not depend on sigma or tau, so convergence pins
cannot see them.  These pins follow single outer steps instead:

  * with enough local steps every local problem is solved exactly, and one
    outer step must equal the exact proximal step of Chambolle-Pock's
    Algorithm 1 applied to the saddle problem (DD), which is what the paper
    says Algorithm 1 is (the sequence agrees with the standard primal-dual
    one, Sec. 4 after Alg. 1);
  * the reference is oracle/textbook.py's dd_saddle_cp: one global torn
    vector, matrices of the torn divergence and of B built from their
    definitions, the proximal step solved by bounded least squares (BVLS).

sigma and tau are chosen unequal and with tau*sigma < 1/2 as well as at the
paper's tau*sigma = 1/2, so a swapped or rescaled scalar moves the result.
tests/test_oracle_mutations.py plants such slips in copies of the oracle and
checks that these functions then report large errors.
"""
import numpy as np
import pytest

import oracle
from oracle import textbook as tb

H, W = 6, 7
RC, CC = [0, 3, 6], [0, 4, 7]
K_EXACT = 20000          # local steps: the local problems are solved to rounding
CASES = [
    dict(alpha=4.0, tau=3.0, sigma=0.11),      # tau sigma = 0.33 < 1/2
    dict(alpha=10.0, tau=50.0, sigma=0.01),    # the paper's tau = 50, tau sigma = 1/2
]


def _image():
    return np.random.default_rng(3).uniform(size=(H, W))


def _oracle(inner, case, lib_path=oracle.LIB_PATH):
    return oracle.Oracle(oracle.Problem(_image(), case["alpha"], np.asarray(RC), np.asarray(CC), inner=inner,
                                        n_inner=K_EXACT, tau=case["tau"], sigma=case["sigma"],
                                        gamma=1.0 / (8.0 * case["tau"])), lib_path=lib_path)


def _random_state(o, Bm, dof, seed):
    """A state of Algorithm 1 with every term nonzero: p^n and p^(n-1) inside
    the box, lambda^n, all random."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(-1, 1, o.n_p) * dof
    p_prev = rng.uniform(-1, 1, o.n_p) * dof
    lam = 0.05 * rng.standard_normal(o.n_lam)
    s_copy, t_copy = (Bm == 1).astype(float) @ p_prev, (Bm == -1).astype(float) @ p_prev
    nh = (len(RC) - 2) * W
    prev = np.concatenate([s_copy[:nh], t_copy[:nh], s_copy[nh:], t_copy[nh:]])
    return p, p_prev, lam, {"u": _image(), "p": p, "lam": lam, "prev": prev, "n_done": 3}


def saddle_errors(inner, case, n_outer=3, start="random", lib_path=oracle.LIB_PATH):
    """Largest differences (p, lambda, u) between n_outer oracle steps with
    exact local solves and the textbook iteration on (DD)."""
    f = _image()
    Div, Bm, dof = tb.torn_operators(H, W, RC, CC)
    o = _oracle(inner, case, lib_path)
    if start == "random":
        p, p_prev, lam, st = _random_state(o, Bm, dof, seed=11)
        o.import_state(st)
    else:                                   # the start of Algorithm 1: all zero
        p = p_prev = lam = None
    ref = tb.dd_saddle_cp(f, case["alpha"], RC, CC, case["tau"], case["sigma"], n_outer, p=p, p_prev=p_prev,
                          lam=lam)
    err = np.zeros(3)
    for q, lam_ref, u_ref in ref:
        o.run(1)
        e = o.export()
        err = np.maximum(err, [np.abs(e["p"] - q).max(), np.abs(e["lam"] - lam_ref).max(),
                               np.abs(e["u"] - u_ref).max()])
    return err


def test_torn_operators_match_the_oracle():
    """The two independent builds of div~ and B agree (integer data: exact)."""
    o = _oracle("FISTA", CASES[0])
    Div, Bm, dof = tb.torn_operators(H, W, RC, CC)
    rng = np.random.default_rng(2)
    p = rng.integers(-5, 6, o.n_p).astype(float) * dof
    assert np.array_equal(o.div(p), (Div @ p).reshape(H, W))
    assert np.array_equal(o.B(p), Bm @ p)
    assert int(dof.sum()) == (H - 1) * W + H * (W - 1) + o.n_lam
    assert np.array_equal(Bm @ Bm.T, 2.0 * np.eye(o.n_lam))      # Prop. B_norm: B B^* = 2 I


@pytest.mark.parametrize("case", CASES, ids=["tau3_sigma0.11", "tau50_sigma0.01"])
@pytest.mark.parametrize("inner", ["FISTA", "CP2"])
def test_one_outer_step_is_the_exact_proximal_step(inner, case):
    """From a random state with nonzero lambda, phat and p^(n-1): lambda^(n+1)
    = lambda^n + sigma B(2p~^n - p~^(n-1)) and p~^(n+1) = the exact minimiser of
    eq. (DD_local_dual) with anchor p~^n - tau B^* lambda^(n+1) and weight
    1/(2 tau); u = f + div~ p / alpha (ROF)."""
    ep, el, eu = saddle_errors(inner, case, n_outer=1)
    assert el <= 1e-13, el
    assert ep <= 1e-9, ep
    assert eu <= 1e-9, eu


@pytest.mark.parametrize("start", ["zero", "random"])
@pytest.mark.parametrize("inner", ["FISTA", "CP2"])
def test_outer_steps_are_textbook_cp_on_the_dd_saddle(inner, start):
    """Five outer steps with exact local solves follow Chambolle-Pock's
    Algorithm 1 on (DD) (sigma on the multipliers, tau on p, extrapolation
    2p~^n - p~^(n-1)) to 1e-8."""
    ep, el, eu = saddle_errors(inner, CASES[0], n_outer=5, start=start)
    assert max(ep, el, eu) <= 1e-8, (ep, el, eu)
