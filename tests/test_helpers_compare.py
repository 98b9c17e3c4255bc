"""The parity comparison itself: a wrong interface row that the global
relative L2 over every dof cannot see is caught by the per-interface check.
The "GPU" state here is the oracle's own state with one planted error (CPU
only)."""
import numpy as np
import pytest

from paper_1901_00682_amd import synth
from tests.helpers import compare, interface_errors, oracle_for, rel_l2


def _state():
    rng = np.random.default_rng(5)
    H = W = 512
    f = (synth.shapes(H, W, rng) + synth.gaussian((H, W), 0.1, rng)).astype(np.float32)
    cuts = np.arange(0, 513, 128)
    o = oracle_for(f, 8.0, cuts, cuts, n_inner=5)
    o.run(4)
    e = o.export()
    Q1, Q2 = o.to_torn(e["p"])
    n = len(e["lam"]) // 1
    gpu = {"u": e["u"].copy(), "P1": Q1.copy(), "P2": Q2.copy(), "lam": e["lam"][:n].copy()}
    return o, gpu


def test_exact_state_passes():
    o, gpu = _state()
    errs = compare(gpu, o)
    assert errs["p"] == 0.0 and errs["if_p"] == 0.0
    assert len(interface_errors(gpu, o)) == 24


def test_wrong_interface_row_is_caught():
    o, gpu = _state()
    k = int(o.row_cuts[2]) + 2 - 1          # the s copy of horizontal interface 2 in the torn P1
    gpu["P1"][k, 128:256] += 2e-4           # the 128 dofs of one interface segment, 2e-4 each
    e = o.export()
    Q1, Q2 = o.to_torn(e["p"])
    glob = rel_l2(np.concatenate([gpu["P1"].ravel(), gpu["P2"].ravel()]), np.concatenate([Q1.ravel(), Q2.ravel()]))
    assert glob <= 1e-5                     # invisible to the global bar
    with pytest.raises(AssertionError, match="interface segment h2.1: p~"):
        compare(gpu, o)


def test_wrong_multiplier_segment_is_caught():
    o, gpu = _state()
    nh = (o.ny - 1) * o.W
    lam = gpu["lam"]
    seg = slice(nh + 2 * o.H, nh + 2 * o.H + 128)  # multipliers of vertical interface 3, first segment
    lam[seg] += 5e-3 * np.abs(lam[seg]).max()
    with pytest.raises(AssertionError, match="interface segment v3.0: lambda"):
        compare(gpu, o, tol_lam=1.0)
