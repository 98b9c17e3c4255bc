"""The outer stopping rule on the GPU (relative primal-dual gap, the outer
rule of Sec. 5.1 with the gap of reading A13) against the same rule applied
to the FP64 oracle's diagnostics, and the TV-L1 inpainting workload (Sec. 5.2,
eq. inpainting_L1) at its full 1000 outer steps.

The stop step comes from the oracle: its diagnostic rows give the relative
gap gap/|J| at every diag_every-th step, the test picks a tolerance halfway
(geometrically) between the first row below a target (1e-2 for ROF, 1e-3 for
Chan-Vese, reached after 50 and 20 outer steps) and the smallest earlier row,
so that FP32 rounding cannot move the decision, and the GPU must stop at that
same step with the same diagnostic rows (1e-6 relative) and the same state
(1e-5 relative L2, per interface 1e-4)."""
import sys

import numpy as np
import pytest

from paper_1901_00682_amd import synth
from tests.helpers import compare, gpu_image_state, oracle_for

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CV_KW = dict(fidelity="CV", inner="CP2", tau=1.0, sigma=0.5, gamma=1.0 / 8.0, c1=0.6, c2=0.1)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_00682_amd import dtvdd
    dtvdd.lib()


def _cases():
    c = synth.config1()
    rng = np.random.default_rng(91)
    fcv = (synth.shapes(96, 112, rng) + synth.gaussian((96, 112), 0.05, rng)).astype(np.float32)
    return {
        # name: (f, alpha, row cuts, col cuts, n_inner, solver keywords, schedule, target relative gap)
        "rof_config1": (c.f.astype(np.float32), c.alpha, c.row_cuts, c.col_cuts, c.n_inner, {}, "fused", 1e-2),
        "chan_vese": (fcv, 10.0, np.array([0, 48, 96]), np.array([0, 40, 112]), 5, CV_KW, "stream", 1e-3),
    }


@pytest.mark.parametrize("name", ["rof_config1", "chan_vese"])
def test_gap_stop_matches_the_oracle_rule(name):
    from paper_1901_00682_amd import dtvdd
    f, alpha, rc, cc, K, kw, sched, target = _cases()[name]
    every, cap = 5, 2000
    okw = {k: v for k, v in kw.items() if k not in ("tau", "sigma", "gamma")}
    o = oracle_for(f, alpha, rc, cc, n_inner=K, tau=kw.get("tau", 50.0), sigma=kw.get("sigma", 0.01),
                   gamma=kw.get("gamma"), **okw)
    rows = o.run(cap, diag_every=every)
    rel = rows[:, 3] / np.abs(rows[:, 1])
    assert (rows[:, 3] >= -1e-9 * np.abs(rows[:, 1])).all()
    k = int(np.argmax(rel < target))
    assert rel[k] < target and k >= 2, "the gap must cross the target within the cap"
    assert rel[:k].min() > 1.4 * rel[k]   # room for FP32 rounding on both sides of the tolerance
    earlier = rel[:k].min()
    tol = float(np.sqrt(rel[k] * earlier))
    stop = int(rows[k, 0])
    _say(f"[gap stop] {name}: oracle stops at {stop} (rel gap {rel[k]:.3e}, smallest earlier {earlier:.3e}, "
         f"tol {tol:.3e})")
    H, W = f.shape
    gk = {kk: v for kk, v in kw.items()}
    plan = dtvdd.Plan([dtvdd.Image(H, W, np.asarray(rc), np.asarray(cc), alpha)], n_outer=cap, n_inner=K,
                      diag_every=every, gap_tol=tol, schedule=sched, **gk)
    ft = torch.from_numpy(f.ravel()).cuda()
    state, stats = plan.solve(ft)
    torch.cuda.synchronize()
    g = stats[0]
    assert g.shape[0] == k + 1, (g.shape, k + 1)
    assert int(g[-1, 0]) == stop
    assert np.array_equal(g[:, 0], rows[: k + 1, 0])
    for q in (1, 2):   # J and D
        assert np.max(np.abs(g[:, q] - rows[: k + 1, q]) / np.abs(rows[: k + 1, q])) <= 1e-6, q
    assert np.max(np.abs(g[:, 3] - rows[: k + 1, 3])) <= 1e-6 * np.abs(rows[: k + 1, 1]).max()
    counts = plan.inner_counts()
    assert (counts[:, 0] == stop * K).all()
    # the state at the stop step
    o2 = oracle_for(f, alpha, rc, cc, n_inner=K, tau=kw.get("tau", 50.0), sigma=kw.get("sigma", 0.01),
                    gamma=kw.get("gamma"), **okw)
    o2.run(stop)
    errs = compare(gpu_image_state(plan, state), o2)
    _say(f"  GPU stopped at {int(g[-1, 0])}; errors {errs}")


@pytest.mark.timeout(900)
def test_parity_config3_full_length():
    """TV-L1 + inpainting mask, 2000 x 3000 (H x W), 13 x 20 uneven subdomains
    (153 or 154 rows, 150 columns), CP2, all 1000 outer steps x 5."""
    c = synth.config3()
    assert c.n_outer == 1000
    _say("[parity] config3 2000x3000 13x20 TV-L1+mask 1000x5 (GPU)")
    from paper_1901_00682_amd import dtvdd
    H, W = c.f.shape
    plan = dtvdd.Plan([dtvdd.Image(H, W, c.row_cuts, c.col_cuts, c.alpha)], has_mask=True, fidelity="L1",
                      inner="CP2", n_outer=c.n_outer, n_inner=c.n_inner)
    ft = torch.from_numpy(np.ascontiguousarray(c.f, dtype=np.float32).ravel()).cuda()
    mt = torch.from_numpy(np.ascontiguousarray(c.mask, dtype=np.uint8).ravel()).cuda()
    state, _ = plan.solve(ft, mt)
    torch.cuda.synchronize()
    g = gpu_image_state(plan, state)
    _say(f"  GPU done ({plan.schedule()}); oracle (CPU)")
    o = oracle_for(c.f, c.alpha, c.row_cuts, c.col_cuts, fidelity="L1", inner="CP2", mask=c.mask, n_inner=c.n_inner)
    o.run(c.n_outer)
    errs = compare(g, o)
    _say(f"  errors {errs}")
