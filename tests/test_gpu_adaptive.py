"""Adaptive local solves (the inner stopping rule of Sec. 5.1) on the GPU: the
per-subdomain step counts equal the FP64 oracle's and the iterates match it to
relative L2 <= 1e-5; the rule degenerates to the fixed-count path (bitwise) for
a vanishing tolerance and to one step for a huge one.

The counts are integers decided by floating point: every case first checks
that no decision of the oracle came near the threshold.  The GPU's iterates
carry FP32 rounding of about 1e-6 relative, so the relative change
|p_k - p_(k-1)| / |p_k| near a tolerance tol is known to about 1e-6 / tol
relative; the cases require the oracle's log-distance of every decision
(in |p_k - p_(k-1)|^2 / |p_k|^2) from the threshold to exceed
max(1e-3, 8e-6 / tol), so that both sides must decide alike."""
import sys

import numpy as np
import pytest

from paper_1901_00682_amd import synth
from tests.helpers import compare, gpu_image_state, oracle_for

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

def margin_needed(tol):
    return max(1e-3, 8e-6 / tol)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_00682_amd import dtvdd
    dtvdd.lib()


def run_gpu(f32, alpha, rc, cc, **kw):
    from paper_1901_00682_amd import dtvdd
    H, W = f32.shape
    plan = dtvdd.Plan([dtvdd.Image(H, W, np.asarray(rc), np.asarray(cc), alpha)], **kw)
    f = torch.from_numpy(np.ascontiguousarray(f32, dtype=np.float32).ravel()).cuda()
    state, stats = plan.solve(f)
    torch.cuda.synchronize()
    return plan, state, stats


GEOMS = {
    # full 128 x 128 tiles beside ragged ones
    "mixed": (300, 357, [0, 128, 256, 300], [0, 101, 229, 357]),
    # only full tiles (the specialised kernel)
    "full2x2": (256, 256, [0, 128, 256], [0, 128, 256]),
    # small ragged tiles
    "ragged": (70, 150, [0, 20, 41, 70], [0, 1, 63, 64, 100, 150]),
}
CASES = [("mixed", 1e-2, 40, 8, 11), ("full2x2", 5e-3, 30, 10, 12), ("ragged", 1e-2, 200, 12, 12),
         ("full2x2", 3e-3, 150, 4, 11)]


@pytest.mark.parametrize("geom,tol,cap,n_outer,seed", CASES)
def test_adaptive_matches_oracle(geom, tol, cap, n_outer, seed):
    H, W, rc, cc = GEOMS[geom]
    rng = np.random.default_rng(seed)
    f = (synth.shapes(H, W, rng) + synth.gaussian((H, W), 0.1, rng)).astype(np.float32)
    o = oracle_for(f, 8.0, rc, cc, n_inner=cap, inner_tol=tol)
    o.run(n_outer)
    assert o.inner_margin() > margin_needed(tol), f"oracle decision within {o.inner_margin():.2e} of the threshold"
    _say(f"[adaptive] {geom} {H}x{W} tol={tol} cap={cap} outer={n_outer}")
    plan, state, _ = run_gpu(f, 8.0, rc, cc, n_outer=n_outer, n_inner=cap, inner_tol=tol)
    assert plan.schedule() in ("fused", "persistent")
    got = plan.inner_counts()
    want = o.inner_counts()
    _say(f"  steps per subdomain {got[:, 0].tolist()} (cap {cap * n_outer})")
    assert np.array_equal(got, want)
    assert got[:, 0].min() < cap * n_outer  # the rule stopped something early
    errs = compare(gpu_image_state(plan, state), o)
    _say(f"  errors {errs}")


@pytest.mark.parametrize("geom,K", [("mixed", 5), ("full2x2", 6), ("ragged", 3)])
def test_vanishing_tolerance_is_the_fixed_count(geom, K):
    H, W, rc, cc = GEOMS[geom]
    rng = np.random.default_rng(20 + K)
    f = (synth.shapes(H, W, rng) + synth.gaussian((H, W), 0.1, rng)).astype(np.float32)
    _say(f"[adaptive=fixed] {geom} K={K}")
    pa, sa, _ = run_gpu(f, 8.0, rc, cc, n_outer=5, n_inner=K, inner_tol=1e-30)
    pf, sf, _ = run_gpu(f, 8.0, rc, cc, n_outer=5, n_inner=K, schedule="fused")
    ga, gf = gpu_image_state(pa, sa), gpu_image_state(pf, sf)
    for q in ga:
        assert np.array_equal(ga[q], gf[q]), q
    assert np.all(pa.inner_counts() == [5 * K, K])


def test_vanishing_tolerance_beyond_the_unrolled_counts():
    """Caps above the fused kernel's fixed counts read the momentum table from
    device memory: bitwise equal to the streaming schedule with 100 steps."""
    H, W, rc, cc = GEOMS["mixed"]
    rng = np.random.default_rng(27)
    f = (synth.shapes(H, W, rng) + synth.gaussian((H, W), 0.1, rng)).astype(np.float32)
    pa, sa, _ = run_gpu(f, 8.0, rc, cc, n_outer=3, n_inner=100, inner_tol=1e-30)
    ps, ss, _ = run_gpu(f, 8.0, rc, cc, n_outer=3, n_inner=100, schedule="stream")
    ga, gs = gpu_image_state(pa, sa), gpu_image_state(ps, ss)
    for q in ga:
        assert np.array_equal(ga[q], gs[q]), q
    assert np.all(pa.inner_counts() == [300, 100])


def test_huge_tolerance_takes_one_step():
    H, W, rc, cc = GEOMS["mixed"]
    rng = np.random.default_rng(31)
    f = (synth.shapes(H, W, rng) + synth.gaussian((H, W), 0.1, rng)).astype(np.float32)
    pa, sa, _ = run_gpu(f, 8.0, rc, cc, n_outer=4, n_inner=50, inner_tol=1e30)
    pf, sf, _ = run_gpu(f, 8.0, rc, cc, n_outer=4, n_inner=1, schedule="fused")
    ga, gf = gpu_image_state(pa, sa), gpu_image_state(pf, sf)
    for q in ga:
        assert np.array_equal(ga[q], gf[q]), q
    assert np.all(pa.inner_counts() == [4, 1])


@pytest.mark.parametrize("tol,cap,n_outer", [(5e-3, 30, 10), (1e-30, 7, 4), (3e-3, 150, 3)])
def test_adaptive_persistent_equals_fused(tol, cap, n_outer):
    """The stopping rule inside the persistent kernel (every outer step in
    one launch): bitwise the fused schedule's iterates and step counts."""
    H, W, rc, cc = 384, 384, [0, 128, 256, 384], [0, 128, 256, 384]
    rng = np.random.default_rng(61 + cap)
    f = (synth.shapes(H, W, rng) + synth.gaussian((H, W), 0.1, rng)).astype(np.float32)
    _say(f"[adaptive persistent==fused] tol={tol} cap={cap} outer={n_outer}")
    res, counts = {}, {}
    for sch in ("fused", "persistent"):
        plan, st, _ = run_gpu(f, 8.0, rc, cc, n_outer=n_outer, n_inner=cap, inner_tol=tol, schedule=sch)
        assert plan.schedule() == sch
        res[sch] = gpu_image_state(plan, st)
        counts[sch] = plan.inner_counts()
    assert np.array_equal(counts["fused"], counts["persistent"])
    for q in res["fused"]:
        assert np.array_equal(res["fused"][q], res["persistent"][q]), q
    _say(f"  steps per subdomain {counts['fused'][:, 0].tolist()}")


def test_adaptive_counts_reset_between_solves():
    H, W, rc, cc = GEOMS["ragged"]
    rng = np.random.default_rng(41)
    f = (synth.shapes(H, W, rng) + synth.gaussian((H, W), 0.1, rng)).astype(np.float32)
    from paper_1901_00682_amd import dtvdd
    plan = dtvdd.Plan([dtvdd.Image(H, W, np.asarray(rc), np.asarray(cc), 8.0)], n_outer=6, n_inner=40, inner_tol=1e-3)
    ft = torch.from_numpy(f.ravel()).cuda()
    plan.solve(ft)
    first = plan.inner_counts().copy()
    plan.solve(ft)
    assert np.array_equal(plan.inner_counts(), first)


def test_adaptive_plan_does_not_take_a_fixed_count_choice():
    """A measured choice of a fixed-count plan of the same shape is not reused
    by an adaptive plan (the streaming schedule has no stopping rule)."""
    from paper_1901_00682_amd import dtvdd
    H, W, rc, cc = GEOMS["mixed"]
    rng = np.random.default_rng(91)
    f = (synth.shapes(H, W, rng) + synth.gaussian((H, W), 0.1, rng)).astype(np.float32)
    ft = torch.from_numpy(f.ravel()).cuda()
    im = dtvdd.Image(H, W, np.asarray(rc), np.asarray(cc), 8.0)
    fixed = dtvdd.Plan([im], n_outer=80, n_inner=40)
    fixed.solve(ft)
    torch.cuda.synchronize()
    adaptive = dtvdd.Plan([im], n_outer=80, n_inner=40, inner_tol=1e-2)
    ch = adaptive.choice()
    _say(f"  fixed-count plan chose {fixed.choice()}; adaptive plan starts from {ch}")
    assert ch["schedule"] in ("fused", "persistent") and ch["source"] != "cached"
    adaptive.solve(ft)
    torch.cuda.synchronize()
    assert adaptive.inner_counts()[:, 0].max() < 80 * 40
