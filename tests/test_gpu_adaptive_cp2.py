"""Adaptive local solves (the inner stopping rule of Sec. 5.1) with the local
accelerated primal-dual solver on the GPU, in the fused and the persistent
schedules: per-subdomain step counts equal the FP64 oracle's and the state
(p~, lambda and u = u^(k) of the last step taken) matches it to relative L2
<= 1e-5; a vanishing tolerance is the fixed-count path (bitwise), also for
caps beyond the kernels' argument tables; a huge one is one step; the
persistent kernel equals the fused one bitwise.  Also the persistent FISTA
kernel with the rule on framed tiles (smaller than 128 x 128) against the
fused schedule.

The counts are integers decided by floating point: every case first checks
that no decision of the oracle came near the threshold (the margin rule of
test_gpu_adaptive.py)."""
import sys

import numpy as np
import pytest

from paper_1901_00682_amd import synth
from tests.helpers import compare, gpu_image_state, oracle_for

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CV = dict(fidelity="CV", inner="CP2", tau=1.0, sigma=0.5, gamma=1.0 / 8.0, c1=0.6, c2=0.1)
L1 = dict(fidelity="L1", inner="CP2", gamma=1.0 / 400.0)
GEOMS = {
    # the last subdomain row (43 rows) and column (45 columns) are framed tiles
    "framed3x3": (299, 301, [0, 128, 256, 299], [0, 128, 256, 301]),
    "full2x2": (256, 256, [0, 128, 256], [0, 128, 256]),
}


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


def _problem(geom, kind, seed):
    H, W, rc, cc = GEOMS[geom]
    rng = np.random.default_rng(100 + seed)
    clean = synth.shapes(H, W, rng)
    if kind == "L1":
        f = synth.salt_and_pepper(clean, 0.3, rng)
        mask = synth.stroke_mask(H, W, 0.1, rng)
        return np.where(mask == 1, f, 0.0).astype(np.float32), mask, 1.5, L1
    return (clean + synth.gaussian((H, W), 0.05, rng)).astype(np.float32), None, 10.0, CV


def run_gpu(f32, alpha, rc, cc, mask=None, **kw):
    from paper_1901_00682_amd import dtvdd
    H, W = f32.shape
    plan = dtvdd.Plan([dtvdd.Image(H, W, np.asarray(rc), np.asarray(cc), alpha)], has_mask=mask is not None, **kw)
    f = torch.from_numpy(np.ascontiguousarray(f32, dtype=np.float32).ravel()).cuda()
    m = None if mask is None else torch.from_numpy(np.ascontiguousarray(mask, dtype=np.uint8).ravel()).cuda()
    state, _ = plan.solve(f, m)
    torch.cuda.synchronize()
    return plan, state


CASES = [  # (geometry, fidelity, seed, tol, cap, n_outer)
    ("framed3x3", "L1", 2, 3e-2, 80, 6),
    ("full2x2", "L1", 1, 2e-2, 80, 5),
    ("full2x2", "CV", 0, 1e-2, 60, 6),
    ("framed3x3", "CV", 0, 1e-2, 60, 5),
]


@pytest.mark.parametrize("schedule", ["fused", "persistent"])
@pytest.mark.parametrize("geom,kind,seed,tol,cap,n_outer", CASES)
def test_cp2_adaptive_matches_oracle(geom, kind, seed, tol, cap, n_outer, schedule):
    H, W, rc, cc = GEOMS[geom]
    f, mask, alpha, kw = _problem(geom, kind, seed)
    o = oracle_for(f, alpha, rc, cc, mask=mask, n_inner=cap, inner_tol=tol, **kw)
    o.run(n_outer)
    assert o.inner_margin() > margin_needed(tol), f"oracle decision within {o.inner_margin():.2e} of the threshold"
    _say(f"[adaptive CP2] {geom} {kind} tol={tol} cap={cap} outer={n_outer} {schedule}")
    plan, state = run_gpu(f, alpha, rc, cc, mask=mask, n_outer=n_outer, n_inner=cap, inner_tol=tol,
                          schedule=schedule, **kw)
    assert plan.schedule() == schedule
    got, want = plan.inner_counts(), o.inner_counts()
    _say(f"  steps per subdomain {got[:, 0].tolist()} (cap {cap * n_outer})")
    assert np.array_equal(got, want)
    assert got[:, 0].max() < cap * n_outer and len(set(got[:, 0].tolist())) > 1
    errs = compare(gpu_image_state(plan, state), o)
    _say(f"  errors {errs}")


@pytest.mark.parametrize("geom,kind,K", [("framed3x3", "L1", 5), ("full2x2", "CV", 6), ("framed3x3", "CV", 3)])
def test_cp2_vanishing_tolerance_is_the_fixed_count(geom, kind, K):
    H, W, rc, cc = GEOMS[geom]
    f, mask, alpha, kw = _problem(geom, kind, 7)
    _say(f"[adaptive CP2=fixed] {geom} {kind} K={K}")
    for sch in ("fused", "persistent"):
        pa, sa = run_gpu(f, alpha, rc, cc, mask=mask, n_outer=5, n_inner=K, inner_tol=1e-30, schedule=sch, **kw)
        pf, sf = run_gpu(f, alpha, rc, cc, mask=mask, n_outer=5, n_inner=K, schedule="fused", **kw)
        ga, gf = gpu_image_state(pa, sa), gpu_image_state(pf, sf)
        for q in ga:
            assert np.array_equal(ga[q], gf[q]), (sch, q)
        assert np.all(pa.inner_counts() == [5 * K, K])


def test_cp2_vanishing_tolerance_beyond_the_argument_tables():
    """A cap of 100 steps (beyond the 64 step scalars the kernels take as
    arguments) reads the scalars from device memory: bitwise equal to the
    streaming schedule with 100 fixed steps."""
    H, W, rc, cc = GEOMS["framed3x3"]
    f, mask, alpha, kw = _problem("framed3x3", "L1", 8)
    pa, sa = run_gpu(f, alpha, rc, cc, mask=mask, n_outer=3, n_inner=100, inner_tol=1e-30, **kw)
    ps, ss = run_gpu(f, alpha, rc, cc, mask=mask, n_outer=3, n_inner=100, schedule="stream", **kw)
    ga, gs = gpu_image_state(pa, sa), gpu_image_state(ps, ss)
    for q in ga:
        assert np.array_equal(ga[q], gs[q]), q
    assert np.all(pa.inner_counts() == [300, 100])


def test_cp2_huge_tolerance_takes_one_step():
    H, W, rc, cc = GEOMS["framed3x3"]
    f, mask, alpha, kw = _problem("framed3x3", "CV", 9)
    pa, sa = run_gpu(f, alpha, rc, cc, n_outer=4, n_inner=50, inner_tol=1e30, **kw)
    pf, sf = run_gpu(f, alpha, rc, cc, n_outer=4, n_inner=1, schedule="fused", **kw)
    ga, gf = gpu_image_state(pa, sa), gpu_image_state(pf, sf)
    for q in ga:
        assert np.array_equal(ga[q], gf[q]), q
    assert np.all(pa.inner_counts() == [4, 1])


@pytest.mark.parametrize("geom,kind,tol,cap,n_outer", [("framed3x3", "L1", 3e-2, 80, 4), ("full2x2", "CV", 1e-2, 60, 5)])
def test_cp2_adaptive_persistent_equals_fused(geom, kind, tol, cap, n_outer):
    H, W, rc, cc = GEOMS[geom]
    f, mask, alpha, kw = _problem(geom, kind, 11)
    res, counts = {}, {}
    for sch in ("fused", "persistent"):
        plan, st = run_gpu(f, alpha, rc, cc, mask=mask, n_outer=n_outer, n_inner=cap, inner_tol=tol, schedule=sch,
                           **kw)
        res[sch], counts[sch] = gpu_image_state(plan, st), plan.inner_counts()
    assert np.array_equal(counts["fused"], counts["persistent"])
    for q in res["fused"]:
        assert np.array_equal(res["fused"][q], res["persistent"][q]), q
    _say(f"  steps per subdomain {counts['fused'][:, 0].tolist()}")


FISTA_FRAMED = {
    # framed tiles with their short sides on the image boundary
    "framed3x3": (299, 301, [0, 128, 256, 299], [0, 128, 256, 301]),
    # framed tiles with interfaces on their short sides (masks)
    "mixed": (300, 357, [0, 128, 256, 300], [0, 101, 229, 357]),
}


@pytest.mark.parametrize("geom", list(FISTA_FRAMED))
def test_fista_adaptive_persistent_framed(geom):
    """The persistent FISTA kernel with the stopping rule on framed tiles
    (full-tile steps in a 128 x 128 frame; the fused schedule runs those tiles
    on its general kernel, whose per-thread partial sums group the edges
    differently): the oracle's step counts and state in both schedules, and
    bitwise equal iterates when the counts agree."""
    H, W, rc, cc = FISTA_FRAMED[geom]
    rng = np.random.default_rng(74)
    f = (synth.shapes(H, W, rng) + synth.gaussian((H, W), 0.1, rng)).astype(np.float32)
    tol, cap, n_outer = 1e-2, 40, 6
    o = oracle_for(f, 8.0, rc, cc, n_inner=cap, inner_tol=tol)
    o.run(n_outer)
    assert o.inner_margin() > margin_needed(tol), f"oracle decision within {o.inner_margin():.2e} of the threshold"
    res, counts = {}, {}
    for sch in ("fused", "persistent"):
        plan, st = run_gpu(f, 8.0, rc, cc, n_outer=n_outer, n_inner=cap, inner_tol=tol, schedule=sch)
        assert plan.schedule() == sch
        res[sch], counts[sch] = gpu_image_state(plan, st), plan.inner_counts()
        assert np.array_equal(counts[sch], o.inner_counts()), sch
        errs = compare(res[sch], o)
        _say(f"  {geom} {sch}: steps per subdomain {counts[sch][:, 0].tolist()}; errors {errs}")
    for q in res["fused"]:
        assert np.array_equal(res["fused"][q], res["persistent"][q]), q
