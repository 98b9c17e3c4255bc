"""Autotuner and hipGraph replay: the choice (schedule x streaming rows) never
changes the numerics, the streaming rows are bitwise interchangeable, graph
replays of outer steps equal eager execution on every replay, and a measured
choice is cached per shape for later plans."""
import sys

import numpy as np
import pytest

from paper_1901_00682_amd import synth
from tests.helpers import gpu_image_state

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_00682_amd import dtvdd
    dtvdd.lib()


def _case(kind):
    rng = np.random.default_rng(77 if kind == "rof" else 78)
    H, W = 200, 263
    clean = synth.shapes(H, W, rng)
    if kind == "rof":
        f = clean + synth.gaussian((H, W), 0.1, rng)
        return f.astype(np.float32), None, dict(fidelity="L2", inner="FISTA")
    f = synth.salt_and_pepper(clean, 0.3, rng)
    mask = synth.stroke_mask(H, W, 0.1, rng)
    f = np.where(mask == 0, 0.0, f)
    return f.astype(np.float32), mask.astype(np.uint8), dict(fidelity="L1", inner="CP2", has_mask=True)


def _run(f, mask, kw, n_outer=9, K=4, state=None, **extra):
    from paper_1901_00682_amd import dtvdd
    H, W = f.shape
    im = dtvdd.Image(H, W, [0, 70, 128, 200], [0, 100, 180, 263], 6.0)
    plan = dtvdd.Plan([im], n_outer=n_outer, n_inner=K, **kw, **extra)
    ft = torch.from_numpy(f.ravel()).cuda()
    mt = None if mask is None else torch.from_numpy(mask.ravel()).cuda()
    st, _ = plan.solve(ft, mt, state=state)
    torch.cuda.synchronize()
    return plan, st


@pytest.mark.parametrize("kind", ["rof", "cp2"])
def test_streaming_rows_bitwise(kind):
    f, mask, kw = _case(kind)
    _say(f"[rows] {kind}")
    ref = None
    for R in (4, 8, 16, 32):
        plan, st = _run(f, mask, kw, schedule="stream", rows=R, graphs=False)
        assert plan.choice() == {"schedule": "stream", "rows": R, "source": "explicit"}
        g = gpu_image_state(plan, st)
        if ref is None:
            ref = g
        for q in ref:
            assert np.array_equal(ref[q], g[q]), (R, q)


@pytest.mark.parametrize("kind,schedule", [("rof", "fused"), ("rof", "stream"), ("cp2", "stream")])
def test_graph_replays_equal_eager(kind, schedule):
    """Several graph-replayed solves, with eager work and synchronisations
    between them, each equal to the eager solve."""
    f, mask, kw = _case(kind)
    _say(f"[graph] {kind} {schedule}")
    plan_e, st_e = _run(f, mask, kw, n_outer=13, schedule=schedule, rows=8, graphs=False)
    ref = gpu_image_state(plan_e, st_e)
    from paper_1901_00682_amd import dtvdd
    H, W = f.shape
    im = dtvdd.Image(H, W, [0, 70, 128, 200], [0, 100, 180, 263], 6.0)
    plan = dtvdd.Plan([im], n_outer=13, n_inner=4, schedule=schedule, rows=8, **kw)
    ft = torch.from_numpy(f.ravel()).cuda()
    mt = None if mask is None else torch.from_numpy(mask.ravel()).cuda()
    st = plan.new_state()
    for rep in range(3):
        plan.solve(ft, mt, state=st)
        torch.cuda.synchronize()
        g = gpu_image_state(plan, st)
        for q in ref:
            assert np.array_equal(ref[q], g[q]), (rep, q)
        # eager work of the program between replays
        _run(f, mask, kw, n_outer=2, schedule=schedule, rows=8, graphs=False)


def test_autotune_measures_caches_and_keeps_numerics():
    from paper_1901_00682_amd import dtvdd
    H, W = 384, 384
    rng = np.random.default_rng(5)
    f = (synth.shapes(H, W, rng) + synth.gaussian((H, W), 0.1, rng)).astype(np.float32)
    cuts = [0, 128, 256, 384]
    im = dtvdd.Image(H, W, cuts, cuts, 8.0)
    ft = torch.from_numpy(f.ravel()).cuda()
    _say("[autotune] 384^2 3x3 full tiles, 60 x 3")
    ref = dtvdd.Plan([im], n_outer=60, n_inner=3, schedule="fused")
    sr, _ = ref.solve(ft)
    auto = dtvdd.Plan([im], n_outer=60, n_inner=3)
    before = auto.choice()
    sa, _ = auto.solve(ft)
    torch.cuda.synchronize()
    after = auto.choice()
    assert before["source"] in ("rule", "cached")
    if before["source"] == "rule":
        assert after["source"] == "measured"
    for k in ("u", "p1", "p2", "lam"):
        assert torch.equal(sr[k], sa[k]), k
    again = dtvdd.Plan([im], n_outer=60, n_inner=3)
    c = again.choice()
    assert c["source"] == "cached"
    assert (c["schedule"], c["rows"]) == (after["schedule"], after["rows"])
    _say(f"  chose {after}")


@pytest.mark.parametrize("fidelity,K", [("CV", 5), ("L1", 4)])
def test_graph_replays_fused_cp2(fidelity, K):
    """The fused primal-dual schedule updates p~ and u in place (one multiplier
    launch and one fused launch per outer step): graph replays equal the eager
    solve on every replay, and the autotuned choice equals both."""
    from paper_1901_00682_amd import dtvdd
    H, W = 256, 384
    rng = np.random.default_rng(90 + K)
    clean = synth.shapes(H, W, rng)
    f = (synth.salt_and_pepper(clean, 0.3, rng) if fidelity == "L1" else clean + synth.gaussian((H, W), 0.05, rng))
    f = f.astype(np.float32)
    extra = dict(tau=1.0, sigma=0.5, gamma=1.0 / 8.0, c1=0.6, c2=0.1) if fidelity == "CV" else {}
    im = dtvdd.Image(H, W, [0, 128, 256], [0, 128, 256, 384], 5.0)
    ft = torch.from_numpy(f.ravel()).cuda()
    _say(f"[graph] fused cp2 {fidelity} K={K}")
    eager = dtvdd.Plan([im], inner="CP2", fidelity=fidelity, n_outer=13, n_inner=K, schedule="fused", graphs=False,
                       **extra)
    se, _ = eager.solve(ft)
    torch.cuda.synchronize()
    ref = gpu_image_state(eager, se)
    plan = dtvdd.Plan([im], inner="CP2", fidelity=fidelity, n_outer=13, n_inner=K, schedule="fused", **extra)
    st = plan.new_state()
    for rep in range(3):
        plan.solve(ft, state=st)
        torch.cuda.synchronize()
        g = gpu_image_state(plan, st)
        for q in ref:
            assert np.array_equal(ref[q], g[q]), (rep, q)
        eager.solve(ft)  # eager work between the replays
    auto = dtvdd.Plan([im], inner="CP2", fidelity=fidelity, n_outer=60, n_inner=K, **extra)
    sa, _ = auto.solve(ft)
    fixed = dtvdd.Plan([im], inner="CP2", fidelity=fidelity, n_outer=60, n_inner=K, schedule="stream", rows=16,
                       graphs=False, **extra)
    sf, _ = fixed.solve(ft)
    torch.cuda.synchronize()
    for k in ("u", "p1", "p2", "lam"):
        assert torch.equal(sa[k], sf[k]), k
    _say(f"  autotuned {auto.choice()}")
