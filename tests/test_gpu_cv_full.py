"""Convex Chan-Vese segmentation (Sec. 3, eq. CCV, with the local primal-dual
solver of Sec. 5) and the undecomposed problem (the N = 1 comparison of
Sec. 5) on the GPU against the FP64 oracle at matched iteration counts:
relative L2 <= 1e-5 on u and on p, FP64 diagnostics within 1e-6 relative."""
import sys

import numpy as np
import pytest

from paper_1901_00682_amd import synth
from tests.helpers import compare, gpu_image_state, oracle_for, rel_l2

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


def run_gpu(f32, alpha, rc, cc, mask=None, **kw):
    from paper_1901_00682_amd import dtvdd
    H, W = f32.shape
    plan = dtvdd.Plan([dtvdd.Image(H, W, np.asarray(rc), np.asarray(cc), alpha)], has_mask=mask is not None, **kw)
    f = torch.from_numpy(np.ascontiguousarray(f32, dtype=np.float32).ravel()).cuda()
    m = None if mask is None else torch.from_numpy(np.ascontiguousarray(mask, dtype=np.uint8).ravel()).cuda()
    state, stats = plan.solve(f, m)
    torch.cuda.synchronize()
    return plan, state, stats


def _oracle_cv(f, alpha, rc, cc, n_inner, **kw):
    args = dict(CV_KW)
    args.update(kw)
    return oracle_for(f, alpha, rc, cc, n_inner=n_inner, **args)


def _check_stats(g, ost):
    assert np.array_equal(g[:, 0], ost[:, 0])
    for q in (1, 2):   # J and D to 1e-6 relative
        assert np.max(np.abs(g[:, q] - ost[:, q]) / np.abs(ost[:, q])) <= 1e-6, q
    # the gap relative to the energy scale
    assert np.max(np.abs(g[:, 3] - ost[:, 3])) <= 1e-6 * np.abs(ost[:, 1]).max()


def test_cv_parity_ragged_grid():
    rng = np.random.default_rng(61)
    H, W, rc, cc = 90, 140, [0, 31, 60, 90], [0, 35, 70, 105, 140]
    f = (synth.shapes(H, W, rng) + synth.gaussian((H, W), 0.05, rng)).astype(np.float32)
    _say(f"[cv] {H}x{W} 3x4 ragged 30x5 with diagnostics")
    plan, state, stats = run_gpu(f, 10.0, rc, cc, n_outer=30, n_inner=5, diag_every=10, schedule="stream", **CV_KW)
    o = _oracle_cv(f, 10.0, rc, cc, 5)
    ost = o.run(30, diag_every=10)
    g = gpu_image_state(plan, state)
    errs = compare(g, o)
    _say(f"  errors {errs}")
    assert g["u"].min() >= 0.0 and g["u"].max() <= 1.0
    _check_stats(stats[0], ost)
    # the gap is finite and non-negative for the Chan-Vese model
    assert np.all(np.isfinite(stats[0][:, 3])) and np.all(stats[0][:, 3] >= -1e-6 * np.abs(stats[0][:, 1]))


@pytest.mark.parametrize("rows", [4, 32])
def test_cv_parity_full_size(rows):
    """The segmentation workload at its full size (2048 x 2048, 16 x 16
    subdomains of 128 x 128) for 12 outer steps, element by element."""
    c = synth.cv_case(n_outer=12)
    _say(f"[cv] {c.name} 12x{c.n_inner} rows={rows}")
    plan, state, _ = run_gpu(c.f, c.alpha, c.row_cuts, c.col_cuts, n_outer=12, n_inner=c.n_inner, rows=rows,
                             schedule="stream", **CV_KW)
    o = _oracle_cv(c.f, c.alpha, c.row_cuts, c.col_cuts, c.n_inner)
    o.run(12)
    errs = compare(gpu_image_state(plan, state), o)
    _say(f"  errors {errs}")


FULL = {
    # name: (H, W, fidelity, inner, masked, alpha, n_outer, n_inner, gamma)
    "fista_restarts": (64, 80, "L2", "FISTA", False, 8.0, 3, 40, None),
    "fista_2048": (2048, 2048, "L2", "FISTA", False, 8.0, 1, 30, None),
    "cp2_l1_mask": (90, 140, "L1", "CP2", True, 1.5, 2, 50, 1.0 / 400.0),
    "cp2_l2_const_steps": (70, 61, "L2", "CP2", False, 6.0, 1, 60, 0.0),
    "cv": (96, 100, "CV", "CP2", False, 10.0, 2, 40, 1.0 / 8.0),
}


@pytest.mark.parametrize("name", list(FULL))
def test_full_problem_parity(name):
    """full_problem = 1: one subdomain without the proximal term, i.e. the
    plain method on the whole dual problem, restarted every outer step."""
    H, W, fid, inner, masked, alpha, n_outer, n_inner, gamma = FULL[name]
    rng = np.random.default_rng(71 + list(FULL).index(name))
    clean = synth.shapes(H, W, rng)
    f = synth.salt_and_pepper(clean, 0.3, rng) if fid == "L1" else clean + synth.gaussian((H, W), 0.08, rng)
    mask = None
    if masked:
        mask = synth.stroke_mask(H, W, 0.1, rng)
        f = np.where(mask == 1, f, 0.0)
    f = f.astype(np.float32)
    rc, cc = [0, H], [0, W]
    _say(f"[full] {name} {H}x{W} {fid}/{inner} {n_outer}x{n_inner}")
    kw = dict(fidelity=fid, inner=inner, n_outer=n_outer, n_inner=n_inner, full_problem=True)
    if gamma is not None:
        kw["gamma"] = gamma
    if fid == "CV":
        kw.update(tau=1.0, sigma=0.5, c1=0.6, c2=0.1)
    plan, state, _ = run_gpu(f, alpha, rc, cc, mask=mask, **kw)
    okw = dict(fidelity=fid, inner=inner, mask=mask, n_inner=n_inner, no_prox_term=True)
    if gamma is not None:
        okw["gamma"] = gamma
    if fid == "CV":
        okw.update(c1=0.6, c2=0.1)
    o = oracle_for(f, alpha, rc, cc, **okw)
    o.run(n_outer)
    errs = compare(gpu_image_state(plan, state), o)
    _say(f"  errors {errs}")


def test_full_problem_ignores_tau():
    """Without the proximal term the outer step sizes play no part."""
    rng = np.random.default_rng(81)
    f = (synth.shapes(60, 70, rng) + synth.gaussian((60, 70), 0.1, rng)).astype(np.float32)
    outs = []
    for tau, sigma in ((50.0, 0.01), (1.0, 0.5)):
        plan, state, _ = run_gpu(f, 8.0, [0, 60], [0, 70], n_outer=2, n_inner=25, full_problem=True, tau=tau,
                                 sigma=sigma)
        outs.append(gpu_image_state(plan, state))
    for q in ("u", "P1", "P2"):
        assert np.array_equal(outs[0][q], outs[1][q]), q
