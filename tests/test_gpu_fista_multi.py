"""The multi-step streaming launch of the local FISTA solver (fista_multi.hip:
steps k .. k + S - 1 of projected FISTA on the local dual problems of Sec. 5 in
one launch, S = 2 .. 5) against one-step launches, bitwise: ragged and
one-pixel subdomains (subdomain boundaries inside a strip, on the strip's halo
rows and on the waves' halo columns), every strip height, inner counts that cut
into one, two and three launches (the c' buffer written by the first launch and
read by the others, the first launch's x_0 buffer reused), images narrower than
a wave and one row high, and the undecomposed problem (one subdomain, many
steps in one outer step)."""
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


GEOMS = {
    # name: (H, W, row cuts, column cuts)
    "uneven": (90, 140, [0, 31, 60, 90], [0, 35, 70, 105, 140]),
    "thin": (70, 190, [0, 1, 2, 9, 10, 33, 70], [0, 1, 59, 60, 61, 62, 122, 123, 190]),
    "ragged": (123, 257, [0, 41, 82, 123], [0, 100, 200, 257]),
    "narrow": (37, 5, [0, 12, 37], [0, 2, 5]),
    "row": (1, 150, [0, 1], [0, 70, 150]),
    "col": (150, 1, [0, 64, 65, 150], [0, 1]),
}


def _input(H, W, seed):
    rng = np.random.default_rng(seed)
    return (synth.shapes(H, W, rng) + synth.gaussian((H, W), 0.1, rng)).astype(np.float32)


def _solve(f, rc, cc, alpha, spl, **kw):
    from paper_1901_00682_amd import dtvdd
    H, W = f.shape
    plan = dtvdd.Plan([dtvdd.Image(H, W, np.asarray(rc), np.asarray(cc), alpha)], schedule="stream",
                      steps_per_launch=spl, **kw)
    ft = torch.from_numpy(np.ascontiguousarray(f).ravel()).cuda()
    state, _ = plan.solve(ft)
    torch.cuda.synchronize()
    return plan, gpu_image_state(plan, state)


# inner counts and the launches steps-per-launch 2, 3, 4, 5 cut them into:
#   K = 2: 2;  K = 5: 2 2 1 | 3 2 | 3 2 | 5;  K = 4: 2 2 | 2 2 | 4 | 4;  K = 9: 2 2 2 2 1 | 3 3 3 | 3 3 3 | 5 4;
#   K = 12: 2 x 6 | 3 3 3 3 | 4 4 4 | 4 4 4
CASES = [(g, K, R) for g in ("uneven", "thin") for K, R in ((2, 4), (5, 8), (4, 16), (9, 32), (12, 8))]
CASES += [("ragged", 5, 16), ("ragged", 10, 32), ("narrow", 4, 4), ("narrow", 7, 32), ("row", 5, 8), ("row", 9, 4),
          ("col", 5, 16), ("col", 6, 4)]


@pytest.mark.parametrize("geom,K,R", CASES)
def test_multi_equals_one_step_launches_bitwise(geom, K, R):
    H, W, rc, cc = GEOMS[geom]
    f = _input(H, W, 13 * K + R + 5 * len(geom))
    _say(f"[fista multi] {geom} {H}x{W} K={K} R={R}")
    res = {}
    for spl in (1, 2, 3, 4, 5):
        _, res[spl] = _solve(f, rc, cc, 6.0, spl, n_outer=4, n_inner=K, rows=R)
    for spl in (2, 3, 4, 5):
        for q in res[1]:
            assert np.array_equal(res[1][q], res[spl][q]), (spl, q)


def test_undecomposed_problem_multi_equals_one_step_bitwise():
    """One subdomain, one outer step of 23 FISTA steps: launches of 5 5 5 4 4
    (the buffers rotate through x_0's buffer), 3 3 3 3 3 3 3 2 and 2 x 11 + 1."""
    H, W = 150, 170
    f = _input(H, W, 77)
    _say(f"[fista multi] undecomposed {H}x{W} 23 steps")
    res = {}
    for spl in (1, 2, 3, 5):
        _, res[spl] = _solve(f, [0, H], [0, W], 8.0, spl, full_problem=True, n_outer=1, n_inner=23, rows=8)
    for spl in (2, 3, 5):
        for q in res[1]:
            assert np.array_equal(res[1][q], res[spl][q]), (spl, q)


def test_multi_kernel_is_timed_and_named():
    H, W, rc, cc = GEOMS["uneven"]
    f = _input(H, W, 3)
    plan, _ = _solve(f, rc, cc, 6.0, 0, n_outer=3, n_inner=5, rows=8, time_kernels=True)
    kt = plan.kernel_time()
    assert kt["name"] == "k_fista_multi"
    assert kt["launches"] == 3  # all five steps in one launch per outer step
    plan2, _ = _solve(f, rc, cc, 6.0, 2, n_outer=3, n_inner=5, rows=8, time_kernels=True)
    assert plan2.kernel_time()["launches"] == 3 * 3
    plan1, _ = _solve(f, rc, cc, 6.0, 1, n_outer=3, n_inner=5, rows=8, time_kernels=True)
    assert plan1.kernel_time()["name"] == "k_fista_step"
    assert plan1.kernel_time()["launches"] == 3 * 5
    # all five steps in one launch: read p~ and f, write p~: 4 (2E + N) bytes
    assert kt["bytes_per_launch"] < plan1.kernel_time()["bytes_per_launch"]
