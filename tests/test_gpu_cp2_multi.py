"""The multi-step streaming launch of the local primal-dual solver (cp2_multi.hip:
steps k .. k + S - 1 of Chambolle-Pock Alg. 2 on the local problems of Sec. 5 in
one launch, S = 2 .. 5) against one-step launches, bitwise: every fidelity,
masks, ragged and one-pixel subdomains (subdomain boundaries inside a strip, on
the strip's halo rows and on the waves' halo columns), every strip height,
inner counts that cut into launches of every length, images narrower than a
wave and one row high; and the TV-L1 inpainting workload at full size against
the oracle."""
import sys

import numpy as np
import pytest

from paper_1901_00682_amd import synth
from tests.helpers import compare, gpu_image_state, oracle_for

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
    # subdomain boundaries one and two rows below a strip start, one-pixel subdomains, columns
    # across the waves' halo lanes (61 output columns per wave)
    "thin": (70, 190, [0, 1, 2, 9, 10, 33, 70], [0, 1, 59, 60, 61, 62, 122, 123, 190]),
    "ragged": (123, 257, [0, 41, 82, 123], [0, 100, 200, 257]),
    "narrow": (37, 5, [0, 12, 37], [0, 2, 5]),
    "row": (1, 150, [0, 1], [0, 70, 150]),
    "col": (150, 1, [0, 64, 65, 150], [0, 1]),
}

FIDS = {
    "L2": dict(fidelity="L2", inner="CP2", alpha=6.0, mask=False),
    "L1_mask": dict(fidelity="L1", inner="CP2", alpha=1.5, mask=True, gamma=1.0 / 400.0),
    "CV": dict(fidelity="CV", inner="CP2", alpha=10.0, mask=False, tau=1.0, sigma=0.5, gamma=1.0 / 8.0, c1=0.6, c2=0.1),
}


def _input(H, W, seed, masked):
    rng = np.random.default_rng(seed)
    clean = synth.shapes(H, W, rng)
    f = (clean + synth.gaussian((H, W), 0.1, rng)).astype(np.float32)
    mask = synth.stroke_mask(H, W, 0.1, rng) if masked else None
    if masked:
        f = np.where(mask == 1, f, 0.0).astype(np.float32)
    return f, mask


def _solve(f, mask, rc, cc, alpha, spl, **kw):
    from paper_1901_00682_amd import dtvdd
    H, W = f.shape
    plan = dtvdd.Plan([dtvdd.Image(H, W, np.asarray(rc), np.asarray(cc), alpha)], has_mask=mask is not None,
                      schedule="stream", steps_per_launch=spl, **kw)
    ft = torch.from_numpy(np.ascontiguousarray(f).ravel()).cuda()
    mt = None if mask is None else torch.from_numpy(np.ascontiguousarray(mask, dtype=np.uint8).ravel()).cuda()
    state, _ = plan.solve(ft, mt)
    torch.cuda.synchronize()
    return plan, gpu_image_state(plan, state)


# inner counts and the launches the steps-per-launch values 2, 3, 4, 5 cut them into:
#   K = 2: 2 | 2 | 2 | 2;  K = 5: 2 2 1 | 3 2 | 3 2 | 5;  K = 4: 2 2 | 2 2 | 4 | 4;  K = 9: 2 2 2 2 1 | 3 3 3 | 3 3 3 | 5 4
CASES = [(g, fid, K, R) for g in ("uneven", "thin") for fid in FIDS for K, R in ((2, 4), (5, 8), (4, 16), (9, 32))]
CASES += [("ragged", "L1_mask", 5, 8), ("ragged", "CV", 7, 16), ("narrow", "L2", 4, 4), ("narrow", "L1_mask", 5, 32),
          ("row", "L2", 5, 8), ("row", "CV", 9, 4), ("col", "L1_mask", 5, 16), ("col", "L2", 6, 4)]


@pytest.mark.parametrize("geom,fid,K,R", CASES)
def test_multi_equals_one_step_launches_bitwise(geom, fid, K, R):
    H, W, rc, cc = GEOMS[geom]
    kw = dict(FIDS[fid])
    alpha, masked = kw.pop("alpha"), kw.pop("mask")
    f, mask = _input(H, W, 11 * K + R + 7 * len(geom), masked)
    _say(f"[cp2 multi] {geom} {H}x{W} {fid} K={K} R={R}")
    res = {}
    for spl in (1, 2, 3, 4, 5):
        plan, res[spl] = _solve(f, mask, rc, cc, alpha, spl, n_outer=4, n_inner=K, rows=R, **kw)
    for spl in (2, 3, 4, 5):
        for q in res[1]:
            assert np.array_equal(res[1][q], res[spl][q]), (spl, q)


def test_multi_kernel_is_timed_and_named():
    H, W, rc, cc = GEOMS["uneven"]
    f, mask = _input(H, W, 3, True)
    kw = dict(FIDS["L1_mask"])
    alpha = kw.pop("alpha")
    kw.pop("mask")
    plan, _ = _solve(f, mask, rc, cc, alpha, 2, n_outer=3, n_inner=5, rows=8, time_kernels=True, **kw)
    kt = plan.kernel_time()
    assert kt["name"] == "k_cp2_multi"
    assert kt["launches"] == 3 * 3  # two two-step launches and one one-step launch per outer step
    plan5, _ = _solve(f, mask, rc, cc, alpha, 5, n_outer=3, n_inner=5, rows=8, time_kernels=True, **kw)
    assert plan5.kernel_time()["name"] == "k_cp2_multi"
    assert plan5.kernel_time()["launches"] == 3
    plan1, _ = _solve(f, mask, rc, cc, alpha, 1, n_outer=3, n_inner=5, rows=8, time_kernels=True, **kw)
    assert plan1.kernel_time()["name"] == "k_cp2_step"
    assert plan1.kernel_time()["launches"] == 3 * 5
    assert plan1.kernel_time()["bytes_per_launch"] > kt["bytes_per_launch"] * 0.5


def test_multi_tvl1_workload_against_the_oracle():
    """TV-L1 + inpainting mask, 2000 x 3000, 13 x 20 uneven subdomains, CP2 x 5,
    on launches of 2 + 2 + 1, 3 + 2 and 5 steps (strips of 8 and 16 rows): the
    first 30 outer steps against the FP64 oracle, and bitwise equal to one-step
    launches."""
    from paper_1901_00682_amd import dtvdd
    c = synth.config3()
    H, W = c.f.shape
    n_outer = 30
    _say(f"[cp2 multi] config3 {H}x{W} 13x20 TV-L1+mask {n_outer}x{c.n_inner}")
    ft = torch.from_numpy(np.ascontiguousarray(c.f, dtype=np.float32).ravel()).cuda()
    mt = torch.from_numpy(np.ascontiguousarray(c.mask, dtype=np.uint8).ravel()).cuda()
    res = {}
    for spl, R in ((5, 16), (3, 8), (2, 8), (1, 8)):
        plan = dtvdd.Plan([dtvdd.Image(H, W, c.row_cuts, c.col_cuts, c.alpha)], has_mask=True, fidelity="L1",
                          inner="CP2", n_outer=n_outer, n_inner=c.n_inner, schedule="stream", rows=R,
                          steps_per_launch=spl)
        state, _ = plan.solve(ft, mt)
        torch.cuda.synchronize()
        res[spl] = gpu_image_state(plan, state)
    for spl in (2, 3, 5):
        for q in res[1]:
            assert np.array_equal(res[1][q], res[spl][q]), (spl, q)
    o = oracle_for(c.f, c.alpha, c.row_cuts, c.col_cuts, fidelity="L1", inner="CP2", mask=c.mask, n_inner=c.n_inner)
    o.run(n_outer)
    errs = compare(res[5], o)
    _say(f"  errors {errs}")
