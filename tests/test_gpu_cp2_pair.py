"""The two-step streaming launch of the local primal-dual solver (cp2_pair.hip:
steps k and k + 1 of Chambolle-Pock Alg. 2 on the local problems of Sec. 5 in
one launch) against one-step launches, bitwise: every fidelity, masks, ragged
and one-pixel subdomains (subdomain boundaries inside a strip, on the strip's
halo rows and on the waves' halo columns), every strip height, odd and even
inner counts, images narrower than a wave and one row high; and the TV-L1
inpainting workload at full size against the oracle."""
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


CASES = [(g, fid, K, R) for g in ("uneven", "thin") for fid in FIDS for K, R in ((2, 4), (5, 8), (6, 16), (7, 32))]
CASES += [("ragged", "L1_mask", 5, 8), ("ragged", "CV", 3, 16), ("narrow", "L2", 4, 4), ("narrow", "L1_mask", 5, 32),
          ("row", "L2", 5, 8), ("row", "CV", 2, 4), ("col", "L1_mask", 3, 16), ("col", "L2", 6, 4)]


@pytest.mark.parametrize("geom,fid,K,R", CASES)
def test_pair_equals_one_step_launches_bitwise(geom, fid, K, R):
    H, W, rc, cc = GEOMS[geom]
    kw = dict(FIDS[fid])
    alpha, masked = kw.pop("alpha"), kw.pop("mask")
    f, mask = _input(H, W, 11 * K + R + 7 * len(geom), masked)
    _say(f"[cp2 pair] {geom} {H}x{W} {fid} K={K} R={R}")
    res = {}
    for spl in (1, 2):
        plan, res[spl] = _solve(f, mask, rc, cc, alpha, spl, n_outer=4, n_inner=K, rows=R, **kw)
    for q in res[1]:
        assert np.array_equal(res[1][q], res[2][q]), q


def test_pair_kernel_is_timed_and_named():
    H, W, rc, cc = GEOMS["uneven"]
    f, mask = _input(H, W, 3, True)
    kw = dict(FIDS["L1_mask"])
    alpha = kw.pop("alpha")
    kw.pop("mask")
    plan, _ = _solve(f, mask, rc, cc, alpha, 0, n_outer=3, n_inner=5, rows=8, time_kernels=True, **kw)
    kt = plan.kernel_time()
    assert kt["name"] == "k_cp2_pair"
    assert kt["launches"] == 3 * 3  # two pairs and one single step per outer step
    plan1, _ = _solve(f, mask, rc, cc, alpha, 1, n_outer=3, n_inner=5, rows=8, time_kernels=True, **kw)
    assert plan1.kernel_time()["name"] == "k_cp2_step"
    assert plan1.kernel_time()["bytes_per_launch"] > kt["bytes_per_launch"] * 0.5


def test_pair_tvl1_workload_against_the_oracle():
    """TV-L1 + inpainting mask, 2000 x 3000, 13 x 20 uneven subdomains, CP2 x 5,
    on the two-step launches (the autotuner's strip height): the first 30 outer
    steps against the FP64 oracle, and bitwise equal to one-step launches."""
    from paper_1901_00682_amd import dtvdd
    c = synth.config3()
    H, W = c.f.shape
    n_outer = 30
    _say(f"[cp2 pair] config3 {H}x{W} 13x20 TV-L1+mask {n_outer}x{c.n_inner}")
    ft = torch.from_numpy(np.ascontiguousarray(c.f, dtype=np.float32).ravel()).cuda()
    mt = torch.from_numpy(np.ascontiguousarray(c.mask, dtype=np.uint8).ravel()).cuda()
    res = {}
    for spl in (2, 1):
        plan = dtvdd.Plan([dtvdd.Image(H, W, c.row_cuts, c.col_cuts, c.alpha)], has_mask=True, fidelity="L1",
                          inner="CP2", n_outer=n_outer, n_inner=c.n_inner, schedule="stream", rows=8,
                          steps_per_launch=spl)
        state, _ = plan.solve(ft, mt)
        torch.cuda.synchronize()
        res[spl] = gpu_image_state(plan, state)
    for q in res[1]:
        assert np.array_equal(res[1][q], res[2][q]), q
    o = oracle_for(c.f, c.alpha, c.row_cuts, c.col_cuts, fidelity="L1", inner="CP2", mask=c.mask, n_inner=c.n_inner)
    o.run(n_outer)
    errs = compare(res[2], o)
    _say(f"  errors {errs}")
