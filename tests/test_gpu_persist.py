"""The persistent schedule (every outer step in one cooperative launch, the
iterates kept on chip between outer steps) against the fused and streaming
schedules, bitwise, and against the FP64 oracle: full-tile geometries with
image boundaries on every combination of sides, smaller subdomains run in a
128 x 128 frame (short sides on the image boundary or interfaces), several
images in one plan,
odd and even inner counts (unrolled and generic kernels), resume from a
returned state."""
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


def _image(H, W, seed):
    rng = np.random.default_rng(seed)
    return (synth.shapes(H, W, rng) + synth.gaussian((H, W), 0.1, rng)).astype(np.float32)


def _solve(imgs, fs, schedule, n_outer, K, state=None, warm=False):
    from paper_1901_00682_amd import dtvdd
    plan = dtvdd.Plan(imgs, n_outer=n_outer, n_inner=K, schedule=schedule, warm_start=warm)
    f = torch.from_numpy(np.concatenate([x.ravel() for x in fs])).cuda()
    st, _ = plan.solve(f, state=state)
    torch.cuda.synchronize()
    return plan, st, f


GEOMS = {
    "full3x3": (384, 384, [0, 128, 256, 384], [0, 128, 256, 384]),
    "full1x1": (128, 128, [0, 128], [0, 128]),
    "full2x4": (256, 512, [0, 128, 256], [0, 128, 256, 384, 512]),
    # framed tiles: the last subdomain row (43 rows) and column (45 columns) end on the image boundary
    "framed3x3": (299, 301, [0, 128, 256, 299], [0, 128, 256, 301]),
    # one framed tile alone (smaller than 128 x 128 on all sides)
    "framed1x1": (77, 100, [0, 77], [0, 100]),
    # framed tiles with interfaces on their short sides (masks): ragged cuts beside full tiles
    "mixed": (300, 357, [0, 128, 256, 300], [0, 101, 229, 357]),
    # equal cuts below 128 (127 rows; 127 or 128 columns)
    "floor": (381, 383, [0, 127, 254, 381], [0, 128, 255, 383]),
    # subdomains one pixel high or wide between two interfaces
    "thin": (257, 257, [0, 128, 129, 257], [0, 128, 129, 257]),
    # 120 rows (the bottom edges open a strip), 64 and 8 columns (the right edges in column a)
    "strip8": (360, 200, [0, 120, 240, 360], [0, 64, 192, 200]),
}


@pytest.mark.parametrize("geom,K,n_outer", [("full3x3", 1, 5), ("full3x3", 2, 6), ("full3x3", 5, 7),
                                            ("full3x3", 11, 3), ("full1x1", 3, 4), ("full2x4", 4, 9),
                                            ("full2x4", 10, 2), ("framed3x3", 5, 6), ("framed3x3", 2, 4),
                                            ("framed3x3", 9, 3), ("framed1x1", 4, 5), ("mixed", 5, 6),
                                            ("mixed", 9, 3), ("floor", 5, 5), ("floor", 2, 4), ("thin", 3, 6),
                                            ("strip8", 5, 5), ("strip8", 4, 3)])
def test_persistent_equals_fused_bitwise(geom, K, n_outer):
    from paper_1901_00682_amd import dtvdd
    H, W, rc, cc = GEOMS[geom]
    f = _image(H, W, 7 + K + n_outer)
    _say(f"[persist==fused] {geom} K={K} n_outer={n_outer}")
    res = {}
    for sch in ("persistent", "fused", "stream"):
        plan, st, _ = _solve([dtvdd.Image(H, W, rc, cc, 8.0)], [f], sch, n_outer, K)
        assert plan.schedule() == sch
        res[sch] = gpu_image_state(plan, st)
    for sch in ("fused", "stream"):
        for q in res["persistent"]:
            assert np.array_equal(res["persistent"][q], res[sch][q]), (sch, q)
    o = oracle_for(f, 8.0, np.array(rc), np.array(cc), n_inner=K)
    o.run(n_outer)
    compare(res["persistent"], o)


def test_persistent_several_images():
    """Two images of different sizes (all tiles full) in one persistent launch
    equal each image solved alone."""
    from paper_1901_00682_amd import dtvdd
    shapes = [(256, 384), (384, 256)]
    imgs = [dtvdd.Image(H, W, synth.tile_cuts(H, 128), synth.tile_cuts(W, 128), 5.0 + 3 * k)
            for k, (H, W) in enumerate(shapes)]
    fs = [_image(H, W, 40 + k) for k, (H, W) in enumerate(shapes)]
    _say("[persist] two images")
    plan, st, _ = _solve(imgs, fs, "persistent", 6, 5)
    assert plan.schedule() == "persistent"
    for k in range(2):
        one, st1, _ = _solve([imgs[k]], [fs[k]], "fused", 6, 5)
        a, b = gpu_image_state(plan, st, k), gpu_image_state(one, st1)
        for q in a:
            assert np.array_equal(a[q], b[q]), (k, q)


def test_persistent_groups_of_images():
    """Three images of 90 subdomains each (full and framed tiles) do not fit on the device at
    once: the persistent schedule runs them as groups of launches and equals the fused
    schedule bitwise."""
    from paper_1901_00682_amd import dtvdd
    H, W = 1100, 1200
    imgs = [dtvdd.Image(H, W, synth.tile_cuts(H, 128), synth.tile_cuts(W, 128), 4.0 + 2 * k) for k in range(3)]
    fs = [_image(H, W, 70 + k) for k in range(3)]
    _say("[persist] three images, 270 subdomains, groups of launches")
    pp, sp, _ = _solve(imgs, fs, "persistent", 4, 5)
    assert pp.schedule() == "persistent"
    pf, sf, _ = _solve(imgs, fs, "fused", 4, 5)
    for k in ("u", "p1", "p2", "lam"):
        assert torch.equal(sp[k], sf[k]), k


def test_persistent_groups_of_images_masked_frames():
    """Three images cut into 9 x 10 equal subdomains (122 x 120 and 123 x 120: framed, with
    interfaces on their short sides), 270 subdomains in groups of launches: the persistent
    schedule equals the fused one bitwise."""
    from paper_1901_00682_amd import dtvdd
    H, W = 1100, 1200
    imgs = [dtvdd.Image(H, W, synth.floor_cuts(H, 9), synth.floor_cuts(W, 10), 4.0 + 2 * k) for k in range(3)]
    fs = [_image(H, W, 80 + k) for k in range(3)]
    _say("[persist] three images, 270 masked framed subdomains, groups of launches")
    pp, sp, _ = _solve(imgs, fs, "persistent", 4, 5)
    assert pp.schedule() == "persistent"
    pf, sf, _ = _solve(imgs, fs, "fused", 4, 5)
    for k in ("u", "p1", "p2", "lam"):
        assert torch.equal(sp[k], sf[k]), k


def test_persistent_resume_bitwise():
    """3 + 4 outer steps through the returned state equal 7 in one launch."""
    from paper_1901_00682_amd import dtvdd
    H, W, rc, cc = GEOMS["full3x3"]
    f = _image(H, W, 99)
    im = dtvdd.Image(H, W, rc, cc, 6.0)
    _say("[persist] resume")
    p7, s7, _ = _solve([im], [f], "persistent", 7, 5)
    p3, s3, _ = _solve([im], [f], "persistent", 3, 5)
    p4, s4, _ = _solve([im], [f], "persistent", 4, 5, state=s3, warm=True)
    for k in ("u", "p1", "p2", "lam"):
        assert torch.equal(s7[k], s4[k]), k


def test_persistent_config2():
    """2048 x 2048, 16 x 16 subdomains of 128 x 128, 500 outer x 5 FISTA: the
    persistent launch equals the fused schedule bitwise."""
    from paper_1901_00682_amd import dtvdd
    c = synth.config2()
    H, W = c.f.shape
    im = dtvdd.Image(H, W, c.row_cuts, c.col_cuts, c.alpha)
    _say("[persist] config2 persistent vs fused")
    pp, sp, _ = _solve([im], [c.f], "persistent", c.n_outer, c.n_inner)
    pf, sf, _ = _solve([im], [c.f], "fused", c.n_outer, c.n_inner)
    for k in ("u", "p1", "p2", "lam"):
        assert torch.equal(sp[k], sf[k]), k


def test_persistent_floor_cuts_full_size():
    """2000 x 2000 cut into 16 x 16 equal subdomains of 125 x 125 (every one framed, with
    interfaces on its short sides), 500 outer x 5 FISTA: the persistent launch equals the fused
    and streaming schedules bitwise."""
    from paper_1901_00682_amd import dtvdd
    H = W = 2000
    rc = cc = synth.floor_cuts(H, 16)
    f = _image(H, W, 2000)
    im = dtvdd.Image(H, W, rc, cc, 8.0)
    _say("[persist] 2000x2000 16x16 floor cuts, persistent vs fused vs stream")
    res = {}
    for sch in ("persistent", "fused", "stream"):
        plan, st, _ = _solve([im], [f], sch, 500, 5)
        assert plan.schedule() == sch
        res[sch] = st
    for sch in ("fused", "stream"):
        for k in ("u", "p1", "p2", "lam"):
            assert torch.equal(res["persistent"][k], res[sch][k]), (sch, k)


def test_persistent_rejected_when_not_applicable():
    from paper_1901_00682_amd import dtvdd
    with pytest.raises(dtvdd.DtvError):  # a subdomain wider than 128
        dtvdd.Plan([dtvdd.Image(300, 357, [0, 128, 256, 300], [0, 200, 357], 8.0)], n_outer=2,
                   schedule="persistent")
    with pytest.raises(dtvdd.DtvError):  # ragged tiles, primal-dual local solves (full tiles only)
        dtvdd.Plan([dtvdd.Image(300, 357, [0, 128, 256, 300], [0, 101, 229, 357], 8.0)], n_outer=2,
                   schedule="persistent", inner="CP2")
    with pytest.raises(dtvdd.DtvError):  # per-step diagnostics
        dtvdd.Plan([dtvdd.Image(256, 256, [0, 128, 256], [0, 128, 256], 8.0)], n_outer=2, diag_every=1,
                   schedule="persistent")


@pytest.mark.parametrize("inner", ["FISTA", "CP2"])
def test_exchange_timeout_is_reported(inner):
    """The persistent schedules' waits are bounded; a poll limit of 1, forced
    from the host, makes a wait give up unless the neighbour's word is already
    there.  The solve then either completes and equals the normal solve, or
    returns DTV_EHIP naming the timeout (every tile leaves its loop, so the
    launch drains); a normal solve afterwards is unaffected."""
    from paper_1901_00682_amd import dtvdd
    H, W, rc, cc = GEOMS["full3x3"]
    f = _image(H, W, 99)
    ft = torch.from_numpy(f.ravel()).cuda()
    im = dtvdd.Image(H, W, rc, cc, 8.0)
    kw = dict(n_outer=20, n_inner=5, schedule="persistent", inner=inner)
    ref, _ = dtvdd.Plan([im], **kw).solve(ft)
    torch.cuda.synchronize()
    try:
        got, _ = dtvdd.Plan([im], spin_limit=1, **kw).solve(ft)
        torch.cuda.synchronize()
        for k in ("u", "p1", "p2", "lam"):
            assert torch.equal(ref[k], got[k]), k
        _say("  spin limit 1: every word was there in time")
    except dtvdd.DtvError as e:
        assert e.code == dtvdd.DTV_EHIP and "timed out" in str(e)
        _say(f"  spin limit 1: {e}")
    again, _ = dtvdd.Plan([im], **kw).solve(ft)
    torch.cuda.synchronize()
    for k in ("u", "p1", "p2", "lam"):
        assert torch.equal(ref[k], again[k]), k
