"""dtv_dd_solve_noalloc (the solve on the library's device scratch array, for
callers that cannot allocate) against dtv_dd_solve with a bound workspace:
the same kernels run, so u, p~ and the lambda state must be bitwise equal.
Two plans in a row on one device, the second with a smaller input, so the
second call re-uploads its metadata over the first one's; each plan is also
called twice (the second call finds its metadata in place)."""
import ctypes
import sys

import numpy as np
import pytest

from paper_1901_00682_amd import synth

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


def _inputs(H, W, seed, mask=False):
    rng = np.random.default_rng(seed)
    f = (synth.shapes(H, W, rng) + synth.gaussian((H, W), 0.1, rng)).astype(np.float32)
    m = None
    if mask:
        m = (rng.uniform(size=(H, W)) > 0.1).astype(np.uint8)
        f = np.where(m == 1, f, 0.0).astype(np.float32)
    return f, m


CASES = [
    # (name, H, W, row cuts, col cuts, plan keywords): the first the larger one
    ("persistent FISTA 512x640, 4x5 of 128^2", 512, 640, [0, 128, 256, 384, 512], [0, 128, 256, 384, 512, 640],
     dict(n_outer=60, n_inner=5, schedule="persistent")),
    ("streaming CP2 L1 + mask 200x300, ragged cuts", 200, 300, [0, 64, 128, 200], [0, 100, 200, 300],
     dict(n_outer=30, n_inner=5, schedule="stream", fidelity="L1", has_mask=True, inner="CP2", rows=8)),
]


def test_noalloc_equals_bound_workspace_on_two_plans_in_a_row():
    from paper_1901_00682_amd import dtvdd
    for k, (name, H, W, rc, cc, kw) in enumerate(CASES):
        _say(f"noalloc case {k}: {name}")
        f, m = _inputs(H, W, 70 + k, mask=kw.get("has_mask", False))
        ft = torch.from_numpy(f.ravel()).cuda()
        mt = None if m is None else torch.from_numpy(m.ravel()).cuda()
        im = dtvdd.Image(H, W, np.asarray(rc, np.int32), np.asarray(cc, np.int32), 8.0 if k == 0 else 1.5)
        ref_plan = dtvdd.Plan([im], **kw)
        ref, _ = ref_plan.solve(ft, mask=mt)
        torch.cuda.synchronize()
        plan = dtvdd.Plan([im], bind=False, **kw)   # no workspace at all
        nb = ctypes.c_size_t()
        assert dtvdd.lib().dtv_dd_workspace_bytes(plan.h, ctypes.byref(nb)) == 0
        assert nb.value <= dtvdd.SCRATCH_BYTES
        for call in range(2):
            got = plan.solve_noalloc(ft, mask=mt)
            torch.cuda.synchronize()
            for key in ("u", "p1", "p2", "lam"):
                assert torch.equal(ref[key], got[key]), (name, call, key)
            _say(f"  call {call}: bitwise equal (workspace {nb.value} bytes)")
        assert float(ref["u"].abs().max()) > 0 and float(ref["p1"].abs().max()) > 0
