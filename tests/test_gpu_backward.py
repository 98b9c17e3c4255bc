"""Reverse mode on the GPU (through the C-ABI) against the FP64 oracle's
reverse pass, which is pinned by finite differences in test_oracle_reverse.py."""
import sys

import numpy as np
import pytest

import oracle
from paper_1901_00682_amd import synth
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def gpu_grad(fs, alphas, rc, cc, ubars, n_outer, K, ckpt_every, schedule="auto", **kw):
    from paper_1901_00682_amd import dtvdd
    H, W = fs[0].shape
    plan = dtvdd.Plan([dtvdd.Image(H, W, rc, cc, a) for a in alphas], n_outer=n_outer, n_inner=K,
                      save_for_backward=True, ckpt_every=ckpt_every, schedule=schedule, **kw)
    f = torch.from_numpy(np.concatenate([x.ravel() for x in fs]).astype(np.float32)).cuda()
    st, _ = plan.solve(f, want_stats=False)
    gu = torch.from_numpy(np.concatenate([x.ravel() for x in ubars]).astype(np.float32)).cuda()
    gf, ga = plan.backward(f, gu)
    torch.cuda.synchronize()
    return gf.cpu().numpy().astype(np.float64).reshape(len(fs), H, W), ga.cpu().numpy().astype(np.float64), plan, st


@pytest.mark.parametrize("H,W,rc,cc,alpha,n_outer,K,C", [
    (64, 64, [0, 16, 32, 48, 64], [0, 16, 32, 48, 64], 8.0, 30, 5, 7),
    (50, 73, [0, 20, 50], [0, 1, 40, 73], 5.0, 12, 4, 5),
    (40, 40, [0, 40], [0, 40], 10.0, 10, 3, 20),
])
def test_backward_matches_oracle(H, W, rc, cc, alpha, n_outer, K, C):
    _say(f"[backward] {H}x{W} grid {len(rc)-1}x{len(cc)-1} {n_outer}x{K} ckpt {C}")
    rng = np.random.default_rng(H + W)
    g = synth.shapes(H, W, rng)
    f = (g + synth.gaussian((H, W), 0.1, rng)).astype(np.float32)
    ubar = rng.standard_normal((H, W))
    gf, ga, _, _ = gpu_grad([f], [alpha], np.array(rc), np.array(cc), [ubar], n_outer, K, C)
    o = oracle.Oracle(oracle.Problem(f.astype(np.float64), alpha, np.array(rc), np.array(cc), n_inner=K))
    fbar, abar = o.backward(n_outer, ubar.astype(np.float32).astype(np.float64))
    e_f = rel_l2(gf[0], fbar)
    e_a = abs(ga[0] - abar) / abs(abar)
    _say(f"  dl/df rel L2 {e_f:.2e}   dl/dalpha rel {e_a:.2e}")
    assert e_f <= 1e-4
    assert e_a <= 1e-4


def test_backward_independent_of_checkpoint_spacing():
    H = W = 48
    rc = cc = np.array([0, 16, 32, 48])
    rng = np.random.default_rng(9)
    f = (synth.shapes(H, W, rng) + synth.gaussian((H, W), 0.1, rng)).astype(np.float32)
    ubar = rng.standard_normal((H, W))
    res = [gpu_grad([f], [8.0], rc, cc, [ubar], 13, 5, C) for C in (1, 4, 13, 50)]
    for r in res[1:]:
        assert np.array_equal(r[0], res[0][0]) and np.array_equal(r[1], res[0][1])


def test_backward_batched_equals_single():
    H, W = 40, 56
    rc, cc = np.array([0, 20, 40]), np.array([0, 28, 56])
    rng = np.random.default_rng(11)
    fs = [(synth.shapes(H, W, rng) + synth.gaussian((H, W), 0.1, rng)).astype(np.float32) for _ in range(3)]
    ub = [rng.standard_normal((H, W)) for _ in range(3)]
    alphas = [4.0, 8.0, 12.0]
    gfb, gab, _, _ = gpu_grad(fs, alphas, rc, cc, ub, 10, 5, 4)
    for b in range(3):
        gf1, ga1, _, _ = gpu_grad([fs[b]], [alphas[b]], rc, cc, [ub[b]], 10, 5, 4)
        assert np.array_equal(gfb[b], gf1[0])
        assert np.array_equal(gab[b], ga1[0])


def test_autograd_function():
    from paper_1901_00682_amd import dtvdd
    H = W = 32
    rng = np.random.default_rng(12)
    g = synth.shapes(H, W, rng)
    f0 = (g + synth.gaussian((H, W), 0.1, rng)).astype(np.float32)
    f = torch.from_numpy(f0).cuda().requires_grad_(True)
    alpha = torch.tensor(8.0, requires_grad=True)
    gt = torch.from_numpy(g.astype(np.float32)).cuda()
    u = dtvdd.DTVDD.apply(f, alpha, (2, 2), 15, 5, 5)
    loss = ((u - gt) ** 2).sum()
    loss.backward()
    o = oracle.Oracle(oracle.Problem(f0.astype(np.float64), 8.0, np.array([0, 16, 32]), np.array([0, 16, 32]), n_inner=5))
    o.run(15)
    u_o = o.export()["u"]
    o2 = oracle.Oracle(oracle.Problem(f0.astype(np.float64), 8.0, np.array([0, 16, 32]), np.array([0, 16, 32]), n_inner=5))
    fbar, abar = o2.backward(15, 2.0 * (u_o - g))
    assert rel_l2(f.grad.cpu().numpy(), fbar) <= 1e-4
    assert abs(float(alpha.grad) - abar) <= 1e-4 * abs(abar)


def test_backward_without_saved_forward_is_an_error():
    from paper_1901_00682_amd import dtvdd
    plan = dtvdd.Plan([dtvdd.Image(16, 16, np.array([0, 16]), np.array([0, 16]), 8.0)], n_outer=2, n_inner=2,
                      save_for_backward=True, ckpt_every=1)
    f = torch.zeros(256, device="cuda")
    with pytest.raises(dtvdd.DtvError) as ei:
        plan.backward(f, f)
    assert ei.value.code == dtvdd.DTV_ESTATE


def test_autograd_function_keep_records_equals_checkpoints():
    """DTVDD with keep_records (the forward keeps every outer step's records) on
    a batch of 128 x 128 subdomains: the same u and gradients, bitwise, as with
    checkpoints."""
    from paper_1901_00682_amd import dtvdd
    B, H, W = 2, 256, 384
    rng = np.random.default_rng(44)
    fb = np.stack([(synth.shapes(H, W, rng) + synth.gaussian((H, W), 0.1, rng)) for _ in range(B)]).astype(np.float32)
    gt = torch.from_numpy(rng.standard_normal((B, H, W)).astype(np.float32)).cuda()
    res = []
    for keep in (False, True):
        f = torch.from_numpy(fb).cuda().requires_grad_(True)
        alpha = torch.tensor([6.0, 9.0], requires_grad=True)
        u = dtvdd.DTVDD.apply(f, alpha, (2, 3), 9, 5, 4, 50.0, 0.01, "auto", keep)
        ((u - gt) ** 2).sum().backward()
        torch.cuda.synchronize()
        res.append((u.detach().cpu(), f.grad.cpu(), alpha.grad.clone()))
    for a, b in zip(res[0], res[1]):
        assert torch.equal(a, b)
