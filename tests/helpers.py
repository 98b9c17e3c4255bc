"""Shared test helpers: run the GPU path and the oracle on the same seeded
input and compare them.  The oracle always receives the FP32 input the GPU
receives, widened to FP64."""
from __future__ import annotations

import numpy as np

import oracle


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def oracle_for(f32, alpha, row_cuts, col_cuts, *, fidelity="L2", inner="FISTA", mask=None, tau=50.0,
               sigma=0.01, tau0=10.0, sigma0=1 / 80, gamma=None, n_inner=10, **kw):
    return oracle.Oracle(oracle.Problem(np.asarray(f32, dtype=np.float64), float(alpha), np.asarray(row_cuts),
                                        np.asarray(col_cuts), fidelity=fidelity, inner=inner, mask=mask, tau=tau,
                                        sigma=sigma, tau0=tau0, sigma0=sigma0, gamma=gamma, n_inner=n_inner, **kw))


def gpu_image_state(plan, state, image=0):
    """Host copies (float64) of one image's u, P1, P2, lambda, prev_s, prev_t."""
    p1, p2 = plan.p_views(state, image)
    lam, ps, pt = plan.lam_view(state, image)
    c = lambda t: t.detach().cpu().numpy().astype(np.float64)
    return {"u": c(plan.u_view(state, image)), "P1": c(p1), "P2": c(p2), "lam": c(lam), "prev_s": c(ps),
            "prev_t": c(pt)}


def compare(gpu: dict, orc: "oracle.Oracle", tol_u=1e-5, tol_p=1e-5, tol_lam=1e-4):
    e = orc.export()
    Q1, Q2 = orc.to_torn(e["p"])
    err_u = rel_l2(gpu["u"], e["u"])
    err_p = rel_l2(np.concatenate([gpu["P1"].ravel(), gpu["P2"].ravel()]), np.concatenate([Q1.ravel(), Q2.ravel()]))
    err_lam = rel_l2(gpu["lam"], e["lam"]) if e["lam"].size else 0.0
    assert err_u <= tol_u, f"u rel L2 {err_u:.3e} > {tol_u}"
    assert err_p <= tol_p, f"p rel L2 {err_p:.3e} > {tol_p}"
    assert err_lam <= tol_lam, f"lambda rel L2 {err_lam:.3e} > {tol_lam}"
    # boundary (non-dof) edges are exactly zero
    assert not gpu["P1"][0].any() and not gpu["P1"][-1].any()
    assert not gpu["P2"][:, 0].any() and not gpu["P2"][:, -1].any()
    return {"u": err_u, "p": err_p, "lam": err_lam}
