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


def interface_errors(gpu: dict, orc: "oracle.Oracle", e: dict | None = None):
    """Per interface segment (the side shared by two neighbouring subdomains):
    the L2 error and the L2 norm of its two copies of p~ together and of its
    multipliers, and the largest absolute error on the copies.  Returns a list
    of (name, n_dofs, err_p, norm_p, err_lam, norm_lam, max_abs_p)."""
    e = orc.export() if e is None else e
    Q1, Q2 = orc.to_torn(e["p"])
    lam_h, lam_v = orc.lam_split(e["lam"])
    H, W = orc.H, orc.W
    glam = np.asarray(gpu["lam"], dtype=np.float64)
    g_h = glam[: (orc.ny - 1) * W].reshape(orc.ny - 1, W)
    g_v = glam[(orc.ny - 1) * W:].reshape(orc.nx - 1, H)
    rc, cc = [int(x) for x in orc.row_cuts], [int(x) for x in orc.col_cuts]
    segs = []
    for r in range(1, orc.ny):
        k = rc[r] + r          # torn P1 row of the t copy; the s copy is the row above
        for c in range(orc.nx):
            a, b = cc[c], cc[c + 1]
            segs.append((f"h{r}.{c}", gpu["P1"][k - 1: k + 1, a:b], Q1[k - 1: k + 1, a:b], g_h[r - 1, a:b],
                         lam_h[r - 1, a:b]))
    for c in range(1, orc.nx):
        k = cc[c] + c          # torn P2 column of the t copy
        for r in range(orc.ny):
            a, b = rc[r], rc[r + 1]
            segs.append((f"v{c}.{r}", gpu["P2"][a:b, k - 1: k + 1], Q2[a:b, k - 1: k + 1], g_v[c - 1, a:b],
                         lam_v[c - 1, a:b]))
    out = []
    for name, g, q, gl, ql in segs:
        d = np.asarray(g, dtype=np.float64) - q
        out.append((name, q.size, float(np.linalg.norm(d)), float(np.linalg.norm(q)),
                    float(np.linalg.norm(gl - ql)), float(np.linalg.norm(ql)), float(np.abs(d).max())))
    return out


def compare(gpu: dict, orc: "oracle.Oracle", tol_u=1e-5, tol_p=1e-5, tol_lam=1e-4, tol_if_p=1e-4, tol_if_lam=1e-3):
    """Relative L2 over every pixel (u), every dof (p~) and every multiplier,
    then per interface segment (interface_errors) at ten times those bars.

    A global relative L2 over every dof could hide a wrong segment (a hundred
    dofs among millions).  A segment's error is measured against the larger of
    its own norm and the global root-mean-square value times the square root of
    its size (so that a segment whose copies are nearly all zero is not judged
    by a vanishing norm): a few 1e-4 on every dof of one segment fails."""
    e = orc.export()
    Q1, Q2 = orc.to_torn(e["p"])
    err_u = rel_l2(gpu["u"], e["u"])
    gp = np.concatenate([gpu["P1"].ravel(), gpu["P2"].ravel()])
    op = np.concatenate([Q1.ravel(), Q2.ravel()])
    err_p = rel_l2(gp, op)
    err_lam = rel_l2(gpu["lam"], e["lam"]) if e["lam"].size else 0.0
    assert err_u <= tol_u, f"u rel L2 {err_u:.3e} > {tol_u}"
    assert err_p <= tol_p, f"p rel L2 {err_p:.3e} > {tol_p}"
    assert err_lam <= tol_lam, f"lambda rel L2 {err_lam:.3e} > {tol_lam}"
    worst_p = worst_lam = worst_abs = 0.0
    if e["lam"].size:
        rms_p = np.linalg.norm(op) / np.sqrt(max(np.count_nonzero(op), 1))
        rms_l = np.linalg.norm(e["lam"]) / np.sqrt(e["lam"].size)
        for name, n, ep, np_, el, nl, ea in interface_errors(gpu, orc, e):
            rp = ep / max(np_, rms_p * np.sqrt(n), 1e-30)
            rl = el / max(nl, rms_l * np.sqrt(n / 2), 1e-30)
            assert rp <= tol_if_p, (f"interface segment {name}: p~ copies error {ep:.3e}, norm {np_:.3e} "
                                    f"(relative {rp:.3e} > {tol_if_p}), max abs {ea:.3e}")
            assert rl <= tol_if_lam, (f"interface segment {name}: lambda error {el:.3e}, norm {nl:.3e} "
                                      f"(relative {rl:.3e} > {tol_if_lam})")
            worst_p, worst_lam, worst_abs = max(worst_p, rp), max(worst_lam, rl), max(worst_abs, ea)
    # boundary (non-dof) edges are exactly zero
    assert not gpu["P1"][0].any() and not gpu["P1"][-1].any()
    assert not gpu["P2"][:, 0].any() and not gpu["P2"][:, -1].any()
    return {"u": err_u, "p": err_p, "lam": err_lam, "if_p": worst_p, "if_lam": worst_lam, "if_abs_p": worst_abs}
