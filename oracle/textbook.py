"""Textbook solvers on the undecomposed problem, used to pin the oracle.

TEST INFRASTRUCTURE ONLY (imported by the tests, never by the product path).

Nothing here calls the C oracle: these are independent global-array
formulations written from the textbook definitions, so that a mistake in the
oracle's decomposition (a dropped term, a wrong sign or index, a transposed
copy) shows up as a disagreement.

  * the forward differences D of eq. (FFD) and the discrete divergence
    div = -D^T (Chambolle's convention), which by Prop. equiv is the RT0
    divergence of Sec. 2.3;
  * projected FISTA (Beck & Teboulle 2009) on the full dual ROF problem;
  * the accelerated primal-dual method (Chambolle & Pock 2011, Alg. 2) on the
    full saddle problem eq. (model_pd);
  * exact references on tiny images: the dual ROF problem as a box-constrained
    least-squares problem (solved by BVLS, certified by the KKT conditions),
    TV-L1 (with or without inpainting mask) and the convex Chan-Vese model
    eq. (CCV) as linear programs, and the binary Chan-Vese problem by
    enumeration of every pixel set;
  * the decomposed saddle problem (DD) of Sec. 4 on one global torn vector,
    with matrices of the torn divergence and of B built from their
    definitions, iterated by the textbook Chambolle-Pock method (their
    Alg. 1) with every proximal step solved exactly by BVLS, so that sigma,
    tau and the proximal weight 1/tau enter exactly as the textbook states
    them.
"""
from __future__ import annotations

import numpy as np


def fd_grad(u):
    """Forward differences, eq. (FFD): returns (D1 [(H-1) x W], D2 [H x (W-1)])
    holding only the differences that are not identically zero."""
    u = np.asarray(u, dtype=np.float64)
    return u[1:, :] - u[:-1, :], u[:, 1:] - u[:, :-1]


def fd_div(q1, q2, H, W):
    """div = -D^T for FD-indexed fields q1 [(H-1) x W], q2 [H x (W-1)]."""
    d = np.zeros((H, W))
    d[:-1, :] += q1
    d[1:, :] -= q1
    d[:, :-1] += q2
    d[:, 1:] -= q2
    return d


def fd_to_edges(q1, q2, H, W):
    """FD-indexed field -> global edge arrays g1 [(H+1) x W], g2 [H x (W+1)]
    (boundary rows / columns are the zero dofs of H_0(div))."""
    g1 = np.zeros((H + 1, W))
    g2 = np.zeros((H, W + 1))
    g1[1:H, :] = q1
    g2[:, 1:W] = q2
    return g1, g2


def tv_aniso(u):
    d1, d2 = fd_grad(u)
    return float(np.abs(d1).sum() + np.abs(d2).sum())


def fista_dual_rof(f, alpha, n_iter, q=None):
    """Projected FISTA on min_{|q|<=1} (1/(2 alpha))|div q + alpha f|^2 with step
    1/L, L = 8/alpha, starting from q (default 0).  Returns (q1, q2, u) with
    u = f + div q / alpha."""
    f = np.asarray(f, dtype=np.float64)
    H, W = f.shape
    L = 8.0 / alpha
    if q is None:
        x1, x2 = np.zeros((H - 1, W)), np.zeros((H, W - 1))
    else:
        x1, x2 = (np.array(a, dtype=np.float64) for a in q)
    y1, y2 = x1.copy(), x2.copy()
    t = 1.0
    for _ in range(n_iter):
        v = f + fd_div(y1, y2, H, W) / alpha
        d1, d2 = fd_grad(v)          # the gradient of the dual energy is -D v
        z1 = np.clip(y1 - (-d1) / L, -1.0, 1.0)
        z2 = np.clip(y2 - (-d2) / L, -1.0, 1.0)
        tn = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
        b = (t - 1.0) / tn
        y1, y2 = z1 + b * (z1 - x1), z2 + b * (z2 - x2)
        x1, x2 = z1, z2
        t = tn
    return x1, x2, f + fd_div(x1, x2, H, W) / alpha


def cv_g(f, c1, c2):
    """g = (f - c1)^2 - (f - c2)^2 of eq. (CCV)."""
    f = np.asarray(f, dtype=np.float64)
    return (f - c1) ** 2 - (f - c2) ** 2


def _prox(fidelity, z, f, m, a, c1=0.6, c2=0.1):
    if fidelity == "L2":
        out = (z + a * f) / (1.0 + a)
    elif fidelity == "CV":
        out = np.minimum(np.maximum(z - a * cv_g(f, c1, c2), 0.0), 1.0)
    else:
        d = z - f
        out = f + np.sign(d) * np.maximum(np.abs(d) - a, 0.0)
    return np.where(m, out, z)


def cp2_full(f, alpha, n_iter, tau0, sigma0, gamma, fidelity="L2", mask=None, q=None, u=None, c1=0.6, c2=0.1):
    """Chambolle-Pock Alg. 2 on min_q max_u <div q, u> + chi_C(q) - alpha F(u)
    (the saddle form of Sec. 5 without the proximal term): u is the ascent
    variable, q the accelerated one."""
    f = np.asarray(f, dtype=np.float64)
    H, W = f.shape
    m = np.ones((H, W), bool) if mask is None else np.asarray(mask).astype(bool)
    if q is None:
        x1, x2 = np.zeros((H - 1, W)), np.zeros((H, W - 1))
    else:
        x1, x2 = (np.array(a, dtype=np.float64) for a in q)
    y = f.copy() if u is None else np.array(u, dtype=np.float64)
    xb1, xb2 = x1.copy(), x2.copy()
    tk, sk = tau0, sigma0
    for _ in range(n_iter):
        y = _prox(fidelity, y + sk * fd_div(xb1, xb2, H, W), f, m, sk * alpha, c1, c2)
        d1, d2 = fd_grad(y)          # div^* y = -D y
        z1 = np.clip(x1 - tk * (-d1), -1.0, 1.0)
        z2 = np.clip(x2 - tk * (-d2), -1.0, 1.0)
        th = 1.0 / np.sqrt(1.0 + 2.0 * gamma * tk)
        tk, sk = th * tk, sk / th
        xb1, xb2 = z1 + th * (z1 - x1), z2 + th * (z2 - x2)
        x1, x2 = z1, z2
    return x1, x2, y


def _div_matrix(H, W):
    """Dense matrix of div acting on the stacked FD-indexed dual dofs."""
    n1, n2 = (H - 1) * W, H * (W - 1)
    A = np.zeros((H * W, n1 + n2))
    for k in range(n1 + n2):
        e = np.zeros(n1 + n2)
        e[k] = 1.0
        A[:, k] = fd_div(e[:n1].reshape(H - 1, W), e[n1:].reshape(H, W - 1), H, W).ravel()
    return A


def rof_exact(f, alpha):
    """Exact ROF solution on a tiny image: the dual min_{|q|<=1} |A q + alpha f|^2
    (A = div) solved by bounded-variable least squares, u = f + A q / alpha.
    Returns (u, kkt_residual); the residual certifies the optimality of u:
    alpha (u - f) = div q with q in [-1, 1] and q_e = sign((Du)_e) where
    (Du)_e != 0 (the sign of the saddle form eq. (model_pd), whose optimality
    conditions are eq. (pd_relation))."""
    from scipy.optimize import lsq_linear

    f = np.asarray(f, dtype=np.float64)
    H, W = f.shape
    A = _div_matrix(H, W)
    res = lsq_linear(A, -alpha * f.ravel(), bounds=(-1.0, 1.0), method="bvls", tol=1e-15,
                     lsmr_tol=None, max_iter=10000)
    q = res.x
    u = f + (A @ q).reshape(H, W) / alpha
    d = np.concatenate([a.ravel() for a in fd_grad(u)])
    big = np.abs(d) > 1e-9
    kkt = max(float(np.abs(alpha * (u - f) - (A @ q).reshape(H, W)).max()),
              float(np.abs(q[big] - np.sign(d[big])).max()) if big.any() else 0.0,
              float(max(np.abs(q).max() - 1.0, 0.0)))
    return u, kkt


def tvl1_exact_energy(f, alpha, mask=None):
    """Exact minimum of alpha sum_m |u - f| + TV(u) (TV-L1, optionally with an
    inpainting mask, Sec. 3) on a tiny image, as a linear program over
    (u, s, t) with |u - f| <= s on observed pixels and |Du| <= t."""
    from scipy.optimize import linprog

    f = np.asarray(f, dtype=np.float64)
    H, W = f.shape
    n = H * W
    m = np.ones(n, bool) if mask is None else np.asarray(mask).astype(bool).ravel()
    # difference matrix rows
    rows = []
    for i in range(H - 1):
        for j in range(W):
            r = np.zeros(n); r[(i + 1) * W + j] = 1; r[i * W + j] = -1; rows.append(r)
    for i in range(H):
        for j in range(W - 1):
            r = np.zeros(n); r[i * W + j + 1] = 1; r[i * W + j] = -1; rows.append(r)
    Dm = np.array(rows).reshape(-1, n)
    ne = Dm.shape[0]
    # variables: u (n), s (n), t (ne)
    c = np.concatenate([np.zeros(n), alpha * m.astype(float), np.ones(ne)])
    I = np.eye(n)
    A_ub = np.block([
        [I, -I, np.zeros((n, ne))],
        [-I, -I, np.zeros((n, ne))],
        [Dm, np.zeros((ne, n)), -np.eye(ne)],
        [-Dm, np.zeros((ne, n)), -np.eye(ne)],
    ])
    fv = f.ravel()
    b_ub = np.concatenate([fv, -fv, np.zeros(ne), np.zeros(ne)])
    bounds = [(None, None)] * n + [(0, None)] * (n + ne)
    res = linprog(c, A_ub=A_ub, b_ub=b_ub, bounds=bounds, method="highs-ds",
                  options={"primal_feasibility_tolerance": 1e-10, "dual_feasibility_tolerance": 1e-10})
    if res.status != 0:
        raise RuntimeError(res.message)
    u = res.x[:n].reshape(H, W)
    return float(res.fun), u


def _diff_matrix(H, W):
    """Rows of D: one per interior edge, (u_b - u_a) with b below / right of a."""
    n = H * W
    rows = []
    for i in range(H - 1):
        for j in range(W):
            r = np.zeros(n); r[(i + 1) * W + j] = 1; r[i * W + j] = -1; rows.append(r)
    for i in range(H):
        for j in range(W - 1):
            r = np.zeros(n); r[i * W + j + 1] = 1; r[i * W + j] = -1; rows.append(r)
    return np.array(rows).reshape(-1, n)


def cv_exact_energy(f, alpha, c1, c2):
    """Exact minimum of alpha <u, g> + TV(u) over 0 <= u <= 1 (eq. CCV) on a
    tiny image, as a linear program over (u, t) with |Du| <= t."""
    from scipy.optimize import linprog

    f = np.asarray(f, dtype=np.float64)
    H, W = f.shape
    n = H * W
    Dm = _diff_matrix(H, W)
    ne = Dm.shape[0]
    c = np.concatenate([alpha * cv_g(f, c1, c2).ravel(), np.ones(ne)])
    A_ub = np.block([[Dm, -np.eye(ne)], [-Dm, -np.eye(ne)]])
    b_ub = np.zeros(2 * ne)
    bounds = [(0.0, 1.0)] * n + [(0, None)] * ne
    res = linprog(c, A_ub=A_ub, b_ub=b_ub, bounds=bounds, method="highs-ds",
                  options={"primal_feasibility_tolerance": 1e-10, "dual_feasibility_tolerance": 1e-10})
    if res.status != 0:
        raise RuntimeError(res.message)
    return float(res.fun), res.x[:n].reshape(H, W)


def cv_binary_min(f, alpha, c1, c2):
    """Minimum of alpha sum_{x in S} g_x + (number of edges cut by S) over every
    pixel set S of a tiny image (at most 20 pixels), by enumeration."""
    f = np.asarray(f, dtype=np.float64)
    H, W = f.shape
    n = H * W
    if n > 20:
        raise ValueError("too many pixels to enumerate")
    g = cv_g(f, c1, c2).ravel()
    S = ((np.arange(1 << n)[:, None] >> np.arange(n)[None, :]) & 1).astype(np.float64)
    Dm = _diff_matrix(H, W)
    E = alpha * S @ g + np.abs(S @ Dm.T).sum(axis=1)
    k = int(np.argmin(E))
    return float(E[k]), S[k].reshape(H, W)


def div_norm_sq(apply_div, apply_divT, n_in, iters=2000, seed=0):
    """Largest eigenvalue of div^* div by power iteration."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n_in)
    x /= np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = apply_divT(apply_div(x))
        lam = float(np.linalg.norm(y))
        x = y / lam
    return lam


# --- the decomposed saddle problem (DD) on one global torn vector -----------
def torn_operators(H, W, row_cuts, col_cuts):
    """Dense matrices of the torn divergence and of the jump operator B on one
    global vector of torn edge dofs (Sec. 2.3-2.4), built here from their
    definitions and not from the oracle.

    The vector follows the oracle's documented export layout (subdomains
    row-major; per subdomain p1 [(h+1) x w], edge above local row k, then
    p2 [h x (w+1)], edge left of local column k), so results can be compared
    entry by entry.  Returns (Div [H*W x n_p], Bm [n_lam x n_p], dof [n_p]):
      * (Div p) at a pixel is the outward flux through its four edges, taken
        from its own subdomain's copies;
      * dof is False on edges of the image boundary (not in H_0(div));
      * (B p)_e = (copy of the upper / left subdomain) - (copy of the lower /
        right one), multipliers ordered horizontal interfaces first
        [(ny-1) x W], then vertical ones [(nx-1) x H]."""
    rc, cc = [int(a) for a in row_cuts], [int(a) for a in col_cuts]
    ny, nx = len(rc) - 1, len(cc) - 1
    base, o = {}, 0
    for r in range(ny):
        for c in range(nx):
            h, w = rc[r + 1] - rc[r], cc[c + 1] - cc[c]
            base[r, c] = (o, o + (h + 1) * w, h, w)
            o += (h + 1) * w + h * (w + 1)
    n_p = o
    Div = np.zeros((H * W, n_p))
    dof = np.zeros(n_p, bool)
    for (r, c), (o1, o2, h, w) in base.items():
        ra, ca = rc[r], cc[c]
        for y in range(h):
            for x in range(w):
                g = (ra + y) * W + ca + x
                Div[g, o1 + (y + 1) * w + x] += 1.0
                Div[g, o1 + y * w + x] -= 1.0
                Div[g, o2 + y * (w + 1) + x + 1] += 1.0
                Div[g, o2 + y * (w + 1) + x] -= 1.0
        for k in range(h + 1):
            on_boundary = (k == 0 and r == 0) or (k == h and r == ny - 1)
            dof[o1 + k * w: o1 + (k + 1) * w] = not on_boundary
        for k in range(w + 1):
            on_boundary = (k == 0 and c == 0) or (k == w and c == nx - 1)
            dof[o2 + k: o2 + h * (w + 1): w + 1] = not on_boundary
    Bm = np.zeros(((ny - 1) * W + (nx - 1) * H, n_p))
    for r in range(1, ny):
        for j in range(W):
            c = int(np.searchsorted(cc, j, side="right")) - 1
            s1, _, hs, ws = base[r - 1, c]
            t1, _, _, wt = base[r, c]
            e = (r - 1) * W + j
            Bm[e, s1 + hs * ws + j - cc[c]] = 1.0
            Bm[e, t1 + j - cc[c]] = -1.0
    for c in range(1, nx):
        for i in range(H):
            r = int(np.searchsorted(rc, i, side="right")) - 1
            _, s2, _, ws = base[r, c - 1]
            _, t2, _, wt = base[r, c]
            e = (ny - 1) * W + (c - 1) * H + i
            Bm[e, s2 + (i - rc[r]) * (ws + 1) + ws] = 1.0
            Bm[e, t2 + (i - rc[r]) * (wt + 1)] = -1.0
    return Div, Bm, dof


def rof_dual_prox(f, alpha, tau, v, Div, dof):
    """prox of tau G at v, G(p) = (alpha F)^*(div~ p) + chi_C(p) for the ROF
    fidelity F(u) = |u - f|^2 / 2: the minimiser of
        (alpha/2)|f + div~ p / alpha|^2 + |p - v|^2 / (2 tau)   over |p_e| <= 1
    (the local problems eq. (DD_local_dual) of every subdomain at once; they
    are independent, so one bounded least-squares problem holds them all).
    Solved exactly by BVLS; non-dof edges stay 0."""
    from scipy.optimize import lsq_linear

    nd = int(dof.sum())
    A = np.vstack([Div[:, dof] / np.sqrt(alpha), np.eye(nd) / np.sqrt(tau)])
    b = np.concatenate([-np.sqrt(alpha) * np.asarray(f, dtype=np.float64).ravel(),
                        np.asarray(v)[dof] / np.sqrt(tau)])
    res = lsq_linear(A, b, bounds=(-1.0, 1.0), method="bvls", tol=1e-15, lsmr_tol=None, max_iter=10000)
    p = np.zeros(len(dof))
    p[dof] = res.x
    return p


def dd_saddle_cp(f, alpha, row_cuts, col_cuts, tau, sigma, n_outer, p=None, p_prev=None, lam=None):
    """Chambolle-Pock 2011, Algorithm 1 (theta = 1), on the saddle problem
    (DD) of Sec. 4, min over torn p, max over lambda of
        G(p) + <B p, lambda>,   G = sum_s (alpha F_s)^*(div p_s) + chi_C,
    for the ROF fidelity, written in the textbook's own variables:
        y_{n+1} = y_n + sigma K xbar_n          (F^* = 0: lambda is free)
        x_{n+1} = prox_{tau G}(x_n - tau K^* y_{n+1})
        xbar_{n+1} = 2 x_{n+1} - x_n
    with x = p, y = lambda, K = B, every prox exact (rof_dual_prox) on the
    global torn vector.  Starts from (p, p_prev, lam) (default all 0, the
    start of Algorithm 1).  Returns the list of (p, lam, u) after each step,
    u = f + div~ p / alpha (the primal recovery of the ROF case)."""
    f = np.asarray(f, dtype=np.float64)
    H, W = f.shape
    Div, Bm, dof = torn_operators(H, W, row_cuts, col_cuts)
    x = np.zeros(Bm.shape[1]) if p is None else np.array(p, dtype=np.float64)
    x_old = x.copy() if p_prev is None else np.array(p_prev, dtype=np.float64)
    y = np.zeros(Bm.shape[0]) if lam is None else np.array(lam, dtype=np.float64)
    out = []
    for _ in range(n_outer):
        xbar = 2.0 * x - x_old
        y = y + sigma * (Bm @ xbar)
        x_old, x = x, rof_dual_prox(f, alpha, tau, x - tau * (Bm.T @ y), Div, dof)
        out.append((x.copy(), y.copy(), f + (Div @ x).reshape(H, W) / alpha))
    return out
