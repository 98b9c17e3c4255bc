"""FP64 CPU oracle for the primal-dual domain decomposition of dual-TV problems.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  It shares no code with the GPU
library: the arithmetic lives in ``dd_oracle.c`` (plain C, double precision)
and this module only marshals arrays.

Citations refer to Lee & Park, arXiv 1901.00682:
  Sec. 2.3  discrete spaces X (P0 pixels) and Y (RT0 edge dofs), box set C;
  Sec. 2.4  torn local spaces, jump operator B;
  Sec. 3    fidelities and their prox operators;
  Sec. 4    saddle problem (DD) and Algorithm 1;
  Sec. 5    local accelerated primal-dual solver and its parameters.

Layout conventions of the oracle (its own):
  * ``p`` is the concatenation over subdomains s (row-major) of p1_s
    [(h+1) x w] then p2_s [h x (w+1)];
  * ``lam`` is lam_h [(ny-1) x W] then lam_v [(nx-1) x H];
  * ``to_torn`` maps ``p`` to the documented torn layout of the C-ABI
    (P1 [(H+ny) x W], P2 [H x (W+nx)]) so results can be compared.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
SRC_PATH = os.path.join(_HERE, "dd_oracle.c")

_lib = None


def build(out_path: str = LIB_PATH, src: str = SRC_PATH, extra: tuple = ()) -> str:
    """Compile the oracle with gcc (double precision, no FMA contraction)."""
    import subprocess

    os.makedirs(os.path.dirname(out_path), exist_ok=True)
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           *extra, "-o", out_path, src, "-lm"]
    subprocess.run(cmd, check=True)
    return out_path


class _Params(ctypes.Structure):
    _fields_ = [
        ("H", ctypes.c_int), ("W", ctypes.c_int), ("ny", ctypes.c_int), ("nx", ctypes.c_int),
        ("alpha", ctypes.c_double),
        ("fidelity", ctypes.c_int), ("inner", ctypes.c_int), ("no_prox_term", ctypes.c_int),
        ("tau", ctypes.c_double), ("sigma", ctypes.c_double),
        ("tau0", ctypes.c_double), ("sigma0", ctypes.c_double), ("gamma", ctypes.c_double),
        ("n_inner", ctypes.c_int),
        ("cv_c1", ctypes.c_double), ("cv_c2", ctypes.c_double),
        ("inner_tol", ctypes.c_double),
    ]


_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_U8 = ctypes.POINTER(ctypes.c_uint8)
_L = ctypes.POINTER(ctypes.c_long)


def load(path: str = LIB_PATH):
    global _lib
    if path == LIB_PATH and _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"oracle library missing at {path}; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    lib.orc_create.restype = vp
    lib.orc_create.argtypes = [ctypes.POINTER(_Params), _I, _I, _D, _U8]
    lib.orc_destroy.argtypes = [vp]
    lib.orc_run.restype = ctypes.c_int
    lib.orc_run.argtypes = [vp, ctypes.c_int, _I, ctypes.c_int, _D, _U8, _D, ctypes.c_int]
    lib.orc_sizes.argtypes = [vp, _L]
    lib.orc_export.argtypes = [vp, _D, _D, _D, _D, _L]
    lib.orc_import.argtypes = [vp, _D, _D, _D, _D, ctypes.c_long]
    lib.orc_diagnostics.argtypes = [vp, _D, _U8, _D]
    lib.orc_apply_div.argtypes = [vp, _D, _D]
    lib.orc_apply_divT.argtypes = [vp, _D, _D]
    lib.orc_apply_B.argtypes = [vp, _D, _D]
    lib.orc_apply_BT.argtypes = [vp, _D, _D]
    lib.orc_tv.restype = ctypes.c_double
    lib.orc_tv.argtypes = [ctypes.c_int, ctypes.c_int, _D]
    lib.orc_primal_energy.restype = ctypes.c_double
    lib.orc_primal_energy.argtypes = [vp, _D, _D, _U8]
    lib.orc_proj_box.argtypes = [ctypes.c_long, _D, _D]
    lib.orc_prox.argtypes = [ctypes.c_int, ctypes.c_long, _D, _D, _U8, ctypes.c_double, ctypes.c_double,
                             ctypes.c_double, _D]
    lib.orc_n_done.restype = ctypes.c_int
    lib.orc_n_done.argtypes = [vp]
    lib.orc_threads.restype = ctypes.c_int
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_inner_counts.argtypes = [vp, _L]
    lib.orc_inner_margin.restype = ctypes.c_double
    lib.orc_inner_margin.argtypes = [vp]
    if hasattr(lib, "orc_backward"):
        lib.orc_backward.restype = ctypes.c_int
        lib.orc_backward.argtypes = [vp, ctypes.c_int, _D, _U8, _D, _D, _D]
    if path == LIB_PATH:
        _lib = lib
    return lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


FIDELITY = {"L2": 0, "L1": 1, "CV": 2}
INNER = {"FISTA": 0, "CP2": 1}


@dataclass
class Problem:
    """Everything Algorithm 1 needs (Sec. 4 and the parameters of Sec. 5)."""

    f: np.ndarray
    alpha: float
    row_cuts: np.ndarray
    col_cuts: np.ndarray
    fidelity: str = "L2"
    inner: str = "FISTA"
    mask: np.ndarray | None = None
    tau: float = 50.0
    sigma: float = 0.01
    tau0: float = 10.0
    sigma0: float = 1.0 / 80.0
    gamma: float | None = None   # default 1/(8 tau)
    n_inner: int = 10
    no_prox_term: bool = False
    c1: float = 0.6              # Chan-Vese intensities (fidelity "CV"), eq. (CCV)
    c2: float = 0.1
    inner_tol: float = 0.0       # > 0: inner stopping rule of Sec. 5.1 (either local solver), n_inner the cap


class Oracle:
    """One run of Algorithm 1 on the CPU, in double precision."""

    def __init__(self, prob: Problem, lib_path: str = LIB_PATH):
        self.lib = load(lib_path)
        self.prob = prob
        f = _f64(prob.f)
        if f.ndim != 2:
            raise ValueError("f must be 2-D")
        H, W = f.shape
        self.H, self.W = H, W
        self.row_cuts = np.ascontiguousarray(prob.row_cuts, dtype=np.int32)
        self.col_cuts = np.ascontiguousarray(prob.col_cuts, dtype=np.int32)
        self.ny, self.nx = len(self.row_cuts) - 1, len(self.col_cuts) - 1
        gamma = prob.gamma if prob.gamma is not None else 1.0 / (8.0 * prob.tau)
        self.params = _Params(H, W, self.ny, self.nx, float(prob.alpha), FIDELITY[prob.fidelity],
                              INNER[prob.inner], int(prob.no_prox_term), float(prob.tau), float(prob.sigma),
                              float(prob.tau0), float(prob.sigma0), float(gamma), int(prob.n_inner),
                              float(prob.c1), float(prob.c2), float(prob.inner_tol))
        self.f = f
        self.mask = None if prob.mask is None else np.ascontiguousarray(prob.mask, dtype=np.uint8)
        self._mp = None if self.mask is None else self.mask.ctypes.data_as(_U8)
        self.h = self.lib.orc_create(ctypes.byref(self.params), self.row_cuts.ctypes.data_as(_I),
                                     self.col_cuts.ctypes.data_as(_I), _dp(f), self._mp)
        if not self.h:
            raise ValueError("oracle rejected the problem (shape / cuts / alpha)")
        sz = np.zeros(3, dtype=np.int64)
        self.lib.orc_sizes(self.h, sz.ctypes.data_as(_L))
        self.n_p, self.n_lam, self.n_u = (int(x) for x in sz)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.orc_destroy(h)
            self.h = None

    # -- Algorithm 1 ---------------------------------------------------
    def run(self, n_outer: int, diag_every: int = 0, order=None) -> np.ndarray:
        """Run n_outer outer steps; returns rows [n, J, D, gap, |Bp|]."""
        rows = n_outer // diag_every if diag_every > 0 else 0
        stats = np.zeros((max(rows, 1), 5))
        op = None
        if order is not None:
            order = np.ascontiguousarray(order, dtype=np.int32)
            op = order.ctypes.data_as(_I)
        got = self.lib.orc_run(self.h, int(n_outer), op, int(diag_every), _dp(self.f), self._mp,
                               _dp(stats), rows)
        return stats[:got]

    def inner_counts(self) -> np.ndarray:
        """[n_subdomains, 2] local steps (total, most in one outer step), row-major."""
        out = np.zeros(2 * self.ny * self.nx, dtype=np.int64)
        self.lib.orc_inner_counts(self.h, out.ctypes.data_as(_L))
        return out.reshape(-1, 2)

    def inner_margin(self) -> float:
        """Smallest |log(relative change^2 / tol^2)| over every stopping test so
        far: how close any decision came to the threshold."""
        return float(self.lib.orc_inner_margin(self.h))

    @property
    def n_done(self) -> int:
        return self.lib.orc_n_done(self.h)

    def export(self) -> dict:
        u = np.zeros((self.H, self.W))
        p = np.zeros(self.n_p)
        lam = np.zeros(self.n_lam)
        prev = np.zeros(2 * self.n_lam)
        nd = np.zeros(1, dtype=np.int64)
        self.lib.orc_export(self.h, _dp(u), _dp(p), _dp(lam), _dp(prev), nd.ctypes.data_as(_L))
        return {"u": u, "p": p, "lam": lam, "prev": prev, "n_done": int(nd[0])}

    def import_state(self, st: dict) -> None:
        self.lib.orc_import(self.h, _dp(_f64(st["u"])), _dp(_f64(st["p"])), _dp(_f64(st["lam"])),
                            _dp(_f64(st["prev"])), int(st["n_done"]))

    def backward(self, n_outer: int, ubar) -> tuple:
        """Reverse mode of n_outer steps of Algorithm 1 from the initial state
        (FISTA local solver, L2, no mask): returns (dl/df, dl/dalpha) for the
        loss gradient ubar = dl/du of the final u = f + div~ p / alpha.  Runs
        the forward itself; the oracle must not have been stepped before."""
        if not hasattr(self.lib, "orc_backward"):
            raise RuntimeError("oracle built without the reverse pass")
        ub = _f64(ubar).reshape(self.H, self.W)
        fbar = np.zeros((self.H, self.W))
        abar = np.zeros(1)
        rc = self.lib.orc_backward(self.h, int(n_outer), _dp(self.f), self._mp, _dp(ub), _dp(fbar), _dp(abar))
        if rc != 0:
            raise ValueError("reverse pass not available for this problem (needs FISTA, L2, no mask, fresh state)")
        return fbar, float(abar[0])

    def diagnostics(self) -> np.ndarray:
        out = np.zeros(4)
        self.lib.orc_diagnostics(self.h, _dp(self.f), self._mp, _dp(out))
        return out

    # -- linear operators (exposed for the pins) --------------------------
    def div(self, p):
        out = np.zeros((self.H, self.W))
        self.lib.orc_apply_div(self.h, _dp(_f64(p)), _dp(out))
        return out

    def divT(self, u):
        out = np.zeros(self.n_p)
        self.lib.orc_apply_divT(self.h, _dp(_f64(u)), _dp(out))
        return out

    def B(self, p):
        out = np.zeros(self.n_lam)
        self.lib.orc_apply_B(self.h, _dp(_f64(p)), _dp(out))
        return out

    def BT(self, lam):
        out = np.zeros(self.n_p)
        self.lib.orc_apply_BT(self.h, _dp(_f64(lam)), _dp(out))
        return out

    def energy(self, u) -> float:
        return self.lib.orc_primal_energy(self.h, _dp(_f64(u)), _dp(self.f), self._mp)

    # -- layout conversion (oracle layout -> documented torn layout) ------
    def subdomains(self):
        for r in range(self.ny):
            for c in range(self.nx):
                ra, rb = int(self.row_cuts[r]), int(self.row_cuts[r + 1])
                ca, cb = int(self.col_cuts[c]), int(self.col_cuts[c + 1])
                yield r, c, ra, rb, ca, cb

    def to_torn(self, p):
        """Map the concatenated p to P1 [(H+ny) x W] and P2 [H x (W+nx)]:
        subdomain (r, c) keeps its edge rows at P1 rows ra + r .. rb + r and its
        edge columns at P2 columns ca + c .. cb + c."""
        P1 = np.zeros((self.H + self.ny, self.W))
        P2 = np.zeros((self.H, self.W + self.nx))
        o = 0
        for r, c, ra, rb, ca, cb in self.subdomains():
            h, w = rb - ra, cb - ca
            P1[ra + r: rb + r + 1, ca:cb] = p[o:o + (h + 1) * w].reshape(h + 1, w)
            o += (h + 1) * w
            P2[ra:rb, ca + c: cb + c + 1] = p[o:o + h * (w + 1)].reshape(h, w + 1)
            o += h * (w + 1)
        return P1, P2

    def from_torn(self, P1, P2):
        parts = []
        for r, c, ra, rb, ca, cb in self.subdomains():
            parts.append(np.asarray(P1[ra + r: rb + r + 1, ca:cb], dtype=np.float64).ravel())
            parts.append(np.asarray(P2[ra:rb, ca + c: cb + c + 1], dtype=np.float64).ravel())
        return np.concatenate(parts)

    def lam_split(self, lam):
        nh = (self.ny - 1) * self.W
        return lam[:nh].reshape(self.ny - 1, self.W), lam[nh:].reshape(self.nx - 1, self.H)


def proj_box(p):
    p = _f64(p)
    out = np.empty_like(p)
    load().orc_proj_box(p.size, _dp(p), _dp(out))
    return out


def prox(fidelity: str, z, f, a: float, mask=None, c1: float = 0.6, c2: float = 0.1):
    z, f = _f64(z), _f64(f)
    out = np.empty_like(z)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    load().orc_prox(FIDELITY[fidelity], z.size, _dp(z), _dp(f), None if m is None else m.ctypes.data_as(_U8),
                    float(a), float(c1), float(c2), _dp(out))
    return out


def threads() -> int:
    """Threads used by the oracle's parallel loop over subdomains."""
    return int(load().orc_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loop over subdomains from now on."""
    load().orc_set_threads(int(n))


def tv(u) -> float:
    u = _f64(u)
    return load().orc_tv(u.shape[0], u.shape[1], _dp(u))
