"""Python binding of libdtvdd.so (ctypes): argument marshalling only.

Every step of the solver runs in the library's HIP kernels; PyTorch provides
device memory and the stream.  If the library is missing the import of the
solver entry points fails loudly: there is no CPU fallback.

Method: Lee & Park, arXiv 1901.00682, Algorithm 1 (Sec. 4) with the local
solvers of Sec. 5; the C-ABI is documented in include/dtvdd.h.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "libdtvdd.so")

DTV_OK, DTV_EINVAL, DTV_ENOWS, DTV_EHIP, DTV_ESTATE, DTV_ENONFINITE = 0, -1, -2, -3, -4, -5
FIDELITY = {"L2": 0, "L1": 1, "CV": 2}
INNER = {"FISTA": 0, "CP2": 1}
SCHEDULE = {"auto": 0, "stream": 1, "fused": 2, "persistent": 3}
SCHEDULE_NAME = {v: k for k, v in SCHEDULE.items()}

# every entry point declared in include/dtvdd.h
EXPORTS = ("dtv_dd_setup", "dtv_dd_layout", "dtv_dd_workspace_bytes", "dtv_dd_bind_workspace", "dtv_dd_solve",
           "dtv_dd_diagnostics", "dtv_dd_backward", "dtv_dd_kernel_time", "dtv_dd_backward_kernel_time", "dtv_dd_schedule", "dtv_dd_choice",
           "dtv_dd_inner_counts", "dtv_dd_status", "dtv_dd_solve_noalloc", "dtv_dd_destroy", "dtv_last_error")

SCRATCH_BYTES = 32 << 20  # DTV_SCRATCH_BYTES: the library's device scratch array (dtv_dd_solve_noalloc)


class DtvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libdtvdd error {code}: {msg}")
        self.code = code


class ImageDesc(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("ny", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("row_cuts", ctypes.POINTER(ctypes.c_int32)), ("col_cuts", ctypes.POINTER(ctypes.c_int32)),
                ("alpha", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("fidelity", ctypes.c_int32), ("inner", ctypes.c_int32), ("has_mask", ctypes.c_int32),
                ("tau", ctypes.c_double), ("sigma", ctypes.c_double),
                ("tau0", ctypes.c_double), ("sigma0", ctypes.c_double), ("gamma", ctypes.c_double),
                ("n_outer", ctypes.c_int32), ("n_inner", ctypes.c_int32), ("diag_every", ctypes.c_int32),
                ("gap_tol", ctypes.c_double), ("warm_start", ctypes.c_int32),
                ("save_for_backward", ctypes.c_int32), ("ckpt_every", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("time_kernels", ctypes.c_int32), ("rows", ctypes.c_int32),
                ("no_graphs", ctypes.c_int32), ("cv_c1", ctypes.c_double), ("cv_c2", ctypes.c_double),
                ("full_problem", ctypes.c_int32), ("spin_limit", ctypes.c_int32), ("inner_tol", ctypes.c_double),
                ("steps_per_launch", ctypes.c_int32), ("keep_records", ctypes.c_int32),
                ("reverse_schedule", ctypes.c_int32)]


class Layout(ctypes.Structure):
    _fields_ = [("px_off", ctypes.c_int64), ("p1_off", ctypes.c_int64), ("p2_off", ctypes.c_int64),
                ("lam_off", ctypes.c_int64), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("nx", ctypes.c_int32), ("p1_rows", ctypes.c_int32),
                ("p1_pitch", ctypes.c_int32), ("p2_cols", ctypes.c_int32), ("p2_pitch", ctypes.c_int32),
                ("n_lam_h", ctypes.c_int32), ("n_lam_v", ctypes.c_int32)]


_lib = None


def lib(path: str = LIB_PATH):
    """Load libdtvdd.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libdtvdd.so not found at {path}: build it with __graft_entry__.build() "
                           "(there is no CPU fallback)")
    L = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.dtv_dd_setup.argtypes = [ctypes.POINTER(ImageDesc), i32, ctypes.POINTER(Params), ctypes.POINTER(vp)]
    L.dtv_dd_layout.argtypes = [vp, i32, ctypes.POINTER(Layout)]
    L.dtv_dd_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.dtv_dd_bind_workspace.argtypes = [vp, vp, ctypes.c_size_t]
    L.dtv_dd_solve.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(dbl), ctypes.POINTER(i32), vp]
    L.dtv_dd_diagnostics.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.POINTER(dbl), vp]
    L.dtv_dd_backward.argtypes = [vp, vp, vp, vp, vp, vp]
    L.dtv_dd_kernel_time.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_char_p),
                                     ctypes.POINTER(dbl)]
    L.dtv_dd_backward_kernel_time.argtypes = [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(i64),
                                              ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(dbl)]
    L.dtv_dd_schedule.argtypes = [vp, ctypes.POINTER(i32)]
    L.dtv_dd_choice.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.dtv_dd_inner_counts.argtypes = [vp, ctypes.POINTER(i32), vp]
    L.dtv_dd_status.argtypes = [vp, vp]
    L.dtv_dd_solve_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.dtv_dd_destroy.argtypes = [vp]
    L.dtv_dd_destroy.restype = None
    L.dtv_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("dtv_dd_destroy", "dtv_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(code: int):
    if code != DTV_OK:
        raise DtvError(code, lib().dtv_last_error().decode())


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


@dataclass
class Image:
    """One image of a solve: size, subdomain cuts and alpha (Sec. 2.4, eq. model)."""

    H: int
    W: int
    row_cuts: np.ndarray
    col_cuts: np.ndarray
    alpha: float


def floor_cuts(n: int, parts: int) -> np.ndarray:
    return np.array([(k * n) // parts for k in range(parts + 1)], dtype=np.int32)


# Plans still alive at interpreter exit are destroyed by an exit hook, while
# the HIP runtime is still up: the plan's graph, stream, events and pinned
# buffer are released before the runtime tears itself down.
_live_plans: "weakref.WeakSet[Plan]" = weakref.WeakSet()


@atexit.register
def _destroy_live_plans():
    for p in list(_live_plans):
        p.close()


class Plan:
    """A validated solver plan bound to a device workspace."""

    def __init__(self, images, *, fidelity="L2", inner=None, has_mask=False, tau=50.0, sigma=0.01, tau0=10.0,
                 sigma0=1.0 / 80.0, gamma=None, n_outer=100, n_inner=10, diag_every=0, gap_tol=0.0,
                 warm_start=False, save_for_backward=False, ckpt_every=20, schedule="auto",
                 time_kernels=False, rows=0, graphs=True, c1=0.6, c2=0.1, full_problem=False, inner_tol=0.0,
                 spin_limit=0, steps_per_launch=0, keep_records=False, reverse_schedule="auto", device=None,
                 bind=True):
        import torch

        L = lib()
        if inner is None:
            inner = "FISTA" if (fidelity == "L2" and not has_mask) else "CP2"
        self.images = list(images)
        self.fidelity, self.inner, self.has_mask = fidelity, inner, bool(has_mask)
        self._cuts = []
        descs = (ImageDesc * len(self.images))()
        for k, im in enumerate(self.images):
            rc = np.ascontiguousarray(im.row_cuts, dtype=np.int32)
            cc = np.ascontiguousarray(im.col_cuts, dtype=np.int32)
            self._cuts += [rc, cc]
            descs[k] = ImageDesc(int(im.H), int(im.W), len(rc) - 1, len(cc) - 1,
                                 rc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                 cc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), float(im.alpha))
        if gamma is None:
            gamma = 1.0 / (8.0 * tau)
        self.params = Params(FIDELITY[fidelity], INNER[inner], int(has_mask), float(tau), float(sigma),
                             float(tau0), float(sigma0), float(gamma), int(n_outer), int(n_inner),
                             int(diag_every), float(gap_tol), int(warm_start), int(save_for_backward),
                             int(ckpt_every), SCHEDULE[schedule], int(time_kernels), int(rows),
                             int(not graphs), float(c1), float(c2), int(full_problem), int(spin_limit),
                             float(inner_tol), int(steps_per_launch), int(keep_records),
                             SCHEDULE[reverse_schedule])
        h = ctypes.c_void_p()
        _check(L.dtv_dd_setup(descs, len(self.images), ctypes.byref(self.params), ctypes.byref(h)))
        self.h = h
        self._L = L
        _live_plans.add(self)
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.ws = None
        if bind:
            nb = ctypes.c_size_t()
            _check(L.dtv_dd_workspace_bytes(self.h, ctypes.byref(nb)))
            self.ws = torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device=self.device)
            _check(L.dtv_dd_bind_workspace(self.h, ctypes.c_void_p(self.ws.data_ptr()), int(nb.value)))

    def close(self):
        """Destroy the library plan (idempotent); the workspace tensor is
        released with the object."""
        h = getattr(self, "h", None)
        L = getattr(self, "_L", None)  # held by the plan: module globals may be gone at interpreter exit
        if h is not None and h.value and L is not None:
            L.dtv_dd_destroy(h)
        self.h = None

    def __del__(self):
        self.close()

    @property
    def n_images(self) -> int:
        return len(self.images)

    def layout(self, image: int = -1) -> Layout:
        out = Layout()
        _check(lib().dtv_dd_layout(self.h, int(image), ctypes.byref(out)))
        return out

    def choice(self) -> dict:
        """Schedule, streaming rows and their source (rule, measured, cached, explicit)."""
        sc, r, src = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().dtv_dd_choice(self.h, ctypes.byref(sc), ctypes.byref(r), ctypes.byref(src)))
        return {"schedule": SCHEDULE_NAME[sc.value], "rows": r.value,
                "source": ("rule", "measured", "cached", "explicit")[src.value]}

    def schedule(self) -> str:
        s = ctypes.c_int32()
        _check(lib().dtv_dd_schedule(self.h, ctypes.byref(s)))
        return SCHEDULE_NAME[s.value]

    def new_state(self):
        """Zeroed device buffers u, p1, p2, lambda sized for this plan."""
        import torch

        T = self.layout(-1)
        z = lambda n: torch.zeros(max(int(n), 1), dtype=torch.float32, device=self.device)
        return {"u": z(T.px_off), "p1": z(T.p1_off), "p2": z(T.p2_off), "lam": z(T.lam_off)}

    def _stream(self, stream):
        import torch

        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(stream.cuda_stream)

    def status(self, stream=None):
        """Raise DtvError if a persistent launch of the last solve gave up a
        wait for a neighbouring subdomain (waits for the stream)."""
        _check(lib().dtv_dd_status(self.h, self._stream(stream)))

    def solve_noalloc(self, f, mask=None, state=None, stream=None, check=True):
        """dtv_dd_solve_noalloc: the solve on the library's device scratch
        array (no workspace, no allocation in the call).  state: dict from
        new_state() (allocated here when None, before the call)."""
        import torch

        if state is None:
            state = self.new_state()
        assert f.dtype == torch.float32 and f.is_contiguous() and f.device.type == "cuda"
        if mask is not None:
            assert mask.dtype == torch.uint8 and mask.is_contiguous()
        _check(lib().dtv_dd_solve_noalloc(self.h, _ptr(f), _ptr(mask), _ptr(state["u"]), _ptr(state["p1"]),
                                          _ptr(state["p2"]), _ptr(state["lam"]), self._stream(stream)))
        if check:
            self.status(stream)
        return state

    def solve(self, f, mask=None, state=None, stream=None, want_stats=True, check=True):
        """Run the plan.  f: flat float32 device tensor (images concatenated);
        state: dict from new_state() (allocated when None).  Returns
        (state, stats) with stats an array [n_images, rows, 5] or None.
        check: read the persistent schedule's wait status afterwards (waits for
        the stream); False leaves the call asynchronous (see status())."""
        import torch

        if state is None:
            state = self.new_state()
        assert f.dtype == torch.float32 and f.is_contiguous() and f.device.type == "cuda"
        if mask is not None:
            assert mask.dtype == torch.uint8 and mask.is_contiguous()
        P = self.params
        rows = P.n_outer // P.diag_every + 1 if P.diag_every > 0 else 0
        stats = np.zeros(max(1, self.n_images * rows * 5))
        nrow = ctypes.c_int32(0)
        sp = stats.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if (want_stats and rows) else None
        code = lib().dtv_dd_solve(self.h, _ptr(f), _ptr(mask), _ptr(state["u"]), _ptr(state["p1"]),
                                  _ptr(state["p2"]), _ptr(state["lam"]), sp, ctypes.byref(nrow),
                                  self._stream(stream))
        _check(code)
        if check:
            self.status(stream)
        st = stats[: self.n_images * rows * 5].reshape(self.n_images, rows, 5)[:, : nrow.value] if sp else None
        return state, st

    def diagnostics(self, f, state, mask=None, stream=None) -> np.ndarray:
        out = np.zeros(4 * self.n_images)
        _check(lib().dtv_dd_diagnostics(self.h, _ptr(f), _ptr(mask), _ptr(state["u"]), _ptr(state["p1"]),
                                        _ptr(state["p2"]), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        self._stream(stream)))
        return out.reshape(self.n_images, 4)

    def backward(self, f, grad_u, stream=None, check=True):
        """Reverse mode of the last solve (which must have run with
        save_for_backward): returns (dl/df, dl/dalpha per image).  check: read
        the persistent reverse's wait status afterwards (waits for the stream)."""
        import torch

        assert f.dtype == torch.float32 and grad_u.dtype == torch.float32
        grad_f = torch.empty_like(f)
        grad_alpha = torch.zeros(self.n_images, dtype=torch.float32, device=self.device)
        _check(lib().dtv_dd_backward(self.h, _ptr(f), _ptr(grad_u.contiguous()), _ptr(grad_f), _ptr(grad_alpha),
                                     self._stream(stream)))
        if check:
            self.status(stream)
        return grad_f, grad_alpha

    def inner_counts(self, stream=None) -> np.ndarray:
        """[n_subdomains, 2] local steps of the last solve per subdomain (total,
        most in one outer step), image-major, row-major over each grid."""
        nsub = sum((len(im.row_cuts) - 1) * (len(im.col_cuts) - 1) for im in self.images)
        out = np.zeros(2 * nsub, dtype=np.int32)
        _check(lib().dtv_dd_inner_counts(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                         self._stream(stream)))
        return out.reshape(nsub, 2)

    def kernel_time(self):
        ms, n, nm, b = ctypes.c_double(), ctypes.c_int64(), ctypes.c_char_p(), ctypes.c_double()
        _check(lib().dtv_dd_kernel_time(self.h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(nm), ctypes.byref(b)))
        return {"avg_ms": ms.value, "launches": n.value, "name": nm.value.decode(), "bytes_per_launch": b.value}

    def backward_kernel_time(self, which: int = 0):
        """Timing of the last backward's launches (time_kernels): which = 0 the
        reverse steps, 1 the recording forward."""
        ms, n, nm, b = ctypes.c_double(), ctypes.c_int64(), ctypes.c_char_p(), ctypes.c_double()
        _check(lib().dtv_dd_backward_kernel_time(self.h, int(which), ctypes.byref(ms), ctypes.byref(n),
                                                 ctypes.byref(nm), ctypes.byref(b)))
        return {"avg_ms": ms.value, "launches": n.value, "name": nm.value.decode(), "bytes_per_launch": b.value}

    # -- views in the documented layout --------------------------------------
    def p_views(self, state, image: int = 0):
        """(P1 [(H+ny) x W], P2 [H x (W+nx)]) views of one image's torn p."""
        Lm = self.layout(image)
        p1 = state["p1"][Lm.p1_off: Lm.p1_off + Lm.p1_rows * Lm.p1_pitch].view(Lm.p1_rows, Lm.p1_pitch)[:, : Lm.W]
        p2 = state["p2"][Lm.p2_off: Lm.p2_off + Lm.H * Lm.p2_pitch].view(Lm.H, Lm.p2_pitch)[:, : Lm.p2_cols]
        return p1, p2

    def u_view(self, state, image: int = 0):
        Lm = self.layout(image)
        return state["u"][Lm.px_off: Lm.px_off + Lm.H * Lm.W].view(Lm.H, Lm.W)

    def lam_view(self, state, image: int = 0):
        """(lambda, prev_s, prev_t), each of n_lam floats."""
        Lm = self.layout(image)
        n = Lm.n_lam_h + Lm.n_lam_v
        blk = state["lam"][Lm.lam_off: Lm.lam_off + 3 * n]
        return blk[:n], blk[n:2 * n], blk[2 * n:]


def solve(f, alpha, *, mask=None, grid=(2, 2), row_cuts=None, col_cuts=None, fidelity="L2", inner=None,
          n_outer=100, n_inner=10, diag_every=0, **kw):
    """Solve one image.  f: 2-D float32 CUDA tensor.  Returns a dict with u,
    p1, p2 (torn layout), lam (multipliers), stats and the plan."""
    import torch

    H, W = f.shape
    rc = floor_cuts(H, grid[0]) if row_cuts is None else np.asarray(row_cuts, np.int32)
    cc = floor_cuts(W, grid[1]) if col_cuts is None else np.asarray(col_cuts, np.int32)
    plan = Plan([Image(H, W, rc, cc, alpha)], fidelity=fidelity, inner=inner, has_mask=mask is not None,
                n_outer=n_outer, n_inner=n_inner, diag_every=diag_every, device=f.device, **kw)
    fl = f.contiguous().view(-1).to(torch.float32)
    ml = None if mask is None else mask.contiguous().view(-1).to(torch.uint8)
    state, stats = plan.solve(fl, ml)
    p1, p2 = plan.p_views(state)
    lam, _, _ = plan.lam_view(state)
    return {"u": plan.u_view(state), "p1": p1, "p2": p2, "lam": lam, "stats": None if stats is None else stats[0],
            "plan": plan, "state": state}


def _torch_function():
    import torch

    class DTVDD(torch.autograd.Function):
        """u = solve(f, alpha) with the unrolled Algorithm 1 (FISTA local
        steps); differentiable in f and alpha through the library's reverse
        mode with outer-step checkpoints.  f: [H, W] or [B, H, W] float32 on the
        GPU; alpha: a scalar or [B] tensor (one weight per image).  keep_records:
        the forward solve keeps every outer step's step records instead
        (about n_outer (9 n_inner + 8) bytes per pixel of device memory), so
        that the backward pass recomputes nothing."""

        @staticmethod
        def forward(ctx, f, alpha, grid=(4, 4), n_outer=200, n_inner=5, ckpt_every=20, tau=50.0, sigma=0.01,
                    schedule="auto", keep_records=False):
            batched = f.dim() == 3
            fb = f if batched else f.unsqueeze(0)
            B, H, W = fb.shape
            al = alpha.detach().reshape(-1).to("cpu", torch.float64)
            if al.numel() == 1 and B > 1:
                al = al.expand(B)
            rc, cc = floor_cuts(H, grid[0]), floor_cuts(W, grid[1])
            plan = Plan([Image(H, W, rc, cc, float(al[b])) for b in range(B)], n_outer=n_outer, n_inner=n_inner,
                        save_for_backward=True, ckpt_every=ckpt_every, tau=tau, sigma=sigma, schedule=schedule,
                        keep_records=keep_records, device=f.device)
            fl = fb.detach().contiguous().reshape(-1).to(torch.float32)
            state, _ = plan.solve(fl, want_stats=False)
            u = state["u"][: B * H * W].view(B, H, W).clone()
            ctx.plan = plan
            ctx.batched = batched
            ctx.alpha_shape = alpha.shape
            ctx.alpha_device = alpha.device
            ctx.save_for_backward(fl)
            return u if batched else u[0]

        @staticmethod
        def backward(ctx, grad_u):
            (fl,) = ctx.saved_tensors
            g = grad_u.contiguous().reshape(-1).to(torch.float32)
            gf, ga = ctx.plan.backward(fl, g)
            gf = gf.view(grad_u.shape)
            if ga.numel() != max(1, int(np.prod(ctx.alpha_shape))):
                ga = ga.sum()   # one alpha shared by the whole batch
            ga = ga.reshape(ctx.alpha_shape).to(ctx.alpha_device)
            return gf, ga, None, None, None, None, None, None, None, None

    return DTVDD


def __getattr__(name):
    if name == "DTVDD":
        return _torch_function()
    raise AttributeError(name)
