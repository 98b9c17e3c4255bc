"""The C-ABI library loads and exports every entry point declared in
include/dtvdd.h; argument validation (host-only) returns the documented codes
without touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1901_00682_amd import dtvdd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "dtvdd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dtv_\w+)\s*\(", text)))


def test_header_matches_binding_list():
    assert declared_functions() == sorted(dtvdd.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = dtvdd.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def _setup(H=64, W=64, rc=(0, 32, 64), cc=(0, 32, 64), alpha=10.0, n_images=1, **kw):
    L = dtvdd.lib()
    rc = np.asarray(rc, np.int32)
    cc = np.asarray(cc, np.int32)
    descs = (dtvdd.ImageDesc * n_images)()
    for k in range(n_images):
        descs[k] = dtvdd.ImageDesc(H, W, len(rc) - 1, len(cc) - 1, rc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   cc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), alpha)
    base = dict(fidelity=0, inner=0, has_mask=0, tau=50.0, sigma=0.01, tau0=10.0, sigma0=1 / 80, gamma=1 / 400,
                n_outer=10, n_inner=5, diag_every=0, gap_tol=0.0, warm_start=0, save_for_backward=0, ckpt_every=20,
                schedule=0, time_kernels=0, rows=0, no_graphs=0)
    base.update(kw)
    prm = dtvdd.Params(**base)
    h = ctypes.c_void_p()
    code = L.dtv_dd_setup(descs, n_images, ctypes.byref(prm), ctypes.byref(h))
    if code == 0:
        assert h.value
    return code, h


def test_valid_setup_and_layout():
    L = dtvdd.lib()
    code, h = _setup(H=70, W=150, rc=(0, 20, 41, 70), cc=(0, 1, 63, 64, 100, 150))
    assert code == 0
    lay = dtvdd.Layout()
    assert L.dtv_dd_layout(h, 0, ctypes.byref(lay)) == 0
    assert (lay.H, lay.W, lay.ny, lay.nx) == (70, 150, 3, 5)
    assert lay.p1_rows == 73 and lay.p1_pitch >= 150 and lay.p1_pitch % 64 == 0
    assert lay.p2_cols == 155 and lay.p2_pitch >= 155
    assert lay.n_lam_h == 2 * 150 and lay.n_lam_v == 4 * 70
    tot = dtvdd.Layout()
    assert L.dtv_dd_layout(h, -1, ctypes.byref(tot)) == 0
    assert tot.px_off == 70 * 150 and tot.lam_off >= 3 * (300 + 280)
    nb = ctypes.c_size_t()
    assert L.dtv_dd_workspace_bytes(h, ctypes.byref(nb)) == 0 and nb.value > 0
    assert L.dtv_dd_layout(h, 1, ctypes.byref(lay)) == dtvdd.DTV_EINVAL
    L.dtv_dd_destroy(h)


@pytest.mark.parametrize("kw,msg", [
    (dict(rc=(0, 40, 30, 64)), "increasing"),
    (dict(rc=(0, 32, 65)), "end"),
    (dict(alpha=0.0), "alpha"),
    (dict(alpha=float("nan")), "alpha"),
    (dict(tau=50.0, sigma=0.02), "tau * sigma"),
    (dict(fidelity=1), "FISTA"),
    (dict(has_mask=1), "FISTA"),
    (dict(inner=1, tau0=10.0, sigma0=0.02), "8 tau0 sigma0"),
    (dict(inner=1, gamma=1.0), "gamma"),
    (dict(n_inner=0), "n_inner"),
    (dict(gap_tol=1e-3), "gap_tol"),
    (dict(H=0), "sizes"),
    (dict(fidelity=7), "fidelity"),
    (dict(schedule=9), "schedule"),
    (dict(rows=5), "rows"),
    (dict(no_graphs=2), "no_graphs"),
    (dict(schedule=3), "persistent"),
    (dict(fidelity=2), "FISTA"),
    (dict(fidelity=2, inner=1, has_mask=1), "Chan-Vese"),
    (dict(fidelity=2, inner=1, cv_c1=float("inf")), "cv_c1"),
    (dict(full_problem=1), "full_problem needs"),
    (dict(full_problem=2), "full_problem must"),
    (dict(full_problem=1, rc=(0, 64), cc=(0, 64), save_for_backward=1), "save_for_backward"),
    (dict(full_problem=1, rc=(0, 64), cc=(0, 64), inner=1, gamma=-1.0), "gamma"),
    (dict(inner_tol=-1.0), "inner_tol"),
    (dict(inner_tol=1e-3, inner=1), "inner_tol needs the fused schedule's subdomains"),
    (dict(inner_tol=1e-3, schedule=1), "inner_tol needs the fused or persistent"),
    (dict(inner_tol=1e-3, save_for_backward=1), "inner_tol needs the fused or persistent"),
    (dict(inner_tol=1e-3, H=300, W=300, rc=(0, 150, 300), cc=(0, 150, 300)), "at most 128"),
    (dict(inner_tol=1e-3, n_inner=100001), "cap"),
    (dict(spin_limit=-1), "spin_limit"),
    (dict(inner=1, steps_per_launch=6), "steps_per_launch"),
    (dict(inner=1, steps_per_launch=-1), "steps_per_launch"),
    (dict(keep_records=2), "keep_records must"),
    (dict(keep_records=1), "keep_records needs save_for_backward"),
    (dict(keep_records=1, save_for_backward=1, schedule=1), "keep_records runs the fused"),
    (dict(keep_records=1, save_for_backward=1), "on-chip reverse"),
    (dict(keep_records=1, save_for_backward=1, H=256, W=256, rc=(0, 128, 256), cc=(0, 128, 256), n_inner=9),
     "on-chip reverse"),
    (dict(reverse_schedule=1), "reverse_schedule must"),
    (dict(reverse_schedule=9), "reverse_schedule must"),
    (dict(save_for_backward=1, reverse_schedule=3), "reverse_schedule persistent needs"),
])
def test_validation_errors(kw, msg):
    code, h = _setup(**kw)
    assert code == dtvdd.DTV_EINVAL
    assert msg in dtvdd.lib().dtv_last_error().decode()


@pytest.mark.parametrize("kw", [
    dict(fidelity=2, inner=1, tau=1.0, sigma=0.5, gamma=0.125, cv_c1=0.6, cv_c2=0.1),
    dict(fidelity=2, inner=1, tau=1.0, sigma=0.5, gamma=0.125, gap_tol=1e-4, diag_every=5),
    # the undecomposed problem ignores tau and sigma, and gamma has no 1/tau bound
    dict(full_problem=1, rc=(0, 64), cc=(0, 64), tau=0.0, sigma=0.0),
    dict(full_problem=1, rc=(0, 64), cc=(0, 64), inner=1, fidelity=1, tau=0.0, sigma=0.0, gamma=5.0),
    # the streaming primal-dual launches: every steps-per-launch value, more than n_inner included
    dict(inner=1, fidelity=1, has_mask=1, steps_per_launch=5),
    dict(inner=1, n_inner=7, steps_per_launch=3),
    dict(inner=1, n_inner=2, steps_per_launch=4),
    dict(inner=1, n_inner=1, steps_per_launch=2),
])
def test_valid_chan_vese_and_full_problem(kw):
    code, h = _setup(**kw)
    assert code == 0, dtvdd.lib().dtv_last_error().decode()
    dtvdd.lib().dtv_dd_destroy(h)


def _kernel_name(h):
    name = ctypes.c_char_p()
    assert dtvdd.lib().dtv_dd_kernel_time(h, None, None, ctypes.byref(name), None) == 0
    return name.value.decode()


def test_multi_step_launches_fall_back_beyond_32_bit_row_offsets():
    """The multi-step primal-dual kernel addresses rows by 32-bit byte offsets;
    an image whose vertical multipliers span 2 GiB (nx H >= 2^29) runs one step
    per launch instead (the same result), a small one the multi-step kernel."""
    L = dtvdd.lib()
    H, W = 1 << 20, 1024
    code, h = _setup(H=H, W=W, rc=(0, H), cc=tuple(range(0, W + 1, 2)), inner=1, steps_per_launch=5)
    assert code == 0
    assert _kernel_name(h) == "k_cp2_step"
    L.dtv_dd_destroy(h)
    code, h = _setup(inner=1, steps_per_launch=5)
    assert code == 0 and _kernel_name(h) == "k_cp2_multi"
    L.dtv_dd_destroy(h)
    code, h = _setup(inner=1, steps_per_launch=1)
    assert code == 0 and _kernel_name(h) == "k_cp2_step"
    L.dtv_dd_destroy(h)
    # the FISTA streaming schedule (schedule 1) likewise
    code, h = _setup(schedule=1)
    assert code == 0 and _kernel_name(h) == "k_fista_multi"
    L.dtv_dd_destroy(h)
    code, h = _setup(schedule=1, steps_per_launch=1)
    assert code == 0 and _kernel_name(h) == "k_fista_step"
    L.dtv_dd_destroy(h)


def test_inner_counts_before_any_solve_are_zero():
    L = dtvdd.lib()
    for kw in (dict(), dict(inner_tol=1e-3, n_inner=500)):
        code, h = _setup(**kw)
        assert code == 0, L.dtv_last_error().decode()
        out = np.full(8, -1, dtype=np.int32)
        assert L.dtv_dd_inner_counts(h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), None) == 0
        assert not out.any()
        sc = ctypes.c_int32()
        assert L.dtv_dd_schedule(h, ctypes.byref(sc)) == 0
        if kw:
            assert sc.value == 2  # the adaptive rule runs in the fused kernel
        L.dtv_dd_destroy(h)


def test_solve_rejects_missing_workspace_and_nulls():
    L = dtvdd.lib()
    code, h = _setup()
    assert code == 0
    dummy = ctypes.c_void_p(256)
    # null outputs -> EINVAL before anything is enqueued
    assert L.dtv_dd_solve(h, dummy, None, None, dummy, dummy, dummy, None, None, None) == dtvdd.DTV_EINVAL
    # no workspace bound -> ENOWS (nothing touches device memory)
    assert L.dtv_dd_solve(h, dummy, None, dummy, dummy, dummy, dummy, None, None, None) == dtvdd.DTV_ENOWS
    assert L.dtv_dd_backward(h, dummy, dummy, dummy, dummy, None) == dtvdd.DTV_ESTATE
    assert L.dtv_dd_bind_workspace(h, dummy, 1) == dtvdd.DTV_ENOWS
    L.dtv_dd_destroy(h)


def test_default_cuts_are_floor():
    L = dtvdd.lib()
    descs = (dtvdd.ImageDesc * 1)()
    descs[0] = dtvdd.ImageDesc(2000, 3000, 13, 20, None, None, 1.5)
    prm = dtvdd.Params(1, 1, 1, 50.0, 0.01, 10.0, 1 / 80, 1 / 400, 10, 5, 0, 0.0, 0, 0, 20, 0, 0)
    h = ctypes.c_void_p()
    assert L.dtv_dd_setup(descs, 1, ctypes.byref(prm), ctypes.byref(h)) == 0
    lay = dtvdd.Layout()
    L.dtv_dd_layout(h, 0, ctypes.byref(lay))
    assert lay.n_lam_h == 12 * 3000 and lay.n_lam_v == 19 * 2000
    L.dtv_dd_destroy(h)


def test_schedule_choice_reporting():
    """Before any solve the choice comes from the fixed rule; explicit
    parameters are reported as explicit (no GPU needed)."""
    L = dtvdd.lib()
    sc, r, src = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    code, h = _setup()
    assert code == 0
    assert L.dtv_dd_choice(h, ctypes.byref(sc), ctypes.byref(r), ctypes.byref(src)) == 0
    assert (r.value, src.value) == (16, 0)
    L.dtv_dd_destroy(h)
    code, h = _setup(schedule=1, rows=8)
    assert code == 0
    assert L.dtv_dd_choice(h, ctypes.byref(sc), ctypes.byref(r), ctypes.byref(src)) == 0
    assert (sc.value, r.value, src.value) == (1, 8, 3)
    L.dtv_dd_destroy(h)
    assert L.dtv_dd_choice(None, None, None, None) == dtvdd.DTV_EINVAL


def test_noalloc_validation_without_a_gpu():
    """dtv_dd_solve_noalloc rejects per-step host work (EINVAL) and plans whose
    workspace exceeds the library's scratch array (ENOWS) before touching a
    device; dtv_dd_status after no solve is OK."""
    L = dtvdd.lib()
    dummy = ctypes.c_void_p(256)
    code, h = _setup(diag_every=5)
    assert code == 0
    assert L.dtv_dd_solve_noalloc(h, dummy, None, dummy, dummy, dummy, dummy, None) == dtvdd.DTV_EINVAL
    assert "diagnostics" in L.dtv_last_error().decode()
    assert L.dtv_dd_status(h, None) == dtvdd.DTV_OK
    L.dtv_dd_destroy(h)
    # 2048^2 with the rotation buffers of the per-step schedules: about 100 MB of workspace
    code, h = _setup(H=2048, W=2048, rc=tuple(range(0, 2049, 128)), cc=tuple(range(0, 2049, 128)))
    assert code == 0
    nb = ctypes.c_size_t()
    assert L.dtv_dd_workspace_bytes(h, ctypes.byref(nb)) == 0 and nb.value > dtvdd.SCRATCH_BYTES
    assert L.dtv_dd_solve_noalloc(h, dummy, None, dummy, dummy, dummy, dummy, None) == dtvdd.DTV_ENOWS
    assert "scratch" in L.dtv_last_error().decode()
    assert L.dtv_dd_solve_noalloc(h, dummy, None, None, dummy, dummy, dummy, None) == dtvdd.DTV_EINVAL
    L.dtv_dd_destroy(h)


def test_scratch_size_matches_header():
    text = open(os.path.join(ROOT, "include", "dtvdd.h")).read()
    m = re.search(r"#define DTV_SCRATCH_BYTES \((\d+)u << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == dtvdd.SCRATCH_BYTES


def test_keep_records_workspace_and_schedule():
    """keep_records: the fused schedule without measuring, the records of every
    outer step (9 n_inner bytes per pixel) and the state before each in the
    workspace."""
    L = dtvdd.lib()
    big = dict(H=256, W=384, rc=(0, 128, 256), cc=(0, 128, 256, 384), save_for_backward=1, n_outer=30, n_inner=5)
    code, h0 = _setup(**big)
    assert code == 0, dtvdd.lib().dtv_last_error().decode()
    code, h1 = _setup(keep_records=1, **big)
    assert code == 0, dtvdd.lib().dtv_last_error().decode()
    n0, n1 = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.dtv_dd_workspace_bytes(h0, ctypes.byref(n0)) == 0
    assert L.dtv_dd_workspace_bytes(h1, ctypes.byref(n1)) == 0
    px = 256 * 384
    # the checkpointed plan keeps the records of one segment (20 outer steps) at most
    assert n1.value >= 30 * 9 * 5 * px and n1.value - n0.value >= 10 * 9 * 5 * px
    sch, rows, src = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    assert L.dtv_dd_choice(h1, ctypes.byref(sch), ctypes.byref(rows), ctypes.byref(src)) == 0
    assert sch.value == 2 and src.value == 0  # DTV_SCHED_FUSED by the rule
    assert _kernel_name(h1) == "k_fused_fista (recording)"
    L.dtv_dd_destroy(h0)
    L.dtv_dd_destroy(h1)
