"""The scalar pins catch the slips they exist for.

Each case plants one plausible mistake in a copy of the oracle's source
(halved sigma in the multiplier update, halved tau in the anchor, a halved
proximal weight in the local FISTA gradient, 2 tau in the local primal-dual
anchor prox, the extrapolation 2p~^n - p~^(n-1) dropped, B^* with the wrong
sign), builds the copy with gcc into a temporary directory and runs the pins
of tests/test_oracle_scalars.py against it: every mutant must fail them by a
wide margin, while the unmodified oracle passes them (that test file).
Only the oracle is modified, only on the CPU.
"""
import os

import pytest

import oracle
from test_oracle_scalars import CASES, saddle_errors

with open(oracle.SRC_PATH) as fh:
    SRC = fh.read()

# (name, local solver the slip lives in, [(original text, planted text), ...])
MUTANTS = [
    ("sigma/2 in the multiplier update", "FISTA", [
        ("st->lam_h[e] += P->sigma * (", "st->lam_h[e] += 0.5 * P->sigma * ("),
        ("st->lam_v[e] += P->sigma * (", "st->lam_v[e] += 0.5 * P->sigma * (")]),
    ("tau/2 in the anchor phat", "FISTA", [
        ("-= P->tau * st->lam_h[e];", "-= 0.5 * P->tau * st->lam_h[e];"),
        ("+= P->tau * st->lam_h[e];", "+= 0.5 * P->tau * st->lam_h[e];"),
        ("-= P->tau * st->lam_v[e];", "-= 0.5 * P->tau * st->lam_v[e];"),
        ("+= P->tau * st->lam_v[e];", "+= 0.5 * P->tau * st->lam_v[e];")]),
    ("halved proximal term in the local FISTA gradient", "FISTA", [
        ("(y1[e] - S->h1[e]) * inv_tau;", "(y1[e] - S->h1[e]) * 0.5 * inv_tau;"),
        ("(y2[e] - S->h2[e]) * inv_tau;", "(y2[e] - S->h2[e]) * 0.5 * inv_tau;")]),
    ("2 tau in the local primal-dual anchor prox", "CP2", [
        ("proj_box((P->tau * pbar + tk * S->h1[e]) / (P->tau + tk))",
         "proj_box((2.0 * P->tau * pbar + tk * S->h1[e]) / (2.0 * P->tau + tk))"),
        ("proj_box((P->tau * pbar + tk * S->h2[e]) / (P->tau + tk))",
         "proj_box((2.0 * P->tau * pbar + tk * S->h2[e]) / (2.0 * P->tau + tk))")]),
    ("extrapolation dropped (B p~^n instead of B(2p~^n - p~^(n-1)))", "CP2", [
        ("((2.0 * *ps - st->prev_hs[e]) - (2.0 * *pt - st->prev_ht[e]))", "(*ps - *pt)"),
        ("((2.0 * *ps - st->prev_vs[e]) - (2.0 * *pt - st->prev_vt[e]))", "(*ps - *pt)")]),
    ("B^* with the sign of each copy swapped", "FISTA", [
        ("s->h1[s->h * s->w + (j - s->ca)] -= P->tau", "s->h1[s->h * s->w + (j - s->ca)] += P->tau"),
        ("t->h1[0 * t->w + (j - t->ca)] += P->tau", "t->h1[0 * t->w + (j - t->ca)] -= P->tau")]),
]


@pytest.mark.parametrize("name,inner,edits", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_fails_the_scalar_pins(name, inner, edits, tmp_path):
    src = SRC
    for old, new in edits:
        assert src.count(old) == 1, f"mutation site not found once: {old!r}"
        src = src.replace(old, new)
    path = tmp_path / "mutant.c"
    path.write_text(src)
    lib = oracle.build(out_path=str(tmp_path / "libmutant.so"), src=str(path))
    worst = 0.0
    for case in CASES:
        worst = max(worst, float(max(saddle_errors(inner, case, n_outer=3, lib_path=lib))))
    assert worst > 1e-4, f"{name}: largest deviation {worst:.2e} (the pins do not see this slip)"
    os.remove(lib)
