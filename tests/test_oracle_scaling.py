"""Pins for the oracle's data equilibration (CPU only).

Sect. 5 states the goals of the scaling (columns of A_hat and b_hat with
norms near one, rows of A_hat and c_hat with similar norms, D constant on
every block of the cone that is not separable) and leaves the algorithm
open.  The oracle's rule (``oracle.scaling.equilibrate``) is pinned here by
facts fixed independently of its code:

* closed forms: on a diagonal matrix each pass maps an entry x to x^(1/4)
  (rows scaled by x^(-1/2), then columns by x^(-1/4)), so after P passes
  D = a^(-1/2 sum_k 4^-k) and E = a^(-1/4 sum_k 4^-k);
* hand-computed single passes: clipping of each factor to [1e-4, 1e4], the
  block mean on a second-order block, zero rows and columns left at 1;
* the definitions of sigma and rho: |b_hat| = 1 and |c_hat| = the mean row
  norm of A_hat;
* the goals of Sect. 5 on the random programs: D constant on every
  second-order, PSD, exponential and power block; column norms of A_hat in a
  narrow band; similar norms for the separable rows;
* mutants of the rule (a wrong exponent, a dropped clip, a dropped block
  mean, rho without the mean row norm) fail at least one of these checks.
"""

import inspect
import math
import textwrap

import numpy as np
import pytest
import scipy.sparse as sp

from datagen import draw_lp, draw_mixed, draw_socp
from oracle import cones as K
from oracle import scaling as SC
from oracle.instances import from_draw


def _col_norms(M):
    return np.sqrt(np.asarray(M.multiply(M).sum(axis=0))).ravel()


def _row_norms(M):
    return np.sqrt(np.asarray(M.multiply(M).sum(axis=1))).ravel()


def _programs():
    return [
        ("lp", from_draw(draw_lp(0))),
        ("socp", from_draw(draw_socp(0, n=1000, m=3000, nonneg=500, density=1e-2))),
        ("mixed", from_draw(draw_mixed(0, n=500, nonneg=200, n_soc=40, n_psd=6, psd_hi=20,
                                       n_exp=50, n_dexp=5, density=2e-2))),
    ]


# ---------------------------------------------------------------------------
# checks, each a function of the rule so that mutants can be run through them
# ---------------------------------------------------------------------------

def check_diagonal_closed_form(eq):
    a = np.array([0.01, 0.3, 1.0, 7.0, 100.0])
    A = sp.vstack([sp.diags(a), sp.csr_matrix((2, 5))]).tocsr()   # two zero rows
    cone = {"f": 0, "l": 7, "q": [], "s": [], "ep": 0, "ed": 0}
    s = eq(A, np.ones(7), np.ones(5), cone)
    geo = sum(4.0 ** -k for k in range(10))
    np.testing.assert_allclose(s.D[:5], a ** (-0.5 * geo), rtol=1e-13)
    np.testing.assert_allclose(s.E, a ** (-0.25 * geo), rtol=1e-13)
    np.testing.assert_array_equal(s.D[5:], 1.0)        # zero rows keep factor 1


def check_clip_single_pass(eq):
    cone = {"f": 0, "l": 1, "q": [], "s": [], "ep": 0, "ed": 0}
    big = sp.csr_matrix(np.array([[1e12]]))
    s = eq(big, np.ones(1), np.ones(1), cone, passes=1)
    # d = 1/sqrt(1e12) = 1e-6 clipped to 1e-4; the entry is then 1e8 and
    # e = 1/sqrt(1e8) = 1e-4 sits at the bound
    assert s.D[0] == 1e-4 and s.E[0] == 1e-4
    s = eq(big, np.ones(1), np.ones(1), cone, passes=2)
    # second pass: entry 1e4 -> d = 1e-2, entry 1e2 -> e = 1e-1
    np.testing.assert_allclose([s.D[0], s.E[0]], [1e-6, 1e-5], rtol=1e-15)
    small = sp.csr_matrix(np.array([[1e-12]]))
    s = eq(small, np.ones(1), np.ones(1), cone, passes=1)
    assert s.D[0] == 1e4 and s.E[0] == 1e4
    # both factors clipped: d = 1e-8 -> 1e-4, entry 1e12, e = 1e-6 -> 1e-4
    huge = sp.csr_matrix(np.array([[1e16]]))
    s = eq(huge, np.ones(1), np.ones(1), cone, passes=1)
    assert s.D[0] == 1e-4 and s.E[0] == 1e-4


def check_block_mean_single_pass(eq):
    # a second-order block of three rows with norms 1, 4, 16: d becomes the
    # mean of 1, 1/2, 1/4 on all three rows; a nonnegative row of norm 9
    # keeps its own 1/3
    A = sp.csr_matrix(np.array([[9.0, 0.0, 0.0, 0.0],
                                [1.0, 0.0, 0.0, 0.0],
                                [0.0, 4.0, 0.0, 0.0],
                                [0.0, 0.0, 16.0, 0.0]]))
    cone = {"f": 0, "l": 1, "q": [3], "s": [], "ep": 0, "ed": 0}
    s = eq(A, np.ones(4), np.ones(4), cone, passes=1)
    mean = (1.0 + 0.5 + 0.25) / 3.0
    np.testing.assert_allclose(s.D, [1.0 / 3.0, mean, mean, mean], rtol=1e-15)
    # columns of D A: (9/3, 1 mean) stacked in column 0, 4 mean, 16 mean; the
    # empty column 3 keeps 1
    k0 = math.hypot(3.0, mean)
    np.testing.assert_allclose(s.E, [1 / math.sqrt(k0), 1 / math.sqrt(4 * mean),
                                     1 / math.sqrt(16 * mean), 1.0], rtol=1e-15)


def check_sigma_rho(eq):
    for _, inst in _programs():
        s = eq(inst.A, inst.b, inst.c, inst.cone)
        Ah, bh, ch = SC.apply(inst.A, inst.b, inst.c, s)
        assert abs(np.linalg.norm(bh) - 1.0) <= 1e-14
        rbar = float(_row_norms(Ah).mean())
        assert abs(np.linalg.norm(ch) - rbar) <= 1e-13 * rbar


def check_goals(eq):
    for name, inst in _programs():
        s = eq(inst.A, inst.b, inst.c, inst.cone)
        Ah, _, _ = SC.apply(inst.A, inst.b, inst.c, s)
        for kind, a, L, _ in K.cone_blocks(inst.cone):
            if kind in ("soc", "psd", "exp", "dexp", "pow"):
                assert np.all(s.D[a:a + L] == s.D[a]), (name, kind, a)
        cn = _col_norms(Ah)
        cn = cn[cn > 0]
        # one common column norm to within 3 %, in [1, 1.5] (A_hat has three
        # rows per column here; Sect. 5: columns near unit norm)
        assert cn.max() / cn.min() <= 1.03, name
        assert 1.0 <= cn.min() and cn.max() <= 1.5, name
        # separable rows (nonnegative orthant): similar norms
        f_l = sum(L for kind, _, L, _ in K.cone_blocks(inst.cone) if kind in ("zero", "nonneg"))
        rn = _row_norms(Ah)[:f_l]
        rn = rn[rn > 0]
        assert rn.max() / rn.min() <= 1.2, name
        # every factor is finite and positive
        assert np.all(s.D > 0) and np.all(s.E > 0)


CHECKS = [check_diagonal_closed_form, check_clip_single_pass, check_block_mean_single_pass,
          check_sigma_rho, check_goals]


@pytest.mark.parametrize("check", CHECKS, ids=lambda f: f.__name__)
def test_rule(check):
    check(SC.equilibrate)


def test_identity_when_disabled():
    inst = from_draw(draw_lp(1))
    s = SC.equilibrate(inst.A, inst.b, inst.c, inst.cone, enabled=False)
    assert np.all(s.D == 1.0) and np.all(s.E == 1.0) and s.sigma == 1.0 and s.rho == 1.0


def test_power_blocks_get_one_factor():
    d = draw_mixed(3, n=60, nonneg=20, n_soc=3, soc_lo=3, soc_hi=5, n_psd=1, psd_lo=3,
                   psd_hi=3, n_exp=2, n_dexp=0, n_pow=4, density=0.2)
    inst = from_draw(d)
    s = SC.equilibrate(inst.A, inst.b, inst.c, inst.cone)
    n_blocks = 0
    for kind, a, L, _ in K.cone_blocks(inst.cone):
        if kind == "pow":
            n_blocks += 1
            assert np.all(s.D[a:a + 3] == s.D[a])
    assert n_blocks == 4


# ---------------------------------------------------------------------------
# planted mistakes: each mutant of the rule must fail some check
# ---------------------------------------------------------------------------

def _mutant(old: str, new: str):
    src = textwrap.dedent(inspect.getsource(SC.equilibrate))
    assert old in src, old
    ns = dict(vars(SC))
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)  # noqa: S102
    return ns["equilibrate"]


MUTANTS = {
    "exponent 1 on rows": ("d[pos] = 1.0 / np.sqrt(r[pos])", "d[pos] = 1.0 / r[pos]"),
    "exponent 1 on columns": ("e[pos] = 1.0 / np.sqrt(k[pos])", "e[pos] = 1.0 / k[pos]"),
    "row clip dropped": ("d = np.clip(d, lo, hi)", "d = d"),
    "column clip dropped": ("e = np.clip(e, lo, hi)", "e = e"),
    "block mean dropped": ("d[a:a + L] = d[a:a + L].mean()", "pass"),
    "rho without the mean row norm": ("rho = rbar /", "rho = 1.0 /"),
    "sigma on b instead of D b": ("np.linalg.norm(D * b)", "np.linalg.norm(b)"),
    "columns before rows": ("D = D * d", "D = D * 1.0"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    eq = _mutant(*MUTANTS[name])
    failed = []
    for check in CHECKS:
        try:
            check(eq)
        except AssertionError:
            failed.append(check.__name__)
    assert failed, f"mutant '{name}' passed every check"
