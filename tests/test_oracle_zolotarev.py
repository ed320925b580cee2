"""Pins of the Zolotarev coefficients of the oracle (CPU).

Each test checks ``oracle.zolotarev`` against something other than itself:
the closed form of the r = 1 case (QDWH's dynamically weighted Halley
function), the equioscillation that characterises a best approximation, the
bounds 0 <= Z <= 1 of Sec. 5.1, the composition rule of Sec. 5 (two type
(2r+1, 2r) steps give the type ((2r+1)^2, (2r+1)^2 - 1) best approximation),
and the paper's statement that r <= 8 terms reach 1 - O(u) on [1e-15, 1].
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import zolotarev as Z


def qdwh_coeffs(ell):
    """QDWH weights (a, b, c) of f(x) = x (a + b x^2) / (1 + c x^2) (Nakatsukasa-Bai-Gygi)."""
    with mp.workdps(60):
        l = mp.mpf(ell)
        d = mp.cbrt(4 * (1 - l * l) / l ** 4)
        a = mp.sqrt(1 + d) + mp.sqrt(8 - 4 * d + 8 * (2 - l * l) / (l * l * mp.sqrt(1 + d))) / 2
        b = (a - 1) ** 2 / 4
        c = a + b - 1
        return a, b, c


@pytest.mark.parametrize("ell", [0.9, 0.5, 1e-1, 1e-3, 1e-6, 1e-10, 1e-15])
def test_r1_matches_qdwh_closed_form(ell):
    # x (a + b x^2)/(1 + c x^2) = (b/c) x (x^2 + a/b)/(x^2 + 1/c): c_1 = 1/c, c_2 = a/b, M = b/c.
    c, a_pf, M, _ = Z.coeffs_mp(ell, 1)
    qa, qb, qc = qdwh_coeffs(ell)
    with mp.workdps(60):
        assert abs(c[0] / (1 / qc) - 1) < mp.mpf("1e-40")
        assert abs(c[1] / (qa / qb) - 1) < mp.mpf("1e-40")
        assert abs(M / (qb / qc) - 1) < mp.mpf("1e-40")


def _extrema(fun, lo, hi, npts=4000):
    """Local extrema of fun on [lo, hi] (log-spaced grid, refined by golden search)."""
    xs = np.exp(np.linspace(math.log(lo), math.log(hi), npts))
    ys = np.array([fun(x) for x in xs])
    pts = [(lo, ys[0])]
    for i in range(1, npts - 1):
        if (ys[i] - ys[i - 1]) * (ys[i + 1] - ys[i]) < 0:
            sign = 1 if ys[i] > ys[i - 1] else -1
            f = lambda t: -sign * fun(t)
            # refine with a bracketed golden-section search on [xs[i-1], xs[i+1]]
            a, b = xs[i - 1], xs[i + 1]
            g = (math.sqrt(5) - 1) / 2
            for _ in range(80):
                c1 = b - g * (b - a)
                c2 = a + g * (b - a)
                if f(c1) < f(c2):
                    b = c2
                else:
                    a = c1
            x = 0.5 * (a + b)
            pts.append((x, fun(x)))
    pts.append((hi, ys[-1]))
    return pts


@pytest.mark.parametrize("r", [1, 2, 3, 5, 8])
@pytest.mark.parametrize("ell", [1e-1, 1e-4, 1e-8])
def test_equioscillation(r, ell):
    """A best approximation of type (2r+1, 2r) to 1 on [ell, 1] alternates 2r+2 times."""
    step = Z.ZoloStep(ell, r)
    fun = lambda x: float(Z.eval_product(x, step.c_mp, step.M_mp))
    pts = _extrema(fun, ell, 1.0, npts=6000)
    vals = np.array([v for _, v in pts])
    assert len(pts) == 2 * r + 2, (len(pts), pts)
    top = vals[1::2]     # ordered from x = ell: minimum, maximum, minimum, ..., maximum at x = 1
    bot = vals[0::2]
    assert np.allclose(top, 1.0, rtol=0, atol=1e-12)
    assert np.allclose(bot, bot[0], rtol=0, atol=1e-12 + 1e-9 * (1 - bot[0]))
    assert abs(pts[-1][0] - 1.0) == 0 and abs(vals[-1] - 1.0) < 1e-14


@pytest.mark.parametrize("r", [1, 2, 4, 8])
@pytest.mark.parametrize("ell", [1e-15, 1e-6, 0.3])
def test_bounds_zero_one(r, ell):
    """Sec. 5.1: 0 <= Z(x) <= 1 on [0, 1], Z(1) = 1, Z(ell) = ell_next."""
    step = Z.ZoloStep(ell, r)
    xs = np.concatenate([np.linspace(0, 1, 2001), np.exp(np.linspace(math.log(1e-18), 0, 2001))])
    vals = np.array([step(x) for x in xs])
    assert vals.min() >= 0.0
    assert vals.max() <= 1.0 + 1e-15
    assert abs(step(1.0) - 1.0) < 1e-15
    assert abs(step(ell) - step.ell_next) <= 1e-15 * step.ell_next


@pytest.mark.parametrize("r", [1, 3, 8])
def test_partial_fraction_identity(r):
    step = Z.ZoloStep(1e-5, r)
    with mp.workdps(60):
        for x in ["1e-7", "1e-5", "0.001", "0.3", "0.99", "1", "1.5"]:
            p = Z.eval_product(mp.mpf(x), step.c_mp, step.M_mp)
            q = Z.eval_partial(mp.mpf(x), step.c_mp, step.a_mp, step.M_mp)
            assert abs(p - q) <= mp.mpf("1e-45") * abs(p)


@pytest.mark.parametrize("r", [1, 2])
def test_composition_is_best_approximation(r):
    """Sec. 5: Z(Z(x; l); l_1) is the type ((2r+1)^2, .) best approximation: (2r+1)^2 + 1 alternations."""
    ell = 1e-3
    s1 = Z.ZoloStep(ell, r)
    s2 = Z.ZoloStep(s1.ell_next, r)
    fun = lambda x: float(Z.eval_product(Z.eval_product(x, s1.c_mp, s1.M_mp), s2.c_mp, s2.M_mp))
    pts = _extrema(fun, ell, 1.0, npts=20000)
    assert len(pts) == (2 * r + 1) ** 2 + 1


def test_paper_eps_needs_at_most_eight_terms():
    """Sec. 5 / 5.1: with eps = 1e-15, two type (17, 16) steps map [eps, 1] to 1 - O(u)."""
    s1, s2, resid = Z.two_step(1e-15, 8)
    assert float(resid) <= Z.U_DOUBLE
    assert Z.choose_r(1e-15) == 8
    # ... and the degree really is needed: seven terms fall short of u
    assert float(Z.two_step(1e-15, 7)[2]) > Z.U_DOUBLE


def test_degree_grows_with_condition():
    rs = [Z.choose_r(l) for l in [0.5, 1e-2, 1e-4, 1e-8, 1e-12]]
    assert rs == sorted(rs)
    assert rs[0] >= 1 and rs[-1] <= 8


def test_weights_positive_and_shifts_interlace():
    for r in [1, 4, 8]:
        for ell in [1e-15, 1e-3, 0.5]:
            st = Z.ZoloStep(ell, r)
            assert all(a > 0 for a in st.a)
            assert all(st.c[i] < st.c[i + 1] for i in range(2 * r - 1))
