"""Pins of the oracle's basis functions against what the paper prints and
against independent mathematics (library routines, symbolic differentiation,
finite differences, normalisation integrals)."""
import math

import numpy as np
import pytest
import sympy as sp
from scipy import integrate

from conftest import golden_lines

xs, ys = sp.symbols("x y", real=True)
rs = sp.sqrt(xs ** 2 + ys ** 2)


def _pts(n=12, seed=0):
    rng = np.random.default_rng(seed)
    ang = rng.uniform(0, 2 * np.pi, n)
    rad = rng.uniform(0.2, 1.95, n)
    return rad * np.cos(ang), rad * np.sin(ang)


def _sym(expr):
    return sp.sympify(expr, locals={"x": xs, "y": ys, "r": rs})


def test_p_of_k_matches_sec31(O):
    for ln in golden_lines("p_of_k_sec31.txt"):
        k, p = map(int, ln.split())
        assert O.p_of_k(k) == p
    assert O.p_of_k(8) == 44


def test_ncrit_matches_sec32(O):
    for ln in golden_lines("ncrit_sec32.txt"):
        k, n = map(int, ln.split())
        assert O.ncrit(k) == n


def test_monomials_match_eq1(O):
    exprs = [_sym(e) for e in golden_lines("monomials_eq1.txt")]
    for px, py in zip(*_pts()):
        X = O.monomials(4, px, py)
        ref = [float(e.subs({xs: px, ys: py})) for e in exprs]
        np.testing.assert_allclose(X[:10], ref, rtol=1e-15, atol=1e-15)


def test_monomials_are_taylor_coefficients(O):
    # eq. (tsc): f(r_j) = f(r_i) + X(r_ji) . D f(r_i) exactly for a polynomial of
    # degree <= k; check with a random degree-6 polynomial and symbolic derivatives
    k = 6
    rng = np.random.default_rng(3)
    terms = [(a, n - a) for n in range(0, k + 1) for a in range(n, -1, -1)]
    coef = rng.standard_normal(len(terms))
    f = sum(c * xs ** a * ys ** b for c, (a, b) in zip(coef, terms))
    xi, yi = 0.3, -0.2
    idx = O.index_table(k)
    D = np.array([float(sp.diff(f, xs, a, ys, b).subs({xs: xi, ys: yi})) if (a or b) else 0.0
                  for a, b in idx])
    for dx, dy in zip(*_pts(5, 1)):
        X = O.monomials(k, dx, dy)
        lhs = float(f.subs({xs: xi + dx, ys: yi + dy}))
        rhs = float(f.subs({xs: xi, ys: yi})) + X @ D
        assert abs(lhs - rhs) < 1e-11 * max(1.0, abs(lhs))


def test_hermite_matches_numpy(O):
    from numpy.polynomial import hermite as H

    for t in (-1.7, -0.3, 0.0, 0.45, 1.9):
        got = O.hermite(8, t)
        for n in range(9):
            c = np.zeros(n + 1)
            c[n] = 1.0
            assert got[n] == pytest.approx(H.hermval(t, c), rel=1e-13, abs=1e-12)


@pytest.mark.parametrize("rbf,expected", [(1, 1.0), (3, 1.0), (4, 1.0), (2, 0.5), (0, 4 * math.pi / 7)])
def test_rbf_normalisation(O, rbf, expected):
    # App. A eq. (unity): 2 pi int_0^2 q W0 dq = 1 for cone, Wendland C6, Gaussian.
    # The quadratic's printed constant 3/(16 pi) integrates to 1/2 (constant cancels in w).
    # Wendland C2 (1-q/2)^4 (1+2q) without constant: 4 pi / 7 (textbook 7/(4 pi h^2)).
    val, _ = integrate.quad(lambda q: 2 * math.pi * q * O.rbf_derivs(rbf, q)[0], 0, 2, epsabs=1e-14,
                            epsrel=1e-13, limit=200)
    assert val == pytest.approx(expected, rel=1e-10 if rbf != 4 else 1e-12)


@pytest.mark.parametrize("rbf", [0, 1, 2, 3, 4])
def test_rbf_derivatives_finite_difference(O, rbf):
    for q in (0.3, 0.9, 1.4, 1.8):
        f = O.rbf_derivs(rbf, q)
        for d in range(3):
            hstep = 1e-5
            fd = (O.rbf_derivs(rbf, q + hstep)[d] - O.rbf_derivs(rbf, q - hstep)[d]) / (2 * hstep)
            assert f[d + 1] == pytest.approx(fd, rel=1e-7, abs=1e-8)


def test_compact_rbfs_vanish_at_support(O):
    # App. A: W0(2) = 0 for the compact RBFs; the quadratic and Wendland also have dW0/dq(2) = 0
    for rbf in (0, 1, 2, 3):
        assert O.rbf_derivs(rbf, 2.0 - 1e-12)[0] == pytest.approx(0.0, abs=1e-11)
    for rbf in (0, 2, 3):
        assert O.rbf_derivs(rbf, 2.0 - 1e-9)[1] == pytest.approx(0.0, abs=1e-7)
    g = O.rbf_derivs(4, 2.0)[0]
    assert g == pytest.approx(6.6e-16, rel=0.05)  # App. A: W^G(2) ~ 6.6e-16


def test_conic_abfs_match_eq_conic_abs(O):
    exprs = [_sym(e) for e in golden_lines("conic_abfs_eq_conic_abs.txt")]
    fac = -3.0 / (8.0 * math.pi)
    for px, py in zip(*_pts()):
        W = O.abfs(4, px, py, family=O.ABF_PAPER, rbf=O.RBF_CONE)
        ref = [fac * float(e.subs({xs: px, ys: py})) for e in exprs]
        np.testing.assert_allclose(W, ref, rtol=1e-13, atol=1e-14)


def test_printed_conic_list_is_derivatives_of_r(O):
    # independent of the print: bracket B1 element (a,b) equals d^(a,b) r
    exprs = [_sym(e) for e in golden_lines("conic_abfs_eq_conic_abs.txt")]
    idx = O.index_table(4)
    for e, (a, b) in zip(exprs, idx):
        d = sp.diff(rs, xs, a, ys, b) if b else sp.diff(rs, xs, a)
        if a == 0:
            d = sp.diff(rs, ys, b)
        assert sp.simplify(d - e) == 0


@pytest.mark.parametrize("rbf", [2, 3, 0])
def test_paper_abfs_low_orders_match_appendix(O, rbf):
    b2, b3 = [ln.split("|")[1].split(";") for ln in golden_lines("appendix_a_brackets.txt")]
    b1 = golden_lines("conic_abfs_eq_conic_abs.txt")[:9]
    B = [[_sym(e) for e in br] for br in (b1, b2, b3)]
    for px, py in zip(*_pts(8, 2)):
        q = math.hypot(px, py)
        f = O.rbf_derivs(rbf, q)
        W = O.abfs(3, px, py, family=O.ABF_PAPER, rbf=rbf)
        ref = [sum(f[i + 1] * float(B[i][m].subs({xs: px, ys: py})) for i in range(3)) for m in range(9)]
        np.testing.assert_allclose(W, ref, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("rbf", [2, 3])
def test_paper_abfs_are_derivatives_of_w0(O, rbf):
    """Elements of order <= 3 are full derivatives D(W0) (Sec. 3.2); elements of
    order >= 4 keep only dW0/dr * d^(a,b) r (App. A truncation).  Symbolic check."""
    qq = sp.symbols("qq", positive=True)
    if rbf == 2:
        W0q = sp.Rational(3, 16) / sp.pi * (qq - 2) ** 2
    else:
        W0q = sp.Rational(78, 28) / sp.pi * (1 - qq / 2) ** 8 * (4 * qq ** 3 + sp.Rational(25, 4) * qq ** 2 + 4 * qq + 1)
    W0 = W0q.subs(qq, rs)
    dW0 = sp.diff(W0q, qq)
    k = 8
    idx = O.index_table(k)
    pts = list(zip(*_pts(4, 5)))
    for m, (a, b) in enumerate(idx):
        n = a + b
        if n <= 3:
            e = W0
            if a:
                e = sp.diff(e, xs, a)
            if b:
                e = sp.diff(e, ys, b)
        else:
            e = dW0.subs(qq, rs) * (sp.diff(sp.diff(rs, xs, a), ys, b) if a and b else
                                    (sp.diff(rs, xs, a) if a else sp.diff(rs, ys, b)))
        fn = sp.lambdify((xs, ys), e, "mpmath")
        for px, py in pts:
            W = O.abfs(k, px, py, family=O.ABF_PAPER, rbf=rbf)
            ref = float(fn(px, py))
            assert W[m] == pytest.approx(ref, rel=1e-11, abs=1e-11 * (1 + abs(ref))), (m, a, b)


def test_hermite_family_definition(O):
    from numpy.polynomial import hermite as H

    k = 8
    idx = O.index_table(k)
    for px, py in zip(*_pts(5, 7)):
        for sigma in (1.0, 1.5):
            W = O.abfs(k, px, py, family=O.ABF_HERMITE, rbf=O.RBF_WENDLAND_C2, sigma=sigma)
            q = math.hypot(px, py)
            phi = (1 - q / 2) ** 4 * (1 + 2 * q)
            for m, (a, b) in enumerate(idx):
                ca = np.zeros(a + 1)
                ca[a] = 1
                cb = np.zeros(b + 1)
                cb[b] = 1
                ref = H.hermval(sigma * px, ca) * H.hermval(sigma * py, cb) * phi
                assert W[m] == pytest.approx(ref, rel=1e-12, abs=1e-12)


def test_paper_abfs_undefined_at_origin(O):
    with pytest.raises(ValueError):
        O.abfs(4, 0.0, 0.0, family=O.ABF_PAPER, rbf=O.RBF_QUADRATIC)
    W = O.abfs(4, 0.0, 0.0, family=O.ABF_HERMITE)
    assert np.all(np.isfinite(W))


@pytest.mark.parametrize("rbf", [2, 3])
def test_paper_d1_family_is_dw0_times_derivatives_of_r(O, rbf):
    """PAPER_D1 keeps only the dW0/dr term in every element (the App. A
    truncation from the first element on): W_m = W0'(|d|) d^(a,b) |d|.
    Checked symbolically, and against the cone family, whose ABFs are exactly
    that shape with a constant W0' (eq. conic_abs)."""
    qq = sp.symbols("qq", positive=True)
    if rbf == 2:
        W0q = sp.Rational(3, 16) / sp.pi * (qq - 2) ** 2
    else:
        W0q = sp.Rational(78, 28) / sp.pi * (1 - qq / 2) ** 8 * (4 * qq ** 3 + sp.Rational(25, 4) * qq ** 2 + 4 * qq + 1)
    dW0 = sp.diff(W0q, qq)
    k = 8
    idx = O.index_table(k)
    pts = list(zip(*_pts(4, 9)))
    for m, (a, b) in enumerate(idx):
        dr = rs
        if a:
            dr = sp.diff(dr, xs, a)
        if b:
            dr = sp.diff(dr, ys, b)
        fn = sp.lambdify((xs, ys), dW0.subs(qq, rs) * dr, "mpmath")
        for px, py in pts:
            W = O.abfs(k, px, py, family=O.ABF_PAPER_D1, rbf=rbf)
            ref = float(fn(px, py))
            assert W[m] == pytest.approx(ref, rel=1e-11, abs=1e-11 * (1 + abs(ref))), (m, a, b)
    # cone: W0' = -3/(8 pi) is constant, so PAPER_D1 = PAPER; quadratic: W0'(q) / W0'_cone = 2 - q
    for px, py in zip(*_pts(6, 10)):
        q = math.hypot(px, py)
        cone = O.abfs(k, px, py, family=O.ABF_PAPER, rbf=O.RBF_CONE)
        np.testing.assert_allclose(O.abfs(k, px, py, family=O.ABF_PAPER_D1, rbf=O.RBF_CONE), cone,
                                   rtol=1e-13, atol=1e-14)
        np.testing.assert_allclose(O.abfs(k, px, py, family=O.ABF_PAPER_D1, rbf=O.RBF_QUADRATIC), (2 - q) * cone,
                                   rtol=1e-12, atol=1e-13)
    # elements of order 1, and of order >= 4, are the same in both PAPER families
    for px, py in zip(*_pts(3, 11)):
        a_ = O.abfs(k, px, py, family=O.ABF_PAPER, rbf=rbf)
        b_ = O.abfs(k, px, py, family=O.ABF_PAPER_D1, rbf=rbf)
        keep = [m for m, (a, b) in enumerate(idx) if a + b == 1 or a + b >= 4]
        np.testing.assert_allclose(b_[keep], a_[keep], rtol=1e-13, atol=1e-14)
