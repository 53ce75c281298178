"""Eigen-spectra of the convective operator A^x (Sec. 4.2, Fig. eigens_convect)
from the oracle's d/dx weights.

A^x is the global matrix of the d/dx operator in difference form
(A_ij = w_ij for j in row i, A_ii = -sum_j w_ij) on a 441-node (21 x 21)
periodic Cartesian set (periodic images give every stencil full support), with
h/dr = 2, orders k = 2, 4, 6, ABFs from the conic, quadratic, Wendland C6 and
Gaussian RBFs (every element keeps the dW0/dr term, the family that reproduces
Table noise_limits), noise eps/dr = 0.5 read as per-coordinate jitter of
half-width 0.25 dr.  Trends the paper states that these spectra reproduce:

* ideal lattice: the conic ABFs give substantially non-zero real parts, the
  quadratic and Wendland ABFs put every eigenvalue on the imaginary axis to
  rounding (dW0/dr = 0 at the edge of the support);
* noisy lattice: the real parts are significant for every ABF; at k = 4 and 6
  the quadratic ABFs lie closer to the imaginary axis than the conic ones and
  the Gaussian ABFs worst of all; at k = 6 the order is quadratic < conic <
  Wendland < Gaussian, the paper's;
* lower k lies closer to the imaginary axis (conic, quadratic, Gaussian).

Not reproduced, and recorded as such: the Gaussian's ideal-lattice real parts
"several orders of magnitude" above the quadratic and Wendland ones (ours sit
at rounding: with W(2) = 6.6e-16 the edge effect is below it), and at k = 4 the
Wendland ABFs lie closer to the axis than the quadratic ones."""
import numpy as np
import pytest

from paper_1912_06441_amd import workloads as WL

RBFS = ("cone", "quad", "wend", "gauss")


def _rbf(O, name):
    return {"cone": O.RBF_CONE, "quad": O.RBF_QUADRATIC, "wend": O.RBF_WENDLAND_C6, "gauss": O.RBF_GAUSSIAN}[name]


def global_matrix(rp, col, w):
    n = rp.size - 1
    A = np.zeros((n, n))
    for i in range(n):
        for q in range(rp[i], rp[i + 1]):
            A[i, col[q]] += w[q]
            A[i, i] -= w[q]
    return A


def max_real(O, seed, eps, k, rbf):
    """max |Re lambda| * dr of A^x (and max |Im lambda| * dr)."""
    x, y, s = WL.jittered_lattice(21, eps=eps, seed=seed, periodic=True)
    dom = WL.unit_domain(True)
    n = x.size
    order = np.full(n, k, np.int8)
    rp, col, R = O.neighbours(x, y, dom, np.full(n, 4.0 * s), order, grow=False)
    w, st, res, _ = O.weights(x, y, dom, R, order, rp, col, family=O.ABF_PAPER_D1, rbf=_rbf(O, rbf), ops=O.OP_DX)
    assert np.all(st == O.ST_OK)
    ev = np.linalg.eigvals(global_matrix(rp, col, w[0])) * s
    return float(np.abs(ev.real).max()), float(np.abs(ev.imag).max())


@pytest.fixture(scope="module")
def spectra(O):
    out = {}
    for seed in (3, 4):
        for eps in (0.0, 0.25):
            for k in (2, 4, 6):
                for r in RBFS:
                    if eps == 0.0 and seed != 3:
                        continue
                    out[(seed, eps, k, r)] = max_real(O, seed, eps, k, r)
    return out


def test_ideal_lattice_conic_off_axis_quadratic_wendland_on_axis(spectra):
    for k in (2, 4, 6):
        re_c, im_c = spectra[(3, 0.0, k, "cone")]
        assert re_c >= 1e-2 and im_c > 0.3
        for r in ("quad", "wend"):
            re, im = spectra[(3, 0.0, k, r)]
            assert re <= 1e-12 * im and re_c >= 1e10 * re, (k, r, re, im)


def test_noisy_lattice_real_parts_and_ordering(spectra):
    for seed in (3, 4):
        for k in (2, 4, 6):
            for r in RBFS:
                assert spectra[(seed, 0.25, k, r)][0] >= 1e-2  # significant for every ABF
        for k in (4, 6):
            re = {r: spectra[(seed, 0.25, k, r)][0] for r in RBFS}
            assert re["quad"] < re["cone"] < re["gauss"], (seed, k, re)
            assert re["gauss"] == max(re.values())
        re6 = {r: spectra[(seed, 0.25, 6, r)][0] for r in RBFS}
        assert re6["quad"] < re6["cone"] < re6["wend"] < re6["gauss"], (seed, re6)


def test_lower_order_closer_to_the_imaginary_axis(spectra):
    for seed in (3, 4):
        for r in ("cone", "quad", "gauss"):
            re = [spectra[(seed, 0.25, k, r)][0] for k in (2, 4, 6)]
            assert re[0] < re[1] < re[2], (seed, r, re)
    re = [spectra[(3, 0.0, k, "cone")][0] for k in (2, 4, 6)]
    assert re[0] < re[1] < re[2]


def test_global_matrix_rows_apply_the_operator(O):
    """A^x u equals the operator applied to u (eq. general_do), so the spectra
    above are those of the discrete operator."""
    x, y, s = WL.jittered_lattice(21, eps=0.25, seed=3, periodic=True)
    dom = WL.unit_domain(True)
    order = np.full(x.size, 4, np.int8)
    rp, col, R = O.neighbours(x, y, dom, np.full(x.size, 4.0 * s), order, grow=False)
    w, st, _, _ = O.weights(x, y, dom, R, order, rp, col, family=O.ABF_PAPER_D1, rbf=O.RBF_QUADRATIC, ops=O.OP_DX)
    u = np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
    A = global_matrix(rp, col, w[0])
    assert np.allclose(A @ u, O.apply(rp, col, w[0], u), rtol=0, atol=1e-12 * np.abs(A @ u).max())
