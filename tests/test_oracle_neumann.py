"""Pins of the oracle's Neumann rows (Sec. 5.2, eq. neu and the ghost-node rows).

Poisson's equation on the unit square with Neumann walls at x = 0, 1 and
Dirichlet walls at y = 0, 1; one ghost node per Neumann wall node at
r_b - n_b dr, whose row of the enlarged global system is the wall node's
discrete normal derivative.

* Each ghost row applied to a field equals n_x L^x + n_y L^y at its parent
  (eq. general_do with the parent's d/dx and d/dy weights).
* Exactness: the discrete operators reproduce polynomials of degree <= k, so
  every row holds exactly for a degree-k solution and the solve returns it at
  every node, ghosts included (k = 2 and 4).
* A smooth solution converges at about k (k = 2, 4; the wall stencils are
  one-sided at order min(k, 4)).
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spl

from oracle import poisson as P
from paper_1912_06441_amd import workloads as WL


def neumann_case(O, k, side, seed=13):
    cfg = WL.config("poisson")
    nd = WL.neumann_square_nodes(side, eps_over_dr=cfg["eps_paper"], seed=seed)
    x, y, s, dom = nd["x"], nd["y"], nd["s"], nd["domain"]
    order = np.full(x.size, k, np.int8)
    rp, col, R = O.neighbours(x, y, dom, 2.0 * cfg["h_over_dr"][k] * s, order, grow=True)
    w, st, _, _ = O.weights(x, y, dom, R, order, rp, col, family=cfg["abf"], rbf=cfg["rbf"],
                            ops=O.OP_DX | O.OP_DY | O.OP_LAP)
    used = (nd["kind"] == 0) | (nd["kind"] == 2)  # rows that use their own weights
    assert np.all(st[used] == O.ST_OK)
    return nd, rp, col, R, w


def _solve(nd, rp, col, w, fields):
    F, x0, fixed = WL.neumann_system(nd, *fields)
    A = P.neumann_matrix(rp, col, w[0], w[1], w[2], nd["parent"], nd["nx"], nd["ny"], fixed)
    return A, F, x0, spl.spsolve(A.tocsc(), F)


def test_ghost_rows_are_normal_derivatives(O):
    nd, rp, col, R, w = neumann_case(O, 4, 16)
    F, x0, fixed = WL.neumann_system(nd, *WL.neumann_poly(2))
    A = P.neumann_matrix(rp, col, w[0], w[1], w[2], nd["parent"], nd["nx"], nd["ny"], fixed)
    u = np.random.default_rng(2).standard_normal(nd["x"].size)
    Au = A @ u
    g = np.nonzero(nd["kind"] == 3)[0]
    p = nd["parent"][g]
    want = nd["nx"][g] * O.apply(rp, col, w[0], u)[p] + nd["ny"][g] * O.apply(rp, col, w[1], u)[p]
    assert g.size == 2 * (16 - 1)
    assert np.allclose(Au[g], want, rtol=0, atol=1e-12 * np.abs(want).max())
    free = (nd["kind"] == 0) | (nd["kind"] == 2)
    assert np.allclose(Au[free], O.apply(rp, col, w[2], u)[free], rtol=0, atol=1e-12 * np.abs(Au[free]).max())
    d = nd["kind"] == 1
    assert np.array_equal(Au[d], u[d])


@pytest.mark.parametrize("k", [2, 4])
def test_polynomial_solution_reproduced(O, k):
    nd, rp, col, R, w = neumann_case(O, k, 20)
    fields = WL.neumann_poly(k)
    A, F, x0, phi = _solve(nd, rp, col, w, fields)
    exact = fields[0](nd["x"], nd["y"])
    assert np.abs(phi - exact).max() <= 1e-8 * np.abs(exact).max()
    xb, it, res, ok = P.bicgstab(A, F, x0=x0, tol=1e-12)
    assert ok and np.abs(xb - exact).max() <= 1e-8 * np.abs(exact).max()


@pytest.mark.parametrize("k,rate", [(2, 2.0), (4, 4.0)])
def test_neumann_convergence(O, k, rate):
    errs = []
    for side in (20, 40, 80):
        nd, rp, col, R, w = neumann_case(O, k, side)
        A, F, x0, phi = _solve(nd, rp, col, w, (lambda a, b: WL.neumann_field(a, b)[0],
                                                lambda a, b: WL.neumann_field(a, b)[1],
                                                lambda a, b: WL.neumann_field(a, b)[2],
                                                lambda a, b: WL.neumann_field(a, b)[3]))
        real = nd["kind"] != 3
        ex = WL.neumann_field(nd["x"], nd["y"])[0]
        errs.append(np.linalg.norm((phi - ex)[real]) / np.linalg.norm(ex[real]))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) >= rate - 0.4, (k, errs, rates)
