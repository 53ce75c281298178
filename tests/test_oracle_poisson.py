"""Pins of the oracle's global Poisson solve (Sec. 5.2).

* The global matrix reproduces the local operators row by row and has
  identity rows at Dirichlet nodes (eq. poisson_system and the Dirichlet row
  rule).
* Jacobi-BiCGStab lands on scipy's direct sparse solution of the same system.
* Periodic case (Fig. poisson_periodic_conv): orders 2 for k = 2, 3, 4 for
  k = 4, 5 and at least 5 for k = 6; Dirichlet square: orders near k.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spl

from oracle import poisson as P
from paper_1912_06441_amd import workloads as WL


def _system(O, k, side, periodic, seed=None):
    cfg = WL.config("poisson")
    seed = cfg["seed"] if seed is None else seed
    if periodic:
        x, y, s = WL.jittered_lattice(side, eps=WL.paper_jitter(cfg["eps_paper"]), seed=seed, periodic=True)
        fixed = np.zeros(x.size, np.int8)
        fixed[0] = 1
    else:
        x, y, s = WL.wall_conforming_lattice(side + 1, eps=WL.paper_jitter(cfg["eps_paper"]), seed=seed)
        fixed = ((x == 0) | (x == 1) | (y == 0) | (y == 1)).astype(np.int8)
    dom = WL.unit_domain(periodic)
    order = np.full(x.size, k, np.int8)
    rp, col, R = O.neighbours(x, y, dom, 2.0 * cfg["h_over_dr"][k] * s, order, grow=True)
    w, st, _, _ = O.weights(x, y, dom, R, order, rp, col, family=cfg["abf"], rbf=cfg["rbf"], ops=O.OP_LAP)
    assert np.all(st[fixed == 0] == O.ST_OK)
    F, x0 = WL.poisson_system(x, y, fixed)
    return dict(x=x, y=y, rp=rp, col=col, w=w[0], fixed=fixed, F=F, x0=x0)


def test_global_matrix_rows(O):
    S = _system(O, 4, 24, False)
    A = P.laplacian_matrix(S["rp"], S["col"], S["w"], S["fixed"])
    u = np.random.default_rng(1).standard_normal(S["x"].size)
    Au = A @ u
    loc = O.apply(S["rp"], S["col"], S["w"], u)
    fx = S["fixed"] == 1
    assert np.allclose(Au[~fx], loc[~fx], rtol=0, atol=1e-12 * np.abs(loc).max())
    assert np.array_equal(Au[fx], u[fx])


@pytest.mark.parametrize("k,periodic", [(4, True), (3, False), (6, True)])
def test_bicgstab_matches_direct_solve(O, k, periodic):
    S = _system(O, k, 30, periodic)
    A = P.laplacian_matrix(S["rp"], S["col"], S["w"], S["fixed"])
    x, it, res, ok = P.bicgstab(A, S["F"], x0=S["x0"], tol=1e-10)
    xd = spl.spsolve(A.tocsc(), S["F"])
    assert ok and res <= 1e-10 and it > 0
    assert np.abs(x - xd).max() <= 1e-8 * np.abs(xd).max()
    assert np.linalg.norm(S["F"] - A @ x) <= 1e-10 * np.linalg.norm(S["F"]) * (1 + 1e-6)


@pytest.mark.parametrize("k,rate,periodic", [(2, 2.0, True), (3, 2.0, True), (4, 4.0, True), (5, 4.0, True),
                                             (6, 5.0, True), (2, 2.0, False), (3, 2.0, False), (4, 4.0, False)])
def test_poisson_orders(O, k, rate, periodic):
    errs = []
    for side in (20, 40, 80):
        S = _system(O, k, side, periodic)
        A = P.laplacian_matrix(S["rp"], S["col"], S["w"], S["fixed"])
        x, it, res, ok = P.bicgstab(A, S["F"], x0=S["x0"], tol=1e-10)
        assert ok
        ex = WL.poisson_solution(S["x"], S["y"])
        errs.append(np.linalg.norm(x - ex) / np.linalg.norm(ex))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) >= rate - 0.35, (k, periodic, errs, rates)
