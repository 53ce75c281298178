"""Neumann ghost rows on the GPU (Sec. 5.2, eq. neu): labfm_neumann_rows and
the solve about each row's centre, against the oracle's enlarged system.

* Rows: from the oracle's d/dx, d/dy and Laplacian weights, the GPU rows
  (column lists and centres bit for bit, weights within the roundings of
  n_x w^x + n_y w^y, with or without a fused multiply-add) assemble to the oracle's matrix; also with random unit
  normals.
* Solve: the GPU solution of the oracle-weight system within 1e-8 of scipy's
  direct solve, the residual at the tolerance.
* The whole GPU path (neighbours, FP64 d/dx, d/dy, Laplacian weights, ghost
  rows, solve): degree-k polynomials reproduced at every node for k = 2, 4;
  the smooth field converges at about k.
* Edge cases: no ghosts (rows and centres equal the Laplacian rows and the
  solve equals the plain one bit for bit), an empty node set, an out-of-range
  parent counting as none.
"""
import math
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from paper_1912_06441_amd import workloads as WL

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch

    import oracle
    import paper_1912_06441_amd as L

    assert torch.cuda.is_available()
    ctx = L.Context(0)
    yield dict(torch=torch, O=oracle, L=L, ctx=ctx)
    torch.cuda.synchronize()
    ctx.close()


def _dev(env, a):
    return env["torch"].from_numpy(np.ascontiguousarray(a)).cuda()


def _assemble(orp, ocol, ow, ocen, fixed):
    """The matrix the documented row layout stands for: row i is
    sum_q w_q (x_col[q] - x_center[i]); identity on fixed rows."""
    n = orp.size - 1
    rows = np.repeat(np.arange(n), np.diff(orp))
    s = np.zeros(n)
    np.add.at(s, rows, ow)
    keep = fixed[rows] == 0
    free = np.nonzero(fixed == 0)[0]
    fx = np.nonzero(fixed)[0]
    r = np.concatenate([rows[keep], free, fx])
    c = np.concatenate([ocol[keep], ocen[free], fx])
    v = np.concatenate([ow[keep], -s[free], np.ones(fx.size)])
    return sp.csr_matrix((v, (r, c)), shape=(n, n))


def _oracle_case(env, k, side, seed=13):
    import test_oracle_neumann as TN

    nd, rp, col, R, w = TN.neumann_case(env["O"], k, side, seed=seed)
    return nd, rp, col, w


def _gpu_rows(env, rp, col, w, nd, nx=None, ny=None):
    ctx = env["ctx"]
    nx = nd["nx"] if nx is None else nx
    ny = nd["ny"] if ny is None else ny
    orp, ocol, ow, ocen = ctx.neumann_rows(_dev(env, rp), _dev(env, col), _dev(env, w[0]), _dev(env, w[1]),
                                           _dev(env, w[2]), _dev(env, nd["parent"]), _dev(env, nx), _dev(env, ny))
    env["torch"].cuda.synchronize()
    return orp.cpu().numpy(), ocol.cpu().numpy(), ow.cpu().numpy(), ocen.cpu().numpy()


@pytest.mark.parametrize("k,side,random_normals", [(2, 16, False), (4, 20, False), (4, 20, True), (6, 24, True)])
def test_rows_parity(env, k, side, random_normals):
    from oracle import poisson as P

    nd, rp, col, w = _oracle_case(env, k, side)
    n = nd["x"].size
    nx, ny = nd["nx"].copy(), nd["ny"].copy()
    if random_normals:
        g = nd["parent"] >= 0
        th = np.random.default_rng(k).uniform(0.0, 2.0 * math.pi, int(g.sum()))
        nx[g], ny[g] = np.cos(th), np.sin(th)
    orp, ocol, ow, ocen = _gpu_rows(env, rp, col, w, nd, nx, ny)
    src = np.where(nd["parent"] >= 0, nd["parent"], np.arange(n))
    want_len = rp[src + 1] - rp[src]
    assert np.array_equal(np.diff(orp), want_len) and orp[0] == 0
    assert np.array_equal(ocen, src.astype(np.int32))
    for i in range(n):
        s, e = rp[src[i]], rp[src[i] + 1]
        assert np.array_equal(ocol[orp[i]:orp[i + 1]], col[s:e])
        if src[i] == i:
            assert np.array_equal(ow[orp[i]:orp[i + 1]], w[2][s:e])
        else:
            a, b = nx[i] * w[0][s:e], ny[i] * w[1][s:e]
            assert np.all(np.abs(ow[orp[i]:orp[i + 1]] - (a + b)) <= 4.5e-16 * (np.abs(a) + np.abs(b)))
    fixed = (nd["kind"] == 1).astype(np.int8)
    A_o = P.neumann_matrix(rp, col, w[0], w[1], w[2], nd["parent"], nx, ny, fixed)
    A_g = _assemble(orp, ocol, ow, ocen, fixed)
    d = abs(A_o - A_g)
    assert d.max() <= 1e-13 * abs(A_o).max()
    _say("  neumann rows k=%d side %d random normals %s: n %d nnz %d  max |A_gpu - A_oracle| %.1e" %
         (k, side, random_normals, n, ocol.size, d.max()))


@pytest.mark.parametrize("k", [2, 4])
def test_solve_parity(env, k):
    import scipy.sparse.linalg as spl

    from oracle import poisson as P

    nd, rp, col, w = _oracle_case(env, k, 24)
    fields = (lambda a, b: WL.neumann_field(a, b)[0], lambda a, b: WL.neumann_field(a, b)[1],
              lambda a, b: WL.neumann_field(a, b)[2], lambda a, b: WL.neumann_field(a, b)[3])
    F, x0, fixed = WL.neumann_system(nd, *fields)
    A = P.neumann_matrix(rp, col, w[0], w[1], w[2], nd["parent"], nd["nx"], nd["ny"], fixed)
    xd = spl.spsolve(A.tocsc(), F)
    ctx = env["ctx"]
    orp, ocol, ow, ocen = ctx.neumann_rows(_dev(env, rp), _dev(env, col), _dev(env, w[0]), _dev(env, w[1]),
                                           _dev(env, w[2]), _dev(env, nd["parent"]), _dev(env, nd["nx"]),
                                           _dev(env, nd["ny"]))
    phi, it, res, ok = ctx.poisson_solve(orp, ocol, ow, _dev(env, F), phi=_dev(env, x0), fixed=_dev(env, fixed),
                                         tol=1e-10, center=ocen)
    x = phi.cpu().numpy()
    _, it_o, _, _ = P.bicgstab(A, F, x0=x0, tol=1e-10)
    _say("  neumann solve k=%d: iters %d (oracle %d) resid %.1e |x - direct| %.1e" %
         (k, it, it_o, res, np.abs(x - xd).max() / np.abs(xd).max()))
    assert ok and res <= 1e-10
    assert np.linalg.norm(F - A @ x) <= 1.01e-10 * np.linalg.norm(F)
    assert np.abs(x - xd).max() <= 1e-8 * np.abs(xd).max()


def _gpu_path(env, k, side, fields, tol):
    L, ctx, torch = env["L"], env["ctx"], env["torch"]
    cfg = WL.config("poisson")
    nd = WL.neumann_square_nodes(side, eps_over_dr=cfg["eps_paper"], seed=13)
    x, y, s = nd["x"], nd["y"], nd["s"]
    n = x.size
    xt, yt = _dev(env, x), _dev(env, y)
    Rt = _dev(env, np.full(n, 2.0 * cfg["h_over_dr"][k] * s))
    ot = _dev(env, np.full(n, k, np.int8))
    rp, col = ctx.build_neighbours(xt, yt, Rt, ot, nd["domain"], grow=True)
    w64, _, st, res, _ = ctx.weights(xt, yt, Rt, ot, rp, col, nd["domain"], ops=L.OP_DX | L.OP_DY | L.OP_LAP,
                                     abf=cfg["abf"], rbf=cfg["rbf"])
    torch.cuda.synchronize()
    used = (nd["kind"] == 0) | (nd["kind"] == 2)
    stn = st.cpu().numpy()
    assert np.all(stn[used] == 0) and float(res.cpu().numpy()[used].max()) <= 1e-10
    orp, ocol, ow, ocen = ctx.neumann_rows(rp, col, w64[0].contiguous(), w64[1].contiguous(), w64[2].contiguous(),
                                           _dev(env, nd["parent"]), _dev(env, nd["nx"]), _dev(env, nd["ny"]))
    F, x0, fixed = WL.neumann_system(nd, *fields)
    phi, it, rr, ok = ctx.poisson_solve(orp, ocol, ow, _dev(env, F), phi=_dev(env, x0), fixed=_dev(env, fixed),
                                        tol=tol, center=ocen)
    assert ok, (k, side, it, rr)
    return nd, phi.cpu().numpy(), it


@pytest.mark.parametrize("k", [2, 4])
def test_polynomial_reproduced_gpu(env, k):
    fields = WL.neumann_poly(k)
    nd, phi, it = _gpu_path(env, k, 40, fields, 1e-12)
    ex = fields[0](nd["x"], nd["y"])
    err = np.abs(phi - ex).max() / np.abs(ex).max()
    _say("  neumann polynomial k=%d: iters %d max rel err %.1e" % (k, it, err))
    assert err <= 1e-8


@pytest.mark.parametrize("k,rate", [(2, 2.0), (4, 4.0)])
def test_neumann_convergence_gpu(env, k, rate):
    fields = (lambda a, b: WL.neumann_field(a, b)[0], lambda a, b: WL.neumann_field(a, b)[1],
              lambda a, b: WL.neumann_field(a, b)[2], lambda a, b: WL.neumann_field(a, b)[3])
    errs = []
    for side in (20, 40, 80):
        nd, phi, it = _gpu_path(env, k, side, fields, 1e-12)
        real = nd["kind"] != 3
        ex = WL.neumann_field(nd["x"], nd["y"])[0]
        errs.append(np.linalg.norm((phi - ex)[real]) / np.linalg.norm(ex[real]))
        _say("  neumann k=%d side %d: iters %d L2 %.3e" % (k, side, it, errs[-1]))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    _say("  rates %s" % np.round(rates, 2))
    assert min(rates) >= rate - 0.4, (errs, rates)


def test_neumann_edge_cases(env):
    torch, ctx = env["torch"], env["ctx"]
    nd, rp, col, w = _oracle_case(env, 2, 12)
    n = nd["x"].size
    none = np.full(n, -1, np.int32)
    args = [_dev(env, rp), _dev(env, col), _dev(env, w[0]), _dev(env, w[1]), _dev(env, w[2])]
    orp, ocol, ow, ocen = ctx.neumann_rows(*args, _dev(env, none), _dev(env, nd["nx"]), _dev(env, nd["ny"]))
    assert np.array_equal(orp.cpu().numpy(), rp) and np.array_equal(ocol.cpu().numpy(), col)
    assert np.array_equal(ow.cpu().numpy(), w[2]) and np.array_equal(ocen.cpu().numpy(), np.arange(n))
    # a parent outside [0, n) counts as none
    bad = nd["parent"].copy()
    g = np.nonzero(bad >= 0)[0]
    bad[g[0]], bad[g[1]] = n, -7
    orp2, _, ow2, ocen2 = ctx.neumann_rows(*args, _dev(env, bad), _dev(env, nd["nx"]), _dev(env, nd["ny"]))
    assert ocen2.cpu().numpy()[g[0]] == g[0] and ocen2.cpu().numpy()[g[1]] == g[1]
    # centre i everywhere: the same solve as without centres, bit for bit
    F = np.random.default_rng(5).standard_normal(n)
    fixed = (nd["kind"] == 1).astype(np.int8)
    a = ctx.poisson_solve(orp, ocol, ow, _dev(env, F), fixed=_dev(env, fixed), tol=1e-10, max_iters=40)
    b = ctx.poisson_solve(orp, ocol, ow, _dev(env, F), fixed=_dev(env, fixed), tol=1e-10, max_iters=40,
                          center=ocen)
    assert a[1] == b[1] and torch.equal(a[0], b[0])
    # empty node set
    z64 = torch.zeros(1, dtype=torch.int64, device="cuda")
    e32 = torch.zeros(0, dtype=torch.int32, device="cuda")
    e64 = torch.zeros(0, dtype=torch.float64, device="cuda")
    orp, ocol, ow, ocen = ctx.neumann_rows(z64, e32, e64, e64, e64, e32, e64, e64)
    assert orp.cpu().tolist() == [0] and ocol.numel() == 0 and ocen.numel() == 0
