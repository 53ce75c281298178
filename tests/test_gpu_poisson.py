"""Global Poisson solve on the GPU (Sec. 5.2): Jacobi-BiCGStab with device-
resident scalars, against scipy's direct solution of the oracle's system and
against the exact solution.

* Parity: periodic (node 0 pinned) and Dirichlet-square systems built from the
  oracle's weights: the GPU solution within 1e-8 of the direct solve, the
  residual at the tolerance, Dirichlet rows at their data; two solves are bit
  for bit identical (fixed-grid reductions).
* The whole GPU path (neighbours, FP64 weights, solve): orders 2 / 4 / >= 5 for
  k = 2, 4, 6 on the periodic case, and parity with the oracle path at the
  smallest size.
* Edge cases: zero right-hand side, max_iters = 0, an empty system.
"""
import math
import sys

import numpy as np
import pytest

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


def _oracle_system(env, k, side, periodic):
    import test_oracle_poisson as TP

    return TP._system(env["O"], k, side, periodic)


@pytest.mark.parametrize("k,periodic", [(4, True), (3, False), (6, True)])
def test_poisson_parity(env, k, periodic):
    import scipy.sparse.linalg as spl

    from oracle import poisson as P

    S = _oracle_system(env, k, 30, periodic)
    A = P.laplacian_matrix(S["rp"], S["col"], S["w"], S["fixed"])
    xd = spl.spsolve(A.tocsc(), S["F"])
    _, it_o, _, _ = P.bicgstab(A, S["F"], x0=S["x0"], tol=1e-10)
    outs = []
    for rep in range(2):
        phi, it, res, ok = env["ctx"].poisson_solve(_dev(env, S["rp"]), _dev(env, S["col"]), _dev(env, S["w"]),
                                                    _dev(env, S["F"]), phi=_dev(env, S["x0"]),
                                                    fixed=_dev(env, S["fixed"]), tol=1e-10)
        outs.append(phi.cpu().numpy())
    x = outs[0]
    _say("  poisson k=%d periodic=%s: iters %d (oracle %d) rel resid %.2e  |x - direct| %.2e" %
         (k, periodic, it, it_o, res, np.abs(x - xd).max() / np.abs(xd).max()))
    assert ok and res <= 1e-10
    assert np.array_equal(outs[0], outs[1])
    assert np.abs(x - xd).max() <= 1e-8 * np.abs(xd).max()
    assert np.linalg.norm(S["F"] - A @ x) <= 1.01e-10 * np.linalg.norm(S["F"])
    fx = S["fixed"] == 1
    assert np.abs(x[fx] - S["F"][fx]).max() <= 1e-8 * np.abs(xd).max()
    assert abs(it - it_o) <= max(3, it_o // 3)


def _gpu_system(env, k, side):
    L = env["L"]
    cfg = WL.config("poisson")
    x, y, s = WL.jittered_lattice(side, eps=WL.paper_jitter(cfg["eps_paper"]), seed=cfg["seed"], periodic=True)
    dom = WL.unit_domain(True)
    n = x.size
    xt, yt = _dev(env, x), _dev(env, y)
    Rt = _dev(env, np.full(n, 2.0 * cfg["h_over_dr"][k] * s))
    ot = _dev(env, np.full(n, k, np.int8))
    rp, col = env["ctx"].build_neighbours(xt, yt, Rt, ot, dom, grow=True)
    w64, _, st, res, _ = env["ctx"].weights(xt, yt, Rt, ot, rp, col, dom, ops=L.OP_LAP, abf=cfg["abf"], rbf=cfg["rbf"])
    env["torch"].cuda.synchronize()
    assert np.all(st.cpu().numpy() == 0) and float(res.max()) <= 1e-10
    fixed = np.zeros(n, np.int8)
    fixed[0] = 1
    F, x0 = WL.poisson_system(x, y, fixed)
    return x, y, rp, col, w64[0].contiguous(), fixed, F, x0


@pytest.mark.parametrize("k,rate", [(2, 2.0), (4, 4.0), (6, 5.0)])
def test_periodic_poisson_orders_gpu(env, k, rate):
    cfg = WL.config("poisson")
    errs = []
    for side in cfg["sides"][1:]:
        x, y, rp, col, w, fixed, F, x0 = _gpu_system(env, k, side)
        # solved to 1e-12 so that the solver's error stays below the k = 6 discretisation error
        phi, it, res, ok = env["ctx"].poisson_solve(rp, col, w, _dev(env, F), phi=_dev(env, x0),
                                                    fixed=_dev(env, fixed), tol=1e-12)
        assert ok, (k, side, it, res)
        ex = WL.poisson_solution(x, y)
        g = phi.cpu().numpy()
        errs.append(np.linalg.norm(g - ex) / np.linalg.norm(ex))
        msg = "  poisson periodic k=%d side %d: iters %d resid %.1e L2 %.3e" % (k, side, it, res, errs[-1])
        if side == cfg["sides"][1]:
            S = _oracle_system(env, k, side, True)
            import scipy.sparse.linalg as spl

            from oracle import poisson as P

            xd = spl.spsolve(P.laplacian_matrix(S["rp"], S["col"], S["w"], S["fixed"]).tocsc(), S["F"])
            par = np.abs(g - xd).max() / np.abs(xd).max()
            msg += "  parity %.1e" % par
            assert par <= 1e-8
        _say(msg)
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    _say("  rates %s" % np.round(rates, 2))
    assert min(rates) >= rate - 0.35, (errs, rates)


def test_poisson_edge_cases(env):
    torch = env["torch"]
    S = _oracle_system(env, 2, 12, True)
    args = (_dev(env, S["rp"]), _dev(env, S["col"]), _dev(env, S["w"]))
    zero = torch.zeros(S["x"].size, dtype=torch.float64, device="cuda")
    phi, it, res, ok = env["ctx"].poisson_solve(*args, zero, fixed=_dev(env, S["fixed"]))
    assert ok and it == 0 and float(phi.abs().max()) == 0.0
    guess = _dev(env, S["x0"])
    phi, it, res, ok = env["ctx"].poisson_solve(*args, _dev(env, S["F"]), phi=guess.clone(), max_iters=0)
    assert it == 0 and not ok and torch.equal(phi, guess)
    e = torch.zeros(0, dtype=torch.float64, device="cuda")
    phi, it, res, ok = env["ctx"].poisson_solve(torch.zeros(1, dtype=torch.int64, device="cuda"),
                                                torch.zeros(0, dtype=torch.int32, device="cuda"), e, e)
    assert ok and it == 0
