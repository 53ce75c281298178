"""Three-dimensional LABFM on the GPU against the oracle.

* Neighbour lists bit-exact (periodic and bounded cubes, several radii).
* FP64 weights of orders 1..6 (p up to 83: two rows per lane at k = 6):
  status equal to the oracle's, moment residual <= 1e-10, per-node weight
  parity <= 1e-10 (max |dw| / max |w| in a row).  On bounded cubes, wall and
  corner stencils with N close to p can be ill-conditioned: a node above
  1e-10 must have cond_1(M) >= 1e8 (weights are defined to about cond 2^-53),
  an OK / NOT_CONVERGED split needs cond_1 >= 1e14, and both stay rare.
* Rows longer than LABFM_MAX_NEIGHBOURS3 (256) get TOO_MANY exactly where the
  oracle's do; rows up to the limit keep their parity.
* Through the whole GPU path (neighbours, weights, application): gradient
  errors fall ~h^k and the Laplacian ~h^(k-1) from 12^3 to 24^3.
* Degenerate requests: order 1 with a Laplacian, stencils with N < p.
* Calls with one to three operators (the unused operator slots of orders 1..4
  run on zero coefficients) keep every status and the weights within 1e-10.
"""
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


def _gpu_neigh(env, x, y, z, R, dom):
    xt, yt, zt = _dev(env, x), _dev(env, y), _dev(env, z)
    Rt = _dev(env, np.full(x.size, R))
    rp, col = env["ctx"].build_neighbours3(xt, yt, zt, Rt, dom)
    env["torch"].cuda.synchronize()
    return xt, yt, zt, Rt, rp, col


@pytest.mark.parametrize("side,periodic,Rs", [(12, True, 2.7), (10, False, 1.9), (9, True, 4.4)])
def test_neighbours3_bit_exact(env, side, periodic, Rs):
    x, y, z, s = WL.jittered_lattice3(side, eps=0.3, seed=side, periodic=periodic)
    dom = WL.unit_domain3(periodic)
    rp_o, col_o = env["O"].neighbours3(x, y, z, dom, Rs * s)
    _, _, _, _, rp, col = _gpu_neigh(env, x, y, z, Rs * s, dom)
    assert np.array_equal(rp.cpu().numpy(), rp_o)
    assert np.array_equal(col.cpu().numpy(), col_o)
    _say("  3-D neighbours side %d periodic %s: nnz %d" % (side, periodic, rp_o[-1]))


def _row_parity(rp, w, w_or):
    n = rp.size - 1
    seg = np.repeat(np.arange(n), np.diff(rp))
    worst = np.zeros(n)
    for d in range(w_or.shape[0]):
        num = np.zeros(n)
        den = np.zeros(n)
        np.maximum.at(num, seg, np.abs(w[d] - w_or[d]))
        np.maximum.at(den, seg, np.abs(w_or[d]))
        worst = np.maximum(worst, num / np.where(den > 0, den, 1.0))
    return worst


def _cond3(O, x, y, z, rp, col, i, R, k, sigma, dom):
    """1-norm condition number of node i's equilibrated moment matrix (rows,
    then columns scaled by their max-abs entry), from the oracle's basis."""
    h = 0.5 * R
    L = [dom["hi"][a] - dom["lo"][a] for a in range(3)]
    d = []
    for j in col[rp[i]:rp[i + 1]]:
        v = np.array([x[j] - x[i], y[j] - y[i], z[j] - z[i]])
        for a in range(3):
            if dom["periodic"][a]:
                v[a] -= L[a] * np.round(v[a] / L[a])
        d.append(v / h)
    X = np.array([O.monomials3(k, *v) for v in d])
    W = np.array([O.abfs3(k, *v, sigma=sigma) for v in d])
    M = X.T @ W
    M = M / np.abs(M).max(axis=1, keepdims=True)
    M = M / np.abs(M).max(axis=0, keepdims=True)
    return np.linalg.cond(M, 1)


@pytest.mark.parametrize("k,periodic,side", [(1, True, 11), (2, True, 11), (3, False, 11), (4, True, 11),
                                             (4, False, 11), (5, True, 11), (5, False, 12), (6, True, 11),
                                             (6, False, 14)])
def test_weights3_parity(env, k, periodic, side):
    O, L = env["O"], env["L"]
    cfg = WL.config("c3d")
    x, y, z, s = WL.jittered_lattice3(side, eps=cfg["eps"], seed=30 + k, periodic=periodic)
    dom = WL.unit_domain3(periodic)
    R = cfg["R_s"][k] * s
    ops = O.OP_DX | O.OP_DY | O.OP_DZ | (O.OP_LAP if k >= 2 else 0)
    rp_o, col_o = O.neighbours3(x, y, z, dom, R)
    w_o, st_o, res_o, _ = O.weights3(x, y, z, dom, R, k, rp_o, col_o, ops=ops, sigma=cfg["sigma"])
    xt, yt, zt, Rt, rp, col = _gpu_neigh(env, x, y, z, R, dom)
    w, st, res, it = env["ctx"].weights3(xt, yt, zt, Rt, k, rp, col, dom, ops=ops, sigma=cfg["sigma"])
    env["torch"].cuda.synchronize()
    st = st.cpu().numpy()
    res = res.cpu().numpy()
    # An OK / NOT_CONVERGED split is excused only on a numerically singular
    # system (cond_1 >= 1e14, so cond * 2^-53 >= 0.01 and neither refinement is
    # bound to converge): wall and corner stencils with N close to p.
    diff = np.nonzero(st != st_o)[0]
    excused = []
    for i in diff:
        c = _cond3(O, x, y, z, rp_o, col_o, i, R, k, cfg["sigma"], dom)
        _say("  node %d: status %d (oracle %d), residual %.3e (oracle %.3e), N %d, cond1 %.2e" %
             (i, st[i], st_o[i], res[i], res_o[i], rp_o[i + 1] - rp_o[i], c))
        assert {int(st[i]), int(st_o[i])} == {0, 1} and c >= 1e14
        excused.append(i)
    assert len(excused) <= max(2, st.size // 500)
    keep = np.ones(st.size, bool)
    keep[excused] = False
    ok = (st == 0) & keep
    assert ok.sum() > 0.5 * ok.size
    assert np.all(res[st == 0] <= 1e-10)
    par = _row_parity(rp_o, w.cpu().numpy(), w_o)
    _say("  3-D weights k=%d periodic %s: %d/%d OK, parity max %.2e median %.2e" %
         (k, periodic, ok.sum(), ok.size, par[ok].max(), np.median(par[ok])))
    # weights are defined to about cond(M) 2^-53: a node above 1e-10 must be
    # ill-conditioned (cond_1 >= 1e8), and such nodes stay rare
    loose = np.nonzero(ok & (par > 1e-10))[0]
    for i in loose:
        c = _cond3(O, x, y, z, rp_o, col_o, i, R, k, cfg["sigma"], dom)
        _say("  node %d: parity %.2e, N %d, cond1 %.2e" % (i, par[i], rp_o[i + 1] - rp_o[i], c))
        assert c >= 1e8 and par[i] <= 1e-6
    assert loose.size <= max(2, st.size // 500)
    failed = (st != 0) & (st != 1)
    assert np.all(w.cpu().numpy()[:, np.repeat(failed, np.diff(rp_o))] == 0.0)


@pytest.mark.parametrize("k,ops", [(4, "DX"), (3, "DZ|LAP"), (2, "DY"), (4, "DX|DY|DZ"), (1, "DZ")])
def test_weights3_fewer_operators(env, k, ops):
    """Calls with one to three operators: the kernels of orders 1..4 always
    compute three operator slots and run the unused ones on zero coefficients;
    nothing of those slots may reach the outputs.  Periodic lattice: every
    status OK as the oracle's, weights within 1e-10 of the oracle's."""
    O = env["O"]
    cfg = WL.config("c3d")
    mask = 0
    for name in ops.split("|"):
        mask |= getattr(O, "OP_" + name)
    x, y, z, s = WL.jittered_lattice3(10, eps=cfg["eps"], seed=60 + k, periodic=True)
    dom = WL.unit_domain3(True)
    R = cfg["R_s"][k] * s
    rp_o, col_o = O.neighbours3(x, y, z, dom, R)
    w_o, st_o, res_o, _ = O.weights3(x, y, z, dom, R, k, rp_o, col_o, ops=mask, sigma=cfg["sigma"])
    xt, yt, zt, Rt, rp, col = _gpu_neigh(env, x, y, z, R, dom)
    w, st, res, it = env["ctx"].weights3(xt, yt, zt, Rt, k, rp, col, dom, ops=mask, sigma=cfg["sigma"])
    env["torch"].cuda.synchronize()
    st = st.cpu().numpy()
    assert w.shape[0] == w_o.shape[0]
    assert np.array_equal(st, st_o) and np.all(st == 0)
    assert float(res.max()) <= 1e-10
    par = _row_parity(rp_o, w.cpu().numpy(), w_o)
    _say("  3-D k=%d ops %s: parity max %.2e" % (k, ops, par.max()))
    assert par.max() <= 1e-10


@pytest.mark.parametrize("k,rg,rl", [(2, 1.7, 0.9), (3, 2.6, 1.6), (4, 3.5, 2.4), (5, 4.5, 3.5), (6, 5.5, 4.5)])
def test_weights3_convergence_gpu(env, k, rg, rl):
    cfg = WL.config("c3d")
    errs = []
    for side in (12, 24):
        x, y, z, s = WL.jittered_lattice3(side, eps=cfg["eps"], seed=cfg["seed"], periodic=True)
        dom = WL.unit_domain3(True)
        xt, yt, zt, Rt, rp, col = _gpu_neigh(env, x, y, z, cfg["R_s"][k] * s, dom)
        w, st, res, _ = env["ctx"].weights3(xt, yt, zt, Rt, k, rp, col, dom, sigma=cfg["sigma"])
        f, fx, fy, fz, lap = WL.trig_field3(x, y, z)
        out = env["ctx"].apply_operator(rp, col, w, _dev(env, f)).cpu().numpy()
        assert np.all(st.cpu().numpy() == 0)
        errs.append([np.linalg.norm(out[d] - ref) / np.linalg.norm(ref) for d, ref in enumerate((fx, fy, lap, fz))])
    r = np.log2(np.array(errs[0]) / np.array(errs[1]))
    _say("  3-D k=%d errors %s rates %s" % (k, np.array(errs[1]).round(8), r.round(2)))
    assert min(r[0], r[1], r[3]) >= rg and r[2] >= rl, r


def test_weights3_degenerate_requests(env):
    O = env["O"]
    x, y, z, s = WL.jittered_lattice3(6, eps=0.3, seed=3, periodic=True)
    dom = WL.unit_domain3(True)
    xt, yt, zt, Rt, rp, col = _gpu_neigh(env, x, y, z, 1.5 * s, dom)
    w, st, _, _ = env["ctx"].weights3(xt, yt, zt, Rt, 1, rp, col, dom)  # order 1 cannot hold a Laplacian
    env["torch"].cuda.synchronize()
    assert np.all(st.cpu().numpy() == O.ST_ORDER_TOO_LOW) and float(w.abs().max()) == 0.0
    w, st, _, _ = env["ctx"].weights3(xt, yt, zt, Rt, 4, rp, col, dom)  # about 14 neighbours < p = 34
    env["torch"].cuda.synchronize()
    assert np.all(st.cpu().numpy() == O.ST_TOO_FEW) and float(w.abs().max()) == 0.0
    w, st, _, _ = env["ctx"].weights3(xt, yt, zt, Rt, 6, rp, col, dom)  # p = 83
    env["torch"].cuda.synchronize()
    assert np.all(st.cpu().numpy() == O.ST_TOO_FEW) and float(w.abs().max()) == 0.0


@pytest.mark.parametrize("k", [5, 6])
def test_weights3_long_rows(env, k):
    """Every seventh node with R = 4.3 s (about 330 neighbours, above the
    256-entry limit), the rest at the order's radius: TOO_MANY, zero weights
    and an infinite residual exactly where the oracle's rows are too long."""
    O = env["O"]
    cfg = WL.config("c3d")
    x, y, z, s = WL.jittered_lattice3(10, eps=cfg["eps"], seed=40 + k, periodic=True)
    dom = WL.unit_domain3(True)
    R = np.full(x.size, cfg["R_s"][k] * s)
    R[::7] = 4.3 * s
    rp_o, col_o = O.neighbours3(x, y, z, dom, R)
    N = np.diff(rp_o)
    assert (N > O.NMAX3).sum() > 0 and (N > O.NMAX3).sum() == R[::7].size
    w_o, st_o, res_o, _ = O.weights3(x, y, z, dom, R, k, rp_o, col_o, sigma=cfg["sigma"])
    xt, yt, zt = _dev(env, x), _dev(env, y), _dev(env, z)
    Rt = _dev(env, R)
    rp, col = env["ctx"].build_neighbours3(xt, yt, zt, Rt, dom)
    w, st, res, it = env["ctx"].weights3(xt, yt, zt, Rt, k, rp, col, dom, sigma=cfg["sigma"])
    env["torch"].cuda.synchronize()
    st, res, w = st.cpu().numpy(), res.cpu().numpy(), w.cpu().numpy()
    assert np.array_equal(rp.cpu().numpy(), rp_o) and np.array_equal(st, st_o)
    long_ = N > O.NMAX3
    assert np.all(st[long_] == O.ST_TOO_MANY) and np.all(np.isinf(res[long_]))
    assert np.all(w[:, np.repeat(long_, N)] == 0.0)
    ok = st == 0
    assert ok.sum() == (~long_).sum() and res[ok].max() <= 1e-10
    par = _row_parity(rp_o, w, w_o)
    _say("  3-D long rows k=%d: %d rows > %d, parity of the rest %.2e" % (k, long_.sum(), O.NMAX3, par[ok].max()))
    assert par[ok].max() <= 1e-10
