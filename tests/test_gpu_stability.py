"""Stability and critical stencil sizes through the GPU path.

* Stability of the Laplacian operators built by the GPU path (Sec. 4.2,
Table noise_limits): on the 441-node periodic noisy lattices, with quadratic
RBF and the PAPER_D1 family, neighbours and FP64 Laplacian weights come from
the GPU; the eigenvalues of the global matrix A^L (dense, on the host) put
every case on the side of the printed limit the table gives, as the oracle's
weights do; the nodes with a usable operator are the oracle's (apart from
residuals within 3x of the 1e-10 gate) and the weights agree within 1e-10
per node (at most one node in a hundred above, on ill-conditioned stencils,
none above 1e-8).
* Critical stencil sizes (Sec. 3.2): 0.2 above each printed h/dr_crit every
node passes the gate, 0.25 below most have fewer neighbours than p; statuses
equal the oracle's node for node.
"""
import math
import sys

import numpy as np
import pytest

from paper_1912_06441_amd import workloads as WL
from test_oracle_heat import NOISE_CASES, _lap_dense, _table

pytestmark = pytest.mark.gpu


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


def _gpu_max_re(env, k, hdr, eps, seed):
    O, torch = env["O"], env["torch"]
    x, y, s = WL.jittered_lattice(21, eps=WL.paper_jitter(eps), seed=seed, periodic=True)
    dom = WL.unit_domain(True)
    n = x.size
    order = np.full(n, k, np.int8)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    Rt = d(np.full(n, 2.0 * hdr * s))
    rp, col = env["ctx"].build_neighbours(d(x), d(y), Rt, d(order), dom, grow=False)
    w, _, st, res, _ = env["ctx"].weights(d(x), d(y), Rt, d(order), rp, col, dom, ops=O.OP_LAP,
                                          abf=O.ABF_PAPER_D1, rbf=O.RBF_QUADRATIC)
    torch.cuda.synchronize()
    rp, col, w, st = rp.cpu().numpy(), col.cpu().numpy(), w[0].cpu().numpy(), st.cpu().numpy()
    res = res.cpu().numpy().astype(np.float64)
    rpo, colo, Ro = O.neighbours(x, y, dom, np.full(n, 2.0 * hdr * s), order, grow=False)
    wo, sto, reso, _ = O.weights(x, y, dom, Ro, order, rpo, colo, family=O.ABF_PAPER_D1, rbf=O.RBF_QUADRATIC,
                                 ops=O.OP_LAP)
    assert np.array_equal(rp, rpo) and np.array_equal(col, colo)
    # usable operators on the same nodes, except where a residual sits at the gate
    split = (st == O.ST_OK) != (sto == O.ST_OK)
    lo, hi = 1e-10 / 3, 3e-10  # both at most 3e-10, one within 3x of the gate
    near = (res <= hi) & (reso <= hi) & (((res > lo) & (res < hi)) | ((reso > lo) & (reso < hi)))
    assert np.all(near[split]), np.nonzero(split & ~near)
    both = np.nonzero((st == O.ST_OK) & (sto == O.ST_OK))[0]
    par = np.array([np.abs(w[rp[i]:rp[i + 1]] - wo[0][rp[i]:rp[i + 1]]).max() /
                    np.abs(wo[0][rp[i]:rp[i + 1]]).max() for i in both])
    # as on the headline set: ill-conditioned stencils (weights ~1e6 here) may
    # pass 1e-10 on a few nodes, none reaches 1e-8
    if par.size:
        assert par.max() <= 1e-8 and int((par > 1e-10).sum()) <= max(1, n // 100), (par.max(), (par > 1e-10).sum())
    if not np.all(st == O.ST_OK):
        return math.inf
    ev = np.linalg.eigvals(_lap_dense(rp, col, w))
    return ev.real.max() * (hdr * s) ** 2


@pytest.mark.parametrize("k,hdr,eps,stable", NOISE_CASES)
def test_noise_limits_through_gpu_weights(env, k, hdr, eps, stable):
    print("noise limit case k=%d h/dr=%.1f eps/dr=%.2f" % (k, hdr, eps), flush=True)
    sys.stdout.flush()
    tab = _table("noise_limits_table.txt")
    assert tab["%.1f" % hdr] is not None
    vals = [_gpu_max_re(env, k, hdr, eps, seed) for seed in (1, 2)]
    if stable:
        assert max(vals) < 1e-8, vals
    else:
        assert max(vals) > 1e-6, vals


@pytest.mark.parametrize("k,crit", [(2, 0.75), (4, 1.15), (6, 1.6), (8, 2.1)])
def test_critical_stencil_sizes_through_gpu(env, k, crit):
    """Sec. 3.2 critical h/dr: 0.2 above the printed value every node of the
    24 x 24 periodic noisy lattice (eps/dr = 0.5) gets weights at the gate
    from the GPU path, 0.25 below it most nodes have fewer neighbours than p;
    statuses equal the oracle's node for node, weights within 1e-10."""
    O, torch = env["O"], env["torch"]
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    for hdr, above in ((crit + 0.2, True), (crit - 0.25, False)):
        print("critical size k=%d h/dr=%.2f" % (k, hdr), flush=True)
        x, y, s = WL.jittered_lattice(24, eps=WL.paper_jitter(0.5), seed=5, periodic=True)
        dom = WL.unit_domain(True)
        n = x.size
        order = np.full(n, k, np.int8)
        Rt = d(np.full(n, 2.0 * hdr * s))
        rp, col = env["ctx"].build_neighbours(d(x), d(y), Rt, d(order), dom, grow=False)
        w, _, st, _, _ = env["ctx"].weights(d(x), d(y), Rt, d(order), rp, col, dom, ops=7,
                                            abf=O.ABF_PAPER_D1, rbf=O.RBF_QUADRATIC)
        torch.cuda.synchronize()
        rp, col, w, st = rp.cpu().numpy(), col.cpu().numpy(), w.cpu().numpy(), st.cpu().numpy()
        rpo, colo, Ro = O.neighbours(x, y, dom, np.full(n, 2.0 * hdr * s), order, grow=False)
        wo, sto, _, _ = O.weights(x, y, dom, Ro, order, rpo, colo, family=O.ABF_PAPER_D1, rbf=O.RBF_QUADRATIC, ops=7)
        assert np.array_equal(rp, rpo) and np.array_equal(col, colo) and np.array_equal(st, sto)
        if above:
            assert np.all(st == O.ST_OK)
        else:
            assert (st == O.ST_TOO_FEW).mean() >= 0.5
        for i in np.nonzero(st == O.ST_OK)[0]:
            a, b = rp[i], rp[i + 1]
            for dd in range(3):
                assert np.abs(w[dd, a:b] - wo[dd, a:b]).max() <= 1e-10 * np.abs(wo[dd, a:b]).max()
