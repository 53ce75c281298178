"""Eigen-spectra of the convective operator A^x (Sec. 4.2, Fig. eigens_convect)
through the GPU path: GPU neighbour sets and GPU FP64 d/dx weights (ABFs
keeping the dW0/dr term, conic / quadratic / Wendland C6 / Gaussian RBFs) on the
441-node periodic sets of the oracle's pin, h/dr = 2, k = 2, 4, 6; the global
matrix and its eigenvalues are formed on the host.  The weights match the
oracle's per node, and the spectra show the trends the oracle pins
(tests/test_oracle_convective.py): on the ideal lattice conic off the imaginary
axis, quadratic and Wendland on it to rounding; with noise eps/dr = 0.5 real
parts for every ABF, quadratic < conic < Gaussian at k = 4, 6 with the Gaussian
worst, the paper's full order at k = 6, and lower k closer to the axis."""
import sys

import numpy as np
import pytest

from paper_1912_06441_amd import workloads as WL
from test_oracle_convective import RBFS, _rbf, global_matrix

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


def _gpu_max_real(env, seed, eps, k, rbf):
    torch, O, ctx = env["torch"], env["O"], env["ctx"]
    x, y, s = WL.jittered_lattice(21, eps=eps, seed=seed, periodic=True)
    dom = WL.unit_domain(True)
    n = x.size
    order = np.full(n, k, np.int8)
    R = np.full(n, 4.0 * s)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    Rt = d(R)
    rp, col = ctx.build_neighbours(d(x), d(y), Rt, d(order), dom, grow=False)
    w, _, st, res, _ = ctx.weights(d(x), d(y), Rt, d(order), rp, col, dom, ops=O.OP_DX, abf=O.ABF_PAPER_D1,
                                   rbf=_rbf(O, rbf))
    torch.cuda.synchronize()
    rp, col, w, st = rp.cpu().numpy(), col.cpu().numpy(), w[0].cpu().numpy(), st.cpu().numpy()
    assert np.all(st == O.ST_OK) and float(res.max()) <= 1e-10
    rpo, colo, Ro = O.neighbours(x, y, dom, R, order, grow=False)
    assert np.array_equal(rp, rpo) and np.array_equal(col, colo)
    wo, sto, _, _ = O.weights(x, y, dom, Ro, order, rpo, colo, family=O.ABF_PAPER_D1, rbf=_rbf(O, rbf), ops=O.OP_DX)
    par = max(np.abs(w[rp[i]:rp[i + 1]] - wo[0][rp[i]:rp[i + 1]]).max() / np.abs(wo[0][rp[i]:rp[i + 1]]).max()
              for i in range(n))
    assert par <= 1e-10, (seed, eps, k, rbf, par)
    ev = np.linalg.eigvals(global_matrix(rp, col, w)) * s
    return float(np.abs(ev.real).max()), float(np.abs(ev.imag).max())


def test_convective_spectra_through_gpu_weights(env):
    sp = {}
    for eps in (0.0, 0.25):
        for k in (2, 4, 6):
            for r in RBFS:
                sp[(eps, k, r)] = _gpu_max_real(env, 3, eps, k, r)
            _say("  eps %.2f k %d: %s" % (eps, k, "  ".join("%s %.2e" % (r, sp[(eps, k, r)][0]) for r in RBFS)))
    for k in (2, 4, 6):
        re_c = sp[(0.0, k, "cone")][0]
        assert re_c >= 1e-2
        for r in ("quad", "wend"):
            re, im = sp[(0.0, k, r)]
            assert re <= 1e-12 * im and re_c >= 1e10 * re
        for r in RBFS:
            assert sp[(0.25, k, r)][0] >= 1e-2
    for k in (4, 6):
        re = {r: sp[(0.25, k, r)][0] for r in RBFS}
        assert re["quad"] < re["cone"] < re["gauss"] and re["gauss"] == max(re.values())
    re6 = {r: sp[(0.25, 6, r)][0] for r in RBFS}
    assert re6["quad"] < re6["cone"] < re6["wend"] < re6["gauss"]
    for r in ("cone", "quad", "gauss"):
        re = [sp[(0.25, k, r)][0] for k in (2, 4, 6)]
        assert re[0] < re[1] < re[2]
