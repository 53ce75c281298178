"""The FP64 route of labfm_weights (two kernels per order: factor, then
weights and refinement, with each node's factors passed through a workspace)
against the single FP64 kernel that labfm_weights_noalloc runs.  Both follow
Sec. 3.1 (eqs. disc_form, lsys, w_abf) with the same equilibration, pivoting
and refinement, so every output must agree bit for bit:

* one to five operators: the two-kernel route always computes operator
  slots 1-3, on zero coefficients when a call asks for fewer, and nothing of
  those slots may reach the outputs;
* the three ABF families;
* a node set larger than the workspace's 262,144 node slots, so that the
  work lists are processed in two chunks."""
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

    import paper_1912_06441_amd as L

    assert torch.cuda.is_available()
    ctx = L.Context(0)
    yield dict(torch=torch, L=L, ctx=ctx)
    torch.cuda.synchronize()
    ctx.close()


def _compare(env, side, seed, k, family, rbf, ops, rs):
    torch, ctx = env["torch"], env["ctx"]
    x, y, s = WL.jittered_lattice(side, eps=0.3, seed=seed)
    dom = WL.unit_domain(False)
    order = WL.order_map(x, y, k, band=rs * s, k_boundary=4)
    R = np.full(x.size, rs * s)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    xt, yt, Rt, ot = d(x), d(y), d(R), d(order)
    rp, col = ctx.build_neighbours(xt, yt, Rt, ot, dom)
    kw = dict(ops=ops, abf=family, rbf=rbf, want32=True)
    two = ctx.weights(xt, yt, Rt, ot, rp, col, dom, **kw)
    one = ctx.weights(xt, yt, Rt, ot, rp, col, dom, noalloc=True, **kw)
    torch.cuda.synchronize()
    for a, b, name in zip(two, one, ("w64", "w32", "status", "resid", "iters")):
        assert torch.equal(a, b), name
    st = two[2].cpu().numpy()
    return x.size, np.bincount(st.astype(np.int64), minlength=7)


@pytest.mark.parametrize("family,rbf,ops,k", [
    ("HERMITE", "WENDLAND_C2", 1, 6),           # one operator: slots 2-3 on zero coefficients
    ("PAPER_D1", "QUADRATIC", 1 | 2, 4),        # two
    ("PAPER", "QUADRATIC", 1 | 2 | 4 | 8, 6),   # four: slot 4 by the run-time count
    ("HERMITE", "WENDLAND_C6", 1 | 2 | 4 | 8 | 16, 8),  # five
])
def test_two_kernels_equal_single_kernel(env, family, rbf, ops, k):
    L = env["L"]
    _say("split route: %s x %s, ops %d, order %d" % (family, rbf, ops, k))
    n, counts = _compare(env, 44, 40 + k, k, getattr(L, "ABF_" + family), getattr(L, "RBF_" + rbf), ops,
                         4.4 if k == 8 else 3.2)
    assert counts[0] > n // 2  # most nodes solved: the comparison covers the refinement


def test_two_chunks_of_the_workspace(env):
    L = env["L"]
    _say("split route: 560 x 560, order 4, two workspace chunks")
    n, counts = _compare(env, 560, 47, 4, L.ABF_HERMITE, L.RBF_WENDLAND_C2, 1 | 2 | 4, 2.85)
    assert n > 262144
    assert counts[0] == n
