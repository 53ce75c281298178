"""labfm_weights_noalloc through the C ABI against labfm_weights.

The entry point that allocates nothing runs the same kernels on work lists
held in the library's fixed per-GPU array; its outputs must equal those of
labfm_weights bit for bit.  Two calls in a row, the second on a smaller node
set (the array keeps the first call's contents, so anything that must start at
zero has to be cleared inside the call), for the FP64 and the mixed path; the
size limit and the unsupported warm-start precision are refused before any
launch."""
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


def _set(side, seed, k):
    x, y, s = WL.jittered_lattice(side, eps=0.3, seed=seed)
    dom = WL.unit_domain(False)
    order = WL.order_map(x, y, k, band=(4.4 if k == 8 else 2.85) * s, k_boundary=4)
    R = np.full(x.size, (4.4 if k == 8 else 2.85) * s)
    return x, y, R, order, dom


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_equals_weights(env, prec):
    torch, L, ctx = env["torch"], env["L"], env["ctx"]
    p = L.PREC_FP64 if prec == "fp64" else L.PREC_MIXED
    for side, seed, k in ((80, 31, 8), (40, 32, 6)):  # the second call is smaller
        _say("noalloc %s: %d x %d, order %d" % (prec, side, side, k))
        x, y, R, order, dom = _set(side, seed, k)
        d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        xt, yt, Rt, ot = d(x), d(y), d(R), d(order)
        rp, col = ctx.build_neighbours(xt, yt, Rt, ot, dom)
        ref = ctx.weights(xt, yt, Rt, ot, rp, col, dom, prec=p, want32=True)
        got = ctx.weights(xt, yt, Rt, ot, rp, col, dom, prec=p, want32=True, noalloc=True)
        torch.cuda.synchronize()
        for r, g, name in zip(ref, got, ("w64", "w32", "status", "resid", "iters")):
            assert torch.equal(r, g), name
        st = got[2].cpu().numpy()
        assert np.all(st == 0) and float(got[3].max()) <= 1e-10


def test_noalloc_refuses_before_launch(env):
    torch, L, ctx = env["torch"], env["L"], env["ctx"]
    n = L.NOALLOC_MAX_NODES + 1
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    order = torch.full((n,), 4, dtype=torch.int8, device="cuda")
    rp = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    col = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(L.LabfmError, match="LABFM_NOALLOC_MAX_NODES"):
        ctx.weights(x, x, x, order, rp, col, WL.unit_domain(False), noalloc=True)
    # the warm-start precision needs library scratch: refused by the C entry point itself
    import ctypes as C

    x, y, R, order, dom = _set(24, 33, 4)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    xt, yt, Rt, ot = d(x), d(y), d(R), d(order)
    rp, col = ctx.build_neighbours(xt, yt, Rt, ot, dom)
    w64, w32, st, res, it = ctx.weights(xt, yt, Rt, ot, rp, col, dom)
    o = L.WOpts(L.ABF_HERMITE, L.RBF_WENDLAND_C2, 1.0, 7, L.PREC_MLP, 1e-13, 1e-10, 5, None)
    dm = L.make_domain(dom)
    p = lambda t: C.c_void_p(t.data_ptr())
    rc = ctx.lib.labfm_weights_noalloc(ctx.h, p(xt), p(yt), xt.numel(), C.byref(dm), p(Rt), p(ot), p(rp), p(col),
                                       col.numel(), C.byref(o), p(w64), None, p(st), p(res), p(it), None)
    assert rc == -4  # LABFM_EUNSUPPORTED
    torch.cuda.synchronize()
