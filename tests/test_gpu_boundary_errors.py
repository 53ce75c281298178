"""Argument checks of the C-ABI entry points added with Neumann rows, 3-D
orders 5-6, the warm start without a factorisation and its training data:
each bad call returns its documented code before any launch, names itself in
labfm_last_error, and leaves the context usable (a good call right after
succeeds)."""
import ctypes as C

import numpy as np
import pytest

from paper_1912_06441_amd import workloads as WL

pytestmark = pytest.mark.gpu

EINVAL, EUNSUPPORTED = -1, -4


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1912_06441_amd as L

    assert torch.cuda.is_available()
    ctx = L.Context(0)
    yield dict(torch=torch, L=L, ctx=ctx)
    torch.cuda.synchronize()
    ctx.close()


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _last(env):
    return env["ctx"].lib.labfm_last_error().decode()


def _small_set(env, k=4, side=12):
    torch = env["torch"]
    x, y, s = WL.jittered_lattice(side, eps=0.2, seed=3, periodic=True)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    xt, yt = d(x), d(y)
    Rt = d(np.full(x.size, 2.85 * s))
    ot = d(np.full(x.size, k, np.int8))
    dom = WL.unit_domain(True)
    rp, col = env["ctx"].build_neighbours(xt, yt, Rt, ot, dom)
    return xt, yt, Rt, ot, rp, col, dom


def test_neumann_rows_refusals(env):
    torch, lib, h = env["torch"], env["ctx"].lib, env["ctx"].h
    xt, yt, Rt, ot, rp, col, dom = _small_set(env)
    n, nnz = xt.numel(), col.numel()
    w = torch.zeros(nnz, dtype=torch.float64, device="cuda")
    parent = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    orp = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    args = [h, _p(rp), _p(col), n, nnz, _p(w), _p(w), _p(w), _p(parent), _p(xt), _p(yt), _p(orp)]
    # count pass without nnz_host
    assert lib.labfm_neumann_rows(*args, None, None, None, None, None) == EINVAL
    assert "labfm_neumann_rows" in _last(env)
    # fill pass without the weight or centre outputs
    ocol = torch.empty(nnz, dtype=torch.int32, device="cuda")
    assert lib.labfm_neumann_rows(*args, _p(ocol), None, None, None, None) == EINVAL
    # negative size, NULL context
    bad = list(args)
    bad[3] = -1
    nh = C.c_int64(0)
    assert lib.labfm_neumann_rows(*bad, None, None, None, C.byref(nh), None) == EINVAL
    bad = list(args)
    bad[0] = None
    assert lib.labfm_neumann_rows(*bad, None, None, None, C.byref(nh), None) == EINVAL
    # the context still works
    out = env["ctx"].neumann_rows(rp, col, w, w, w, parent, xt, yt)
    torch.cuda.synchronize()
    assert torch.equal(out[0], rp) and torch.equal(out[1], col)


def test_moment_systems_refusals(env):
    torch, L, lib, h = env["torch"], env["L"], env["ctx"].lib, env["ctx"].h
    xt, yt, Rt, ot, rp, col, dom = _small_set(env)
    n, nnz = xt.numel(), col.numel()
    M = torch.empty((n, 14, 14), dtype=torch.float32, device="cuda")
    psi = torch.empty((n, 3 * 14), dtype=torch.float32, device="cuda")
    st = torch.empty(n, dtype=torch.int8, device="cuda")
    dm = L.make_domain(dom)
    good = L.WOpts(L.ABF_HERMITE, L.RBF_WENDLAND_C2, 1.0, 7, L.PREC_FP64, 0.0, 0.0, 0, None)

    def call(k, o, Mp=M):
        return lib.labfm_moment_systems(h, _p(xt), _p(yt), n, C.byref(dm), _p(Rt), k, _p(rp), _p(col), nnz,
                                        C.byref(o), _p(Mp), _p(psi), _p(st), None)

    assert call(0, good) == EINVAL and call(9, good) == EINVAL
    assert "labfm_moment_systems" in _last(env)
    assert call(4, L.WOpts(L.ABF_HERMITE, L.RBF_WENDLAND_C2, 1.0, 0, L.PREC_FP64, 0.0, 0.0, 0, None)) == EINVAL
    assert call(4, L.WOpts(L.ABF_HERMITE, 7, 1.0, 7, L.PREC_FP64, 0.0, 0.0, 0, None)) == EINVAL
    assert call(4, L.WOpts(L.ABF_HERMITE, L.RBF_WENDLAND_C2, -1.0, 7, L.PREC_FP64, 0.0, 0.0, 0, None)) == EINVAL
    assert call(4, good, Mp=None) == EINVAL
    assert call(4, good) == 0
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == 0)


def test_weights3_order_range_and_warm_start_refusals(env):
    torch, L, lib, h = env["torch"], env["L"], env["ctx"].lib, env["ctx"].h
    x, y, z, s = WL.jittered_lattice3(10, eps=0.3, seed=3, periodic=True)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    xt, yt, zt = d(x), d(y), d(z)
    Rt = d(np.full(x.size, 3.4 * s))
    dom3 = WL.unit_domain3(True)
    rp, col = env["ctx"].build_neighbours3(xt, yt, zt, Rt, dom3)
    with pytest.raises(L.LabfmError, match="k must be 1..6"):
        env["ctx"].weights3(xt, yt, zt, Rt, 7, rp, col, dom3)
    with pytest.raises(L.LabfmError, match="k must be 1..6"):
        env["ctx"].weights3(xt, yt, zt, Rt, 0, rp, col, dom3)
    w, st, res, it = env["ctx"].weights3(xt, yt, zt, Rt, 6, rp, col, dom3)  # p = 83: still served
    torch.cuda.synchronize()
    assert set(np.unique(st.cpu().numpy())) <= {0, 1}
    # the warm-start routes: refused without a network, and by the batched and allocation-free calls
    xt, yt, Rt, ot, rp, col, dom = _small_set(env)
    with pytest.raises(L.LabfmError, match="needs a network"):
        env["ctx"].weights(xt, yt, Rt, ot, rp, col, dom, prec=L.PREC_MLP_NOLU)
    w64, w32, st, res, it = env["ctx"].weights(xt, yt, Rt, ot, rp, col, dom)
    o = L.WOpts(L.ABF_HERMITE, L.RBF_WENDLAND_C2, 1.0, 7, L.PREC_MLP_NOLU, 1e-13, 1e-10, 5, None)
    dm = L.make_domain(dom)
    rc = lib.labfm_weights_noalloc(h, _p(xt), _p(yt), xt.numel(), C.byref(dm), _p(Rt), _p(ot), _p(rp), _p(col),
                                   col.numel(), C.byref(o), _p(w64), None, _p(st), _p(res), _p(it), None)
    assert rc == EUNSUPPORTED
    o.prec = 4
    rc = lib.labfm_weights(h, _p(xt), _p(yt), xt.numel(), C.byref(dm), _p(Rt), _p(ot), _p(rp), _p(col),
                           col.numel(), C.byref(o), _p(w64), None, _p(st), _p(res), _p(it), None)
    assert rc == EINVAL and "bad prec" in _last(env)
    torch.cuda.synchronize()
