"""Learned warm start on the GPU against the FP64 oracle (oracle/mlp.py).

* features: bit-exact (same FP64 offsets, same ranking, FP32 rounding).
* matrix-core GEMM layouts: inputs exactly representable in BF16 make the
  forward product and the weight/bias gradients exact in FP32 (products of
  short dyadic numbers, sums far below 2^24 ulps), so they must equal the
  FP64 reference to FP32 rounding.
* full network: loss and every gradient against the FP64 reference with the
  same BF16-rounded weights; the GPU also rounds activations to BF16 at each
  product, so the bound is relative 3e-2 in the Frobenius norm.
* Adam: FP32 update against the FP64 formula, relative 1e-6.
* training on oracle stencils, then warm-started weights: every node passes the
  1e-10 moment gate and matches the oracle's weights like the mixed path; the
  trained network's initial residual beats a zero start.
* the warm start without a factorisation (PREC_MLP_NOLU): a zero network sends
  every node to the FP64 LU path (weights equal PREC_FP64's bit for bit,
  iters 64 + its count); on a perfect lattice (one stencil shape) a network
  that outputs the exact Psi finishes every node without a factorisation at a
  gate that FP32 Psi can meet, with the oracle's weights to FP32 accuracy.
* full scale (2 M training stencils, the 1024^2 set): the three routes and
  the LU-free one timed side by side; every route at the 1e-10 gate.
"""
import sys

import numpy as np
import pytest

from oracle import mlp as OM
from paper_1912_06441_amd import workloads as WL

import mlp_data as MD

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


def _dev(env, a, dtype=None):
    t = env["torch"].from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _bf16_round(a):
    """Round-to-nearest-even to BF16, returned as float64 (numpy bit arithmetic)."""
    f = np.ascontiguousarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _net(env, dims, seed, order=8, ops=7, kmax=None):
    L = env["L"]
    kmax = dims[0] // 3 if kmax is None else kmax
    return L.MLP(env["ctx"], dims=dims, order=order, ops=ops, kmax=kmax, seed=seed)


def _params64(net):
    Ws = [_bf16_round(w.cpu().numpy()) for w in net.W]
    bs = [b.cpu().numpy().astype(np.float64) for b in net.b]
    return Ws, bs


def _relF(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ---------------------------------------------------------------------------- features

@pytest.mark.parametrize("periodic,kmax", [(True, 64), (False, 64), (True, 16)])
def test_features_parity(env, periodic, kmax):
    O = env["O"]
    _say("features periodic=%s kmax=%d" % (periodic, kmax))
    x, y, s = WL.jittered_lattice(40, eps=0.35, seed=31, periodic=periodic)
    dom = WL.unit_domain(periodic)
    order = np.full(x.size, 8, np.int8)
    rp, col, R = O.neighbours(x, y, dom, 4.4 * s, order, grow=True)
    ref = OM.stencil_features(x, y, dom, R, rp, col, kmax=kmax)
    f = env["ctx"].mlp_features(_dev(env, x), _dev(env, y), _dev(env, R), _dev(env, rp), _dev(env, col), dom,
                                kmax=kmax)
    got = f.cpu().numpy()
    assert got.shape == ref.shape
    assert np.array_equal(got, ref)


# ---------------------------------------------------------------------------- GEMM layouts

def test_gemm_layouts_exact(env):
    """One linear layer with ragged sizes: forward, dW and db exact in FP32."""
    torch = env["torch"]
    rng = np.random.default_rng(1)
    K, N, B = 70, 45, 77
    net = _net(env, (K, N), seed=3, ops=1, order=1, kmax=1)
    W = rng.integers(-16, 17, (N, K)) / 16.0
    b = rng.integers(-8, 9, N) / 8.0
    net.W[0].copy_(torch.from_numpy(W).float())
    net.b[0].copy_(torch.from_numpy(b).float())
    net.sync_bf16()
    X = rng.integers(-8, 9, (B, K)) / 8.0
    Xt = _dev(env, X.astype(np.float32))
    out = net.forward(Xt)
    ref = X @ W.T + b
    assert np.max(np.abs(out.cpu().numpy() - ref)) <= 1e-6 * np.max(np.abs(ref))
    dY = rng.integers(-4, 5, (B, N)) / 4.0
    net.backward(Xt, None, _dev(env, dY.astype(np.float32)))
    torch.cuda.synchronize()
    assert np.array_equal(net.gW[0].cpu().numpy().astype(np.float64), dY.T @ X)
    assert np.array_equal(net.gb[0].cpu().numpy().astype(np.float64), dY.sum(0))


def test_gemm_forward_tiled_exact(env):
    """Layers whose K is a multiple of 32 take the 128 x 128 tiled kernel: exact
    on BF16-representable inputs with ragged M and N; a SiLU layer within the
    BF16 bound of the FP64 reference."""
    rng = np.random.default_rng(11)
    torch = env["torch"]
    B = 300
    net = _net(env, (64, 136), seed=5, ops=1, order=1, kmax=1)
    W = rng.integers(-16, 17, (136, 64)) / 16.0
    b = rng.integers(-8, 9, 136) / 8.0
    net.W[0].copy_(torch.from_numpy(W).float())
    net.b[0].copy_(torch.from_numpy(b).float())
    net.sync_bf16()
    X = rng.integers(-8, 9, (B, 64)) / 8.0
    Xt = _dev(env, X.astype(np.float32))
    ref = X @ W.T + b
    for out in (net.forward(Xt), net.forward(Xt, cache=net.cache_for(B))):  # fused inference, tiled layer
        assert np.max(np.abs(out.cpu().numpy() - ref)) <= 1e-6 * np.max(np.abs(ref))
    net2 = _net(env, (32, 256, 40), seed=6, ops=1, order=1, kmax=1)
    X2 = rng.standard_normal((B, 32))
    cache = net2.cache_for(B)
    out2 = net2.forward(_dev(env, X2.astype(np.float32)), cache=cache)
    Ws, bs = _params64(net2)
    ref2, _ = OM.forward(Ws, bs, X2)
    assert _relF(out2.cpu().numpy(), ref2) < 1e-2


def test_gemm_two_layers_backward(env):
    """Hidden SiLU layer: the dH = dZ W path and the SiLU derivative."""
    torch = env["torch"]
    rng = np.random.default_rng(2)
    dims, B = (20, 33, 9), 50
    net = _net(env, dims, seed=4, ops=1, order=1, kmax=1)
    X = rng.standard_normal((B, dims[0]))
    Xt = _dev(env, X.astype(np.float32))
    cache = net.cache_for(B)
    out = net.forward(Xt, cache=cache)
    Ws, bs = _params64(net)
    ref, rc = OM.forward(Ws, bs, X)
    assert _relF(out.cpu().numpy(), ref) < 1e-2
    dY = rng.standard_normal((B, dims[-1]))
    net.backward(Xt, cache, _dev(env, dY.astype(np.float32)))
    dWs, dbs = OM.backward(Ws, rc, dY)
    torch.cuda.synchronize()
    for l in range(2):
        assert _relF(net.gW[l].cpu().numpy(), dWs[l]) < 2e-2, l
        assert _relF(net.gb[l].cpu().numpy(), dbs[l]) < 2e-2, l


# ---------------------------------------------------------------------------- loss, gradients, Adam

@pytest.fixture(scope="module")
def small_set():
    """Order-8 stencils of one jittered lattice with oracle targets."""
    cfg = WL.config("c4")
    L = MD.lattice_stencils(32, 0.3, 4100, cfg["k"], cfg["R_s"])
    psi, M, st = MD.targets(L, cfg["k"], cfg["ops"])
    assert np.all(st == 0)
    feat = OM.stencil_features(L["x"], L["y"], L["domain"], L["R"], L["rp"], L["col"], kmax=cfg["kmax"])
    return dict(L=L, psi=psi, M=M, feat=feat, cfg=cfg)


def test_fused_inference_matches_layers(env, small_set):
    """Inference through all layers in one kernel (activations kept in LDS as
    BF16) against the layer-by-layer kernels and the FP64 reference."""
    cfg = small_set["cfg"]
    net = _net(env, cfg["dims"], seed=12)
    mu, sd = MD.robust_scaling(small_set["psi"])
    net.set_output_scaling(mu, sd)
    X = small_set["feat"][:777]
    Xt = _dev(env, X)
    fused = net.forward(Xt, denorm=True).cpu().numpy()
    layered = net.forward(Xt, cache=net.cache_for(X.shape[0]), denorm=True).cpu().numpy()
    assert np.max(np.abs(fused - layered)) <= 1e-5 * np.max(np.abs(layered))
    Ws, bs = _params64(net)
    ref, _ = OM.forward(Ws, bs, X.astype(np.float64))
    assert _relF(net.forward(Xt).cpu().numpy(), ref) < 1e-2


def test_moment_loss_parity(env, small_set):
    torch = env["torch"]
    cfg = small_set["cfg"]
    B = 200
    rng = np.random.default_rng(5)
    net = _net(env, cfg["dims"], seed=1)
    mu, sd = MD.robust_scaling(small_set["psi"])
    net.set_output_scaling(mu, sd)
    y = rng.standard_normal((B, cfg["dims"][-1])).astype(np.float32)
    M = small_set["M"][:B].astype(np.float32)
    loss, dy = net.moment_loss(_dev(env, y), _dev(env, M))
    torch.cuda.synchronize()
    C = env["O"].targets(cfg["ops"], cfg["k"])
    mu32 = np.float32(mu).astype(np.float64)
    sd32 = np.float32(sd).astype(np.float64)
    lref, gref = OM.moment_loss(y.astype(np.float64), M.astype(np.float64), C, mu32, sd32)
    assert abs(loss.sum().item() / B - lref) <= 1e-9 * lref
    assert np.max(np.abs(dy.cpu().numpy() - gref)) <= 1e-6 * np.max(np.abs(gref))


def test_network_gradients_vs_oracle(env, small_set):
    torch = env["torch"]
    cfg = small_set["cfg"]
    B = 256
    net = _net(env, cfg["dims"], seed=7)
    mu, sd = MD.robust_scaling(small_set["psi"])
    net.set_output_scaling(mu, sd)
    X = small_set["feat"][:B]
    M = small_set["M"][:B].astype(np.float32)
    Xt, Mt = _dev(env, X), _dev(env, M)
    cache = net.cache_for(B)
    y = net.forward(Xt, cache=cache)
    loss, dy = net.moment_loss(y, Mt)
    net.backward(Xt, cache, dy)
    torch.cuda.synchronize()
    Ws, bs = _params64(net)
    yref, rc = OM.forward(Ws, bs, X.astype(np.float64))
    C = env["O"].targets(cfg["ops"], cfg["k"])
    lref, gref = OM.moment_loss(yref, M.astype(np.float64), C, np.float32(mu).astype(np.float64),
                                np.float32(sd).astype(np.float64))
    dWs, dbs = OM.backward(Ws, rc, gref)
    _say("  loss gpu %.6e oracle %.6e" % (loss.sum().item() / B, lref))
    assert abs(loss.sum().item() / B - lref) <= 3e-2 * lref
    for l in range(len(Ws)):
        eW, eb = _relF(net.gW[l].cpu().numpy(), dWs[l]), _relF(net.gb[l].cpu().numpy(), dbs[l])
        _say("  layer %d grad rel err W %.2e b %.2e" % (l, eW, eb))
        assert eW < 3e-2 and eb < 3e-2


def test_adam_parity(env):
    torch = env["torch"]
    rng = np.random.default_rng(9)
    net = _net(env, (30, 20, 6), seed=2, ops=1, order=1, kmax=10)
    W0 = net.W[0].cpu().numpy().astype(np.float64)
    m = np.zeros_like(W0)
    v = np.zeros_like(W0)
    th = W0.copy()
    for t in range(1, 4):
        g = rng.standard_normal(W0.shape)
        for l in range(net.L):
            net.gW[l].copy_(torch.from_numpy(g if l == 0 else np.zeros(net.gW[l].shape)).float())
            net.gb[l].zero_()
        net.adam(lr=1e-2)
        th, m, v = OM.adam_step(th, np.float32(g).astype(np.float64), m, v, t, 1e-2)
    torch.cuda.synchronize()
    got = net.W[0].cpu().numpy()
    assert np.max(np.abs(got - th)) <= 1e-6 * max(1.0, np.max(np.abs(th)))
    assert np.array_equal(net.Wb[0].cpu().float().numpy(), _bf16_round(got).astype(np.float32))


# ---------------------------------------------------------------------------- training + warm start

def _train(env, cfg, sets, epochs, seed=0):
    """Train on oracle stencils of `sets` lattices; returns the network."""
    torch = env["torch"]
    feats, Ms, psis = [], [], []
    for i in range(sets):
        eps = float(np.random.default_rng(cfg["train_seed0"] + i).uniform(0.0, cfg["eps_max"]))
        L = MD.lattice_stencils(cfg["train_side"], eps, cfg["train_seed0"] + i, cfg["k"], cfg["R_s"])
        psi, M, st = MD.targets(L, cfg["k"], cfg["ops"])
        keep = st == 0
        f = env["ctx"].mlp_features(_dev(env, L["x"]), _dev(env, L["y"]), _dev(env, L["R"]), _dev(env, L["rp"]),
                                    _dev(env, L["col"]), L["domain"], kmax=cfg["kmax"])
        feats.append(f[_dev(env, keep)])
        Ms.append(_dev(env, M[keep].astype(np.float32)))
        psis.append(psi[keep])
    X = torch.cat(feats)
    M = torch.cat(Ms)
    mu, sd = MD.robust_scaling(np.concatenate(psis))
    n = X.shape[0]
    net = env["L"].MLP(env["ctx"], dims=cfg["dims"], order=cfg["k"], ops=cfg["ops"], kmax=cfg["kmax"], seed=seed)
    net.set_output_scaling(mu, sd)
    g = torch.Generator(device="cuda").manual_seed(seed)
    batch = cfg["batch"]
    cache = net.cache_for(batch)
    steps = epochs * (n // batch)
    t = 0
    for e in range(epochs):
        perm = torch.randperm(n, device="cuda", generator=g)
        tot = 0.0
        for b in range(n // batch):
            idx = perm[b * batch:(b + 1) * batch]
            lr = cfg["lr"] * 0.5 * (1.0 + np.cos(np.pi * t / steps))
            loss = net.train_step(X[idx].contiguous(), M[idx].contiguous(), lr, cache=cache)
            t += 1
            if b == 0:
                tot = loss.mean().item()
        _say("  epoch %d first-batch loss %.4e" % (e, tot))
    return net, n


def test_mlp_training_and_warm_start(env):
    torch = env["torch"]
    O = env["O"]
    L = env["L"]
    cfg = WL.config("c4")
    _say("training on %d lattices of %d^2 stencils" % (cfg["test_sets"], cfg["train_side"]))
    net, ntrain = _train(env, cfg, cfg["test_sets"], cfg["test_epochs"])
    # evaluation node set (held out)
    E = MD.lattice_stencils(cfg["test_eval_side"], cfg["eval_eps"], cfg["eval_seed"], cfg["k"], cfg["R_s"])
    psi_e, M_e, st_e = MD.targets(E, cfg["k"], cfg["ops"])
    assert np.all(st_e == 0)
    xt, yt, Rt = _dev(env, E["x"]), _dev(env, E["y"]), _dev(env, E["R"])
    ot, rpt, colt = _dev(env, E["order"]), _dev(env, E["rp"]), _dev(env, E["col"])
    # initial moment residuals: trained network vs untrained network vs zero start
    feat = env["ctx"].mlp_features(xt, yt, Rt, rpt, colt, E["domain"], kmax=cfg["kmax"])
    Mt = _dev(env, M_e.astype(np.float32))
    fresh = L.MLP(env["ctx"], dims=cfg["dims"], order=cfg["k"], ops=cfg["ops"], kmax=cfg["kmax"], seed=99)
    fresh.set_output_scaling(net.mu.cpu().numpy(), net.sd.cpu().numpy())
    r_tr = net.moment_loss(net.forward(feat), Mt)[0].sqrt().cpu().numpy()
    r_un = fresh.moment_loss(fresh.forward(feat), Mt)[0].sqrt().cpu().numpy()
    C = O.targets(cfg["ops"], cfg["k"])
    r_zero = float(np.sqrt((C * C).sum()))
    _say("  initial |r|_2 median: trained %.3e  untrained %.3e  zero start %.3e" %
         (np.median(r_tr), np.median(r_un), r_zero))
    assert np.median(r_tr) < 0.5 * r_zero
    assert np.median(r_tr) < 0.5 * np.median(r_un)
    # warm-started weights vs the oracle and vs the mixed path
    w_or, st_or, res_or, _ = O.weights(E["x"], E["y"], E["domain"], E["R"], E["order"], E["rp"], E["col"])
    out = {}
    for name, prec in (("mixed", L.PREC_MIXED), ("mlp", L.PREC_MLP)):
        w64, _, st, res, it = env["ctx"].weights(xt, yt, Rt, ot, rpt, colt, E["domain"], prec=prec, mlp=net)
        torch.cuda.synchronize()
        out[name] = (w64.cpu().numpy(), st.cpu().numpy(), res.cpu().numpy(), it.cpu().numpy().astype(int))
    # zero start through the same warm-start path (network output scaled to 0)
    zero = L.MLP(env["ctx"], dims=cfg["dims"], order=cfg["k"], ops=cfg["ops"], kmax=cfg["kmax"], seed=1)
    zero.set_output_scaling(np.zeros(cfg["dims"][-1]), np.zeros(cfg["dims"][-1]))
    w64, _, st, res, it = env["ctx"].weights(xt, yt, Rt, ot, rpt, colt, E["domain"], prec=L.PREC_MLP, mlp=zero)
    torch.cuda.synchronize()
    out["zero"] = (w64.cpu().numpy(), st.cpu().numpy(), res.cpu().numpy(), it.cpu().numpy().astype(int))
    for name, (w, st, res, it) in out.items():
        fb = int((it >= 64).sum())
        sweeps = np.where(it >= 64, np.nan, it)
        _say("  %-5s status ok %d/%d  max resid %.2e  fallback %d  mean sweeps %.3f" %
             (name, int((st == 0).sum()), st.size, float(res.max()), fb, float(np.nanmean(sweeps))))
        assert np.all(st == 0) and float(res.max()) <= 1e-10
        # same bar as the mixed path: weights of every node against the oracle
        rel = np.abs(w - w_or).max() / np.abs(w_or).max()
        assert rel <= 1e-8, (name, rel)
    m_tr = np.nanmean(np.where(out["mlp"][3] >= 64, np.nan, out["mlp"][3]))
    m_zero = np.nanmean(np.where(out["zero"][3] >= 64, np.nan, out["zero"][3]))
    assert m_tr <= m_zero


@pytest.mark.parametrize("k,abf,rbf", [(8, 0, 0), (4, 2, 2)])
def test_moment_systems_parity(env, k, abf, rbf):
    """Training data made on the GPU: moment matrices within FP32 rounding of the
    oracle's, coefficients within 1e-5 per node (one FP64 solve, then FP32),
    statuses equal."""
    O = env["O"]
    E = MD.lattice_stencils(40, 0.3, 11, k, {8: 4.4, 4: 2.85}[k], periodic=(k == 8))
    dx, dy, N = MD.padded_offsets(E)
    psi_o, st_o, _, M_o = O.stencils_psi(k, dx, dy, N, want_M=True, ops=7, family=abf, rbf=rbf)
    xt, yt, Rt = _dev(env, E["x"]), _dev(env, E["y"]), _dev(env, E["R"])
    rpt, colt = _dev(env, E["rp"]), _dev(env, E["col"])
    M, psi, st = env["ctx"].moment_systems(xt, yt, Rt, k, rpt, colt, E["domain"], ops=7, abf=abf, rbf=rbf)
    env["torch"].cuda.synchronize()
    M, psi, st = M.cpu().numpy(), psi.cpu().numpy(), st.cpu().numpy()
    ok = st_o == 0
    assert np.all(st[ok] == 0) and ok.mean() > 0.9
    final = (st_o != 0) & (st_o != 1)  # failures before any refinement
    assert np.array_equal(st[final], st_o[final])
    dM = np.abs(M[ok] - M_o[ok]).max(axis=(1, 2)) / np.abs(M_o[ok]).max(axis=(1, 2))
    po = psi_o.reshape(psi_o.shape[0], -1)[ok]
    dP = np.abs(psi[ok] - po).max(axis=1) / np.abs(po).max(axis=1)
    _say("  moment systems k=%d abf %d: M rel max %.2e, Psi rel max %.2e median %.2e" %
         (k, abf, dM.max(), dP.max(), np.median(dP)))
    assert dM.max() <= 1e-6 and dP.max() <= 1e-5
    bad = st != 0
    assert np.all(M[bad] == 0) and np.all(psi[bad] == 0)


def test_warm_start_without_factorisation(env):
    torch, O, L = env["torch"], env["O"], env["L"]
    k, ops, kmax = 4, 7, 16
    P = O.p_of_k(k)
    dims = (3 * kmax, 16, 3 * P)
    cases = {}
    for name, eps in (("jittered", 0.3), ("perfect", 0.0)):
        E = MD.lattice_stencils(24, eps, 7, k, 2.85)
        cases[name] = (E, [_dev(env, E[a]) for a in ("x", "y", "R", "order", "rp", "col")])
    # (a) zero network: every node above the gate, all solved by the FP64 LU path
    E, (xt, yt, Rt, ot, rpt, colt) = cases["jittered"]
    zero = L.MLP(env["ctx"], dims=dims, order=k, ops=ops, kmax=kmax, seed=1)
    zero.set_output_scaling(np.zeros(dims[-1]), np.zeros(dims[-1]))
    ref = env["ctx"].weights(xt, yt, Rt, ot, rpt, colt, E["domain"], prec=L.PREC_FP64)
    got = env["ctx"].weights(xt, yt, Rt, ot, rpt, colt, E["domain"], prec=L.PREC_MLP_NOLU, mlp=zero)
    torch.cuda.synchronize()
    assert torch.equal(got[0], ref[0]) and torch.equal(got[2], ref[2]) and torch.equal(got[3], ref[3])
    assert torch.equal(got[4].to(torch.int32), ref[4].to(torch.int32) + 64)
    # (b) the exact Psi of the one stencil shape, rounded to FP32: no node needs a factorisation
    E, (xt, yt, Rt, ot, rpt, colt) = cases["perfect"]
    psi, M, st = MD.targets(E, k, ops)
    assert np.all(st == 0) and np.abs(psi - psi[0]).max() <= 1e-12 * np.abs(psi[0]).max()
    exact = L.MLP(env["ctx"], dims=dims, order=k, ops=ops, kmax=kmax, seed=2)
    exact.set_output_scaling(psi[0], np.zeros(dims[-1]))
    w64, _, st, res, it = env["ctx"].weights(xt, yt, Rt, ot, rpt, colt, E["domain"], prec=L.PREC_MLP_NOLU,
                                             mlp=exact, tol_pass=1e-6)
    torch.cuda.synchronize()
    w_or, st_or, _, _ = O.weights(E["x"], E["y"], E["domain"], E["R"], E["order"], E["rp"], E["col"])
    rel = np.abs(w64.cpu().numpy() - w_or).max() / np.abs(w_or).max()
    _say("  no factorisation, exact Psi in FP32: max residual %.2e, weights vs oracle %.2e" %
         (float(res.max()), rel))
    assert np.all(st.cpu().numpy() == 0) and np.all(it.cpu().numpy() == 0) and float(res.max()) <= 1e-6
    assert rel <= 1e-6
    # at the 1e-10 gate the FP32 Psi cannot finish a node: all go to the FP64 path
    w64, _, st, res, it = env["ctx"].weights(xt, yt, Rt, ot, rpt, colt, E["domain"], prec=L.PREC_MLP_NOLU,
                                             mlp=exact)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == 0) and np.all(it.cpu().numpy() >= 64) and float(res.max()) <= 1e-10


def test_mlp_full_scale_measurement(env):
    """Configured scale: train on stencils of train_sets lattices, evaluate on the
    1024x1024 set against the mixed and FP64 paths (time per node, refinement
    sweeps, fallback rate, residual), weights checked against the oracle on a sample."""
    import time

    torch = env["torch"]
    O = env["O"]
    L = env["L"]
    cfg = WL.config("c4")
    cfg["test_epochs"] = int(__import__("os").environ.get("LABFM_C4_EPOCHS", "6"))
    cfg["batch"] = 2048
    _say("full scale: %d lattices of %d^2 training stencils, %d epochs" %
         (cfg["train_sets"], cfg["train_side"], cfg["test_epochs"]))
    t0 = time.time()
    net, ntrain = _train(env, cfg, cfg["train_sets"], cfg["test_epochs"])
    _say("  trained on %d stencils in %.0f s" % (ntrain, time.time() - t0))
    E = MD.lattice_stencils(cfg["eval_side"], cfg["eval_eps"], cfg["eval_seed"], cfg["k"], cfg["R_s"])
    xt, yt, Rt = _dev(env, E["x"]), _dev(env, E["y"]), _dev(env, E["R"])
    ot, rpt, colt = _dev(env, E["order"]), _dev(env, E["rp"]), _dev(env, E["col"])
    n = E["x"].size
    res = {}
    for name, prec in (("fp64", L.PREC_FP64), ("mixed", L.PREC_MIXED), ("mlp", L.PREC_MLP),
                       ("nolu", L.PREC_MLP_NOLU)):
        out = env["ctx"].weights(xt, yt, Rt, ot, rpt, colt, E["domain"], prec=prec, mlp=net)
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            t1 = time.perf_counter()
            env["ctx"].weights(xt, yt, Rt, ot, rpt, colt, E["domain"], prec=prec, mlp=net, out=out)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t1)
        st = out[2].cpu().numpy()
        it = out[4].cpu().numpy().astype(int)
        r = out[3].cpu().numpy()
        sweeps = it[it < 64]
        res[name] = out
        _say("  %-5s %.1f ms (%.1f ns/node)  ok %d/%d  max resid (ok nodes) %.2e  fallback %d (%.2e)  "
             "mean sweeps %.3f" %
             (name, 1e3 * min(ts), 1e9 * min(ts) / n, int((st == 0).sum()), n, float(r[st == 0].max()),
              int((it >= 64).sum()), float((it >= 64).mean()), float(sweeps.mean()) if sweeps.size else 0.0))
        # as for the mixed path at 512^2: at most n/10000 nodes (cond(M) >= 1e8) may miss the gate
        assert int((st != 0).sum()) <= max(1, n // 10000) and float(r[st == 0].max()) <= 1e-10
    # oracle on a sample of nodes: weights of the warm-started path
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(n, 2000, replace=False))
    w_mlp = res["mlp"][0].cpu().numpy()
    dx, dy = OM.stencil_offsets(E["x"], E["y"], E["domain"], E["R"], E["rp"], E["col"])
    st_mlp = res["mlp"][2].cpu().numpy()
    for i in sample:
        if st_mlp[i] != 0:
            continue
        s0, s1 = E["rp"][i], E["rp"][i + 1]
        r_ = O.node_weights(cfg["k"], dx[s0:s1], dy[s0:s1])
        h = 0.5 * E["R"][i]
        ref = r_["what"] / np.array([h, h, h * h])[:, None]
        got = w_mlp[:, s0:s1]
        assert np.abs(got - ref).max() <= 1e-8 * np.abs(ref).max(), i
