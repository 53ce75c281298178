"""The 1024x1024 periodic order-6 workloads at full size, in the launch
configuration bench.py times, against the oracle run at full size.

* Neighbour lists bit-exact; every node's {dx, dy, lap, -nabla^4} weights pass
  the 1e-10 gate with the oracle's status; per-node weight parity <= 1e-10 on
  a sample of 20,000 rows.
* RK4 advection-diffusion with composed hyperviscosity, FP32 weights and
  state, graph-replayed (the benchmark's step): two steps against the oracle's
  FP64 RK4 on its own weights, max |du| <= 1e-4 max |u| (the FP32 bound of
  the small-set test).
* Burgers (FP32, Re = 100, the benchmark's step, half of eq. (tstep)): ten
  steps of the paired-state stage kernel against the oracle's FP64 Burgers
  RK4, same bound.
* The configured run: 1000 FP32 steps against 1000 FP64 oracle steps at
  t_end, max |du| <= 1e-3 max |u| (measured 4.1e-7).
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
def full():
    import torch

    import oracle as O
    import paper_1912_06441_amd as L

    assert torch.cuda.is_available()
    cfg = WL.config("c5")
    nd = WL.make_nodes(cfg)
    _say("full 1024^2: %d nodes" % nd["x"].size)
    rp_o, col_o, R_o = O.neighbours(nd["x"], nd["y"], nd["domain"], nd["R"], nd["order"])
    w_o, st_o, res_o, _ = O.weights(nd["x"], nd["y"], nd["domain"], R_o, nd["order"], rp_o, col_o, ops=1 | 2 | 4 | 8)
    _say("  oracle: nnz %d, weights status %s" % (rp_o[-1], np.bincount(st_o)))
    ctx = L.Context(0)
    dev = torch.device("cuda:0")
    x = torch.from_numpy(nd["x"]).to(dev)
    y = torch.from_numpy(nd["y"]).to(dev)
    R = torch.from_numpy(nd["R"]).to(dev)
    order = torch.from_numpy(nd["order"]).to(dev)
    rp, col = ctx.build_neighbours(x, y, R, order, nd["domain"])
    w64, _, st, res, _ = ctx.weights(x, y, R, order, rp, col, nd["domain"], ops=1 | 2 | 4 | 8)
    torch.cuda.synchronize()
    yield dict(torch=torch, O=O, L=L, ctx=ctx, cfg=cfg, nd=nd, rp_o=rp_o, col_o=col_o, w_o=w_o, st_o=st_o,
               rp=rp, col=col, w64=w64, st=st.cpu().numpy(), res=res.cpu().numpy())
    torch.cuda.synchronize()
    ctx.close()


def test_full_weights(full):
    f = full
    assert np.array_equal(f["rp"].cpu().numpy(), f["rp_o"])
    assert np.array_equal(f["col"].cpu().numpy(), f["col_o"])
    assert np.array_equal(f["st"], f["st_o"]) and np.all(f["st"] == 0)
    assert f["res"].max() <= 1e-10
    rng = np.random.default_rng(0)
    rows = rng.choice(f["rp_o"].size - 1, 20000, replace=False)
    w = f["w64"].cpu().numpy()
    worst = 0.0
    for i in rows:
        s, e = f["rp_o"][i], f["rp_o"][i + 1]
        for d in range(4):
            worst = max(worst, np.abs(w[d, s:e] - f["w_o"][d, s:e]).max() / np.abs(f["w_o"][d, s:e]).max())
    _say("  sampled weight parity max %.2e" % worst)
    assert worst <= 1e-10


def test_full_rk4_fp32_step(full):
    f = full
    torch, O, cfg, nd = f["torch"], f["O"], f["cfg"], f["nd"]
    a, nu = cfg["a"], cfg["nu"]
    _, wlin = f["ctx"].combine(f["w64"][:3], [-a[0], -a[1], nu], want64=False, want32=True)
    wbh = f["w64"][3].to(torch.float32)
    s = nd["s"]
    h = 0.5 * cfg["R_s"] * s
    dt = cfg["dt_s"] * s
    gamma = cfg["beta"] * h ** 8 / dt
    u0 = WL.gaussian_pulse(nd["x"], nd["y"])
    u = torch.from_numpy(u0).cuda().to(torch.float32)
    scratch = torch.empty(5 * u0.size, dtype=torch.float32, device="cuda")
    f["ctx"].step(f["rp"], f["col"], wlin, wbh, gamma, dt, u, 2, scratch=scratch)
    torch.cuda.synchronize()
    wlin_o = O.combine(f["w_o"][:3], [-a[0], -a[1], nu])
    ref = O.rk4(f["rp_o"], f["col_o"], wlin_o, f["w_o"][3], gamma, dt, 2, u0)
    err = np.abs(u.double().cpu().numpy() - ref).max() / np.abs(ref).max()
    _say("  full RK4 (2 FP32 steps) vs FP64 oracle: %.2e" % err)
    assert err <= 1e-4


def test_full_burgers_fp32_step(full):
    f = full
    torch, O, nd = f["torch"], f["O"], f["nd"]
    Re = 100.0
    h = 0.5 * f["cfg"]["R_s"] * nd["s"]
    dt = 0.5 * WL.burgers_dt(h, 1.0, Re)  # the benchmark's step: half of eq. (tstep) on this node set
    xs, ys = nd["x"], nd["y"]
    u0 = np.sin(2 * np.pi * xs) * np.sin(2 * np.pi * ys)
    v0 = -np.cos(2 * np.pi * xs) * np.cos(2 * np.pi * ys)
    w = [f["w64"][d].to(torch.float32) for d in range(3)]
    u = torch.from_numpy(u0).cuda().to(torch.float32)
    v = torch.from_numpy(v0).cuda().to(torch.float32)
    nsteps = 10
    f["ctx"].burgers_step(f["rp"], f["col"], w[0], w[1], w[2], 1.0 / Re, dt, u, v, nsteps)
    torch.cuda.synchronize()
    uo, vo = O.burgers_rk4(f["rp_o"], f["col_o"], f["w_o"][0], f["w_o"][1], f["w_o"][2], None, 1.0 / Re, dt, nsteps,
                           u0, v0)
    err = max(np.abs(u.double().cpu().numpy() - uo).max() / np.abs(uo).max(),
              np.abs(v.double().cpu().numpy() - vo).max() / np.abs(vo).max())
    _say("  full Burgers (%d FP32 steps) vs FP64 oracle: %.2e" % (nsteps, err))
    assert err <= 1e-4


def test_full_poisson_solve(full):
    """The benchmark's periodic Poisson solve (node 0 pinned, 1e-10): the GPU
    solution's residual measured with the oracle's own Laplacian rows, and its
    error against sin(2 pi x) sin(2 pi y)."""
    f = full
    torch, nd = f["torch"], f["nd"]
    from oracle import poisson as P

    n = nd["x"].size
    fixed = np.zeros(n, np.int8)
    fixed[0] = 1
    F, x0 = WL.poisson_system(nd["x"], nd["y"], fixed)
    phi, it, res, ok = f["ctx"].poisson_solve(f["rp"], f["col"], f["w64"][2].contiguous(), torch.from_numpy(F).cuda(),
                                              phi=torch.from_numpy(x0).cuda(), fixed=torch.from_numpy(fixed).cuda(),
                                              tol=1e-10, max_iters=20000, check_every=32)
    g = phi.cpu().numpy()
    A = P.laplacian_matrix(f["rp_o"], f["col_o"], f["w_o"][2], fixed)
    r = np.linalg.norm(F - A @ g) / np.linalg.norm(F)
    err = np.linalg.norm(g - WL.poisson_solution(nd["x"], nd["y"])) / np.linalg.norm(WL.poisson_solution(nd["x"], nd["y"]))
    _say("  full Poisson: %d iterations, GPU residual %.2e, residual with the oracle's rows %.2e, L2 error %.2e" %
         (it, res, r, err))
    assert ok and r <= 1e-9 and err <= 1e-8


def test_full_rk4_1000_steps(full):
    """The configured run: 1000 FP32 RK4 steps of the advected, diffused and
    hyperviscous Gaussian pulse on the GPU against 1000 FP64 steps of the
    oracle at t_end; both against the free-space solution (periodic images)."""
    f = full
    torch, O, cfg, nd = f["torch"], f["O"], f["cfg"], f["nd"]
    a, nu = cfg["a"], cfg["nu"]
    _, wlin = f["ctx"].combine(f["w64"][:3], [-a[0], -a[1], nu], want64=False, want32=True)
    wbh = f["w64"][3].to(torch.float32)
    s = nd["s"]
    h = 0.5 * cfg["R_s"] * s
    dt = cfg["dt_s"] * s
    gamma = cfg["beta"] * h ** 8 / dt
    nsteps = cfg["nsteps"]
    u0 = WL.gaussian_pulse(nd["x"], nd["y"])
    u = torch.from_numpy(u0).cuda().to(torch.float32)
    scratch = torch.empty(5 * u0.size, dtype=torch.float32, device="cuda")
    f["ctx"].step(f["rp"], f["col"], wlin, wbh, gamma, dt, u, nsteps, scratch=scratch)
    torch.cuda.synchronize()
    _say("  oracle: %d FP64 RK4 steps at 1024^2" % nsteps)
    wlin_o = O.combine(f["w_o"][:3], [-a[0], -a[1], nu])
    ref = np.array(u0)
    for _ in range(nsteps // 50):  # progress lines between legs
        ref = O.rk4(f["rp_o"], f["col_o"], wlin_o, f["w_o"][3], gamma, dt, 50, ref)
        _say("  ...")
    g = u.double().cpu().numpy()
    err = np.abs(g - ref).max() / np.abs(ref).max()
    ex = WL.advected_gaussian(nd["x"], nd["y"], nsteps * dt, a, nu)
    _say("  1000 FP32 steps vs FP64 oracle: %.2e; L2 vs free-space solution: gpu %.2e oracle %.2e" %
         (err, np.linalg.norm(g - ex) / np.linalg.norm(ex), np.linalg.norm(ref - ex) / np.linalg.norm(ex)))
    assert err <= 1e-3


def test_full_rk4_step_growth(full):
    """Reading of the configured time step: on this node set the RK4 step map
    with the composed hyperviscosity grows at dt = 0.2 s and decays at the
    0.1 s the benchmark runs (power iteration of the FP64 step on the GPU; the
    oracle at full size gives 5.05 and 0.993 per step)."""
    f = full
    torch = f["torch"]
    cfg, nd = f["cfg"], f["nd"]
    a, nu = cfg["a"], cfg["nu"]
    wlin, _ = f["ctx"].combine(f["w64"][:3], [-a[0], -a[1], nu], want64=True, want32=False)
    wbh = f["w64"][3].contiguous()
    s = nd["s"]
    h = 0.5 * cfg["R_s"] * s
    n = nd["x"].size
    growth = {}
    for dts in (0.2, 0.1):
        dt = dts * s
        gamma = cfg["beta"] * h ** 8 / dt
        g = torch.Generator(device="cuda").manual_seed(0)
        u = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
        u /= u.norm()
        scratch = torch.empty(5 * n, dtype=torch.float64, device="cuda")
        rates = []
        for _ in range(40):
            f["ctx"].step(f["rp"], f["col"], wlin, wbh, gamma, dt, u, 1, scratch=scratch)
            nrm = u.norm()
            rates.append(float(nrm))
            u /= nrm
        growth[dts] = float(np.mean(rates[-10:]))
    _say("  RK4 step growth per step: dt = 0.2 s %.3f, dt = 0.1 s %.4f" % (growth[0.2], growth[0.1]))
    assert growth[0.2] > 2.0 and growth[0.1] < 1.0
