"""Pins of the warm-start network reference (oracle/mlp.py) and of the batched
oracle solve that produces its training data.

What pins what:
  * SiLU and its derivative: closed-form values and central differences.
  * forward/backward: every parameter gradient against central differences
    of the forward pass (a dropped term, a sign or a transposed operand in the
    chain rule fails these).
  * moment_loss: zero at the solution of M Psi = C (numpy.linalg.solve), and
    its gradient against central differences.
  * adam_step: the closed form of bias-corrected Adam under a constant
    gradient (every update has size lr * |g| / (|g| + eps)).
  * stencil_features: brute force over all node pairs on a tiny set.
  * stencils_psi: X^T (W Psi^d) = C^d with X, W evaluated point by point
    (eq. disc_form and eq. lsys of Sec. 3.1).
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import mlp as OM
from paper_1912_06441_amd import workloads as WL


def test_silu_values_and_derivative():
    assert OM.silu(np.array([0.0]))[0] == 0.0
    assert OM.silu_grad(np.array([0.0]))[0] == 0.5
    z = np.array([-40.0, 40.0])
    assert abs(OM.silu(z)[0]) < 1e-15 and abs(OM.silu(z)[1] - 40.0) < 1e-12
    z = np.linspace(-6, 6, 25)
    h = 1e-6
    fd = (OM.silu(z + h) - OM.silu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - OM.silu_grad(z))) < 1e-8


def test_mlp_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    dims = (7, 6, 5, 4)
    Ws, bs = OM.init_params(dims, seed=5)
    bs = [rng.standard_normal(b.shape) * 0.3 for b in bs]
    X = rng.standard_normal((5, dims[0]))
    G = rng.standard_normal((5, dims[-1]))  # loss = sum(G * output)

    def loss():
        return float((OM.forward(Ws, bs, X)[0] * G).sum())

    _, cache = OM.forward(Ws, bs, X)
    dWs, dbs = OM.backward(Ws, cache, G)
    h = 1e-6
    for l in range(len(Ws)):
        for P, D in ((Ws[l], dWs[l]), (bs[l], dbs[l])):
            fd = np.zeros_like(P)
            for idx in np.ndindex(P.shape):
                old = P[idx]
                P[idx] = old + h
                lp = loss()
                P[idx] = old - h
                lm = loss()
                P[idx] = old
                fd[idx] = (lp - lm) / (2 * h)
            assert np.max(np.abs(fd - D)) <= 1e-7 * max(1.0, np.max(np.abs(D))), l


def test_moment_loss_zero_at_solution_and_gradient():
    rng = np.random.default_rng(7)
    B, nops, p = 3, 2, 5
    M = rng.standard_normal((B, p, p)) + 3 * np.eye(p)
    C = rng.standard_normal((nops, p))
    mu = rng.standard_normal(nops * p)
    sd = rng.uniform(0.5, 2.0, nops * p)
    # at the exact solution the loss vanishes
    Psi = np.stack([np.linalg.solve(M[s], C.T).T for s in range(B)]).reshape(B, nops * p)
    y_star = (Psi - mu) / sd
    loss, g = OM.moment_loss(y_star, M, C, mu, sd)
    assert loss < 1e-24 and np.max(np.abs(g)) < 1e-11
    # gradient by central differences away from it
    y = rng.standard_normal((B, nops * p))
    _, g = OM.moment_loss(y, M, C, mu, sd)
    h = 1e-6
    fd = np.zeros_like(y)
    for idx in np.ndindex(y.shape):
        yp = y.copy()
        yp[idx] += h
        ym = y.copy()
        ym[idx] -= h
        fd[idx] = (OM.moment_loss(yp, M, C, mu, sd)[0] - OM.moment_loss(ym, M, C, mu, sd)[0]) / (2 * h)
    assert np.max(np.abs(fd - g)) < 1e-6 * max(1.0, np.max(np.abs(g)))


def test_adam_constant_gradient_closed_form():
    g = np.array([2.0, -0.5, 1e-3, 0.0])
    theta = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 0.01, 1e-8
    for t in range(1, 6):
        new, m, v = OM.adam_step(theta, g, m, v, t, lr, eps=eps)
        step = new - theta
        expect = -lr * g / (np.abs(g) + eps)
        assert np.allclose(step, expect, rtol=1e-9, atol=1e-15), t
        theta = new


def test_stencil_features_brute_force():
    x, y, s = WL.jittered_lattice(10, eps=0.35, seed=11, periodic=True)
    dom = WL.unit_domain(True)
    order = np.full(x.size, 4, np.int8)
    rp, col, R = O.neighbours(x, y, dom, 2.9 * s, order, grow=True)
    kmax = 16
    F = OM.stencil_features(x, y, dom, R, rp, col, kmax=kmax).reshape(x.size, kmax, 3)
    for i in range(x.size):
        h = 0.5 * R[i]
        cand = []
        for j in range(x.size):
            if j == i:
                continue
            dx = x[j] - x[i]
            dy = y[j] - y[i]
            dx -= round(dx)
            dy -= round(dy)
            if dx * dx + dy * dy < R[i] * R[i]:
                a, b = dx / h, dy / h
                cand.append((a * a + b * b, j, a, b))
        cand.sort()
        k = min(len(cand), kmax)
        assert int(F[i, :, 2].sum()) == k
        for t in range(k):
            assert F[i, t, 0] == np.float32(cand[t][2]) and F[i, t, 1] == np.float32(cand[t][3])
        assert np.all(F[i, k:, :] == 0)
        assert np.all(F[i, :k, 0] ** 2 + F[i, :k, 1] ** 2 < 4.0 + 1e-5)


def test_stencils_psi_satisfies_moment_equations():
    x, y, s = WL.jittered_lattice(12, eps=0.3, seed=21, periodic=True)
    dom = WL.unit_domain(True)
    k = 6
    order = np.full(x.size, k, np.int8)
    rp, col, R = O.neighbours(x, y, dom, 4.0 * s, order, grow=True)
    dxa, dya = OM.stencil_offsets(x, y, dom, R, rp, col)
    nodes = [0, 17, 60, 143]
    N = np.array([rp[i + 1] - rp[i] for i in nodes], np.int32)
    Nmax = int(N.max())
    dx = np.zeros((len(nodes), Nmax))
    dy = np.zeros((len(nodes), Nmax))
    for t, i in enumerate(nodes):
        dx[t, :N[t]] = dxa[rp[i]:rp[i + 1]]
        dy[t, :N[t]] = dya[rp[i]:rp[i + 1]]
    ops = O.OP_DX | O.OP_DY | O.OP_LAP | O.OP_BIHARM
    psi, st, res, M = O.stencils_psi(k, dx, dy, N, want_M=True, ops=ops)
    assert np.all(st == 0)
    Ct = O.targets(ops, k)
    for t in range(len(nodes)):
        X = np.stack([O.monomials(k, dx[t, j], dy[t, j]) for j in range(N[t])])
        W = np.stack([O.abfs(k, dx[t, j], dy[t, j]) for j in range(N[t])])
        w = W @ psi[t].T  # [N, nops]
        assert np.max(np.abs(X.T @ w - Ct.T)) < 1e-9
        assert np.max(np.abs(M[t] - X.T @ W)) < 1e-9 * np.max(np.abs(M[t]))
