"""Pins of the oracle's time stepping (classical RK4, Sec. 5.1) against
closed-form solutions of the heat and advection-diffusion equations."""
import math

import numpy as np
import pytest

from paper_1912_06441_amd import workloads as WL


def _periodic_ops(O, side, k, Rs, eps, seed, ops=None):
    x, y, s = WL.jittered_lattice(side, eps=eps, seed=seed, periodic=True)
    dom = WL.unit_domain(True)
    rp, col, R = O.neighbours(x, y, dom, Rs * s, k)
    kw = {} if ops is None else dict(ops=ops)
    w, st, res, _ = O.weights(x, y, dom, R, k, rp, col, **kw)
    assert np.all(st == O.ST_OK)
    return x, y, s, rp, col, R, w


def test_heat_equation_decay():
    """Sec. 5.1 heat equation, periodic: u = sin(2 pi x) sin(2 pi y) exp(-8 pi^2 kappa t),
    kappa = 1, dt = 0.05 h^2 / kappa, eps/dr = 0.5, h/dr = 2; error falls ~ h^k."""
    import oracle as O

    errs = []
    for side in (24, 48):
        x, y, s, rp, col, R, w = _periodic_ops(O, side, 4, 4.0, 0.5, 3)
        h = 2.0 * s
        dt = 0.05 * h * h
        t_end = 0.25 / (8 * math.pi ** 2)
        nsteps = int(math.ceil(t_end / dt))
        dt = t_end / nsteps
        u0 = np.sin(2 * math.pi * x) * np.sin(2 * math.pi * y)
        u = O.rk4(rp, col, w[2], None, 0.0, dt, nsteps, u0)
        exact = u0 * math.exp(-8 * math.pi ** 2 * t_end)
        errs.append(np.linalg.norm(u - exact) / np.linalg.norm(exact))
    assert errs[1] < errs[0] / 8.0, errs  # order ~ k (k = 4), at least 3
    assert errs[1] < 1e-4


def test_advection_diffusion_gaussian():
    """u_t = -a.grad u + nu lap u from a Gaussian pulse on the unit torus;
    the closed form is the spreading, translating Gaussian summed over images.
    Order 6, h/dr = 2, eps/dr = 0.3, dt = 0.2 dr."""
    import oracle as O

    a, nu = (1.0, 0.5), 1e-3
    errs = []
    for side in (48, 96):
        x, y, s, rp, col, R, w = _periodic_ops(O, side, 6, 4.0, 0.3, 5)
        wlin = O.combine(w, [-a[0], -a[1], nu])
        dt = 0.2 * s
        nsteps = int(round(0.1 / dt))
        u0 = WL.gaussian_pulse(x, y)
        u = O.rk4(rp, col, wlin, None, 0.0, dt, nsteps, u0)
        exact = WL.advected_gaussian(x, y, nsteps * dt, a, nu)
        errs.append(np.abs(u - exact).max())
    assert errs[1] < errs[0] / 16.0, errs
    assert errs[1] < 1e-4, errs


def test_composed_hyperviscosity_is_dissipative():
    """The composed -gamma B(B u) term (B = -nabla^4 stencil, B o B ~ nabla^8)
    removes energy from a grid-scale mode and leaves a smooth mode almost
    untouched."""
    import oracle as O

    x, y, s, rp, col, R, w = _periodic_ops(O, 32, 6, 4.0, 0.3, 7, ops=O.OP_BIHARM)
    h = 2.0 * s
    dt = 0.2 * s
    gamma = 1e-7 * h ** 8 / dt  # beta = dt gamma / h^8 = 1e-7 (stable with RK4)
    zero = np.zeros_like(w[0])
    smooth = np.sin(2 * math.pi * x) * np.cos(2 * math.pi * y)
    rough = np.sin(2 * math.pi * 12 * x) * np.sin(2 * math.pi * 12 * y)
    us = O.rk4(rp, col, zero, w[0], gamma, dt, 50, smooth)
    ur = O.rk4(rp, col, zero, w[0], gamma, dt, 50, rough)
    assert np.linalg.norm(ur) < 0.9 * np.linalg.norm(rough)
    assert np.linalg.norm(us - smooth) < 1e-6 * np.linalg.norm(smooth)
    # exact check of one application: B applied to a degree-4 polynomial is -nabla^4
    i = 17
    s_, e_ = rp[i], rp[i + 1]
    dx = (x[col[s_:e_]] - x[i] + 0.5) % 1.0 - 0.5
    dy = (y[col[s_:e_]] - y[i] + 0.5) % 1.0 - 0.5
    f = dx ** 4 + dy ** 2 * dx ** 2
    assert (f * w[0][s_:e_]).sum() == pytest.approx(-(24.0 + 2 * 4.0), rel=1e-7)


def _csr_matrix(rp, col, w):
    """Dense matrix of L_i(u) = sum_j (u_j - u_i) w_ij (Sec. 3.1)."""
    n = rp.size - 1
    A = np.zeros((n, n))
    for i in range(n):
        for e in range(rp[i], rp[i + 1]):
            A[i, col[e]] += w[e]
            A[i, i] -= w[e]
    return A


@pytest.mark.parametrize("with_bh", [False, True])
def test_rk4_is_degree4_taylor_polynomial_with_dirichlet_nodes(with_bh):
    """On a linear system du/dt = D (A - gamma B B) u, where D zeroes the rows
    of the Dirichlet nodes, one classical RK4 step is exactly the degree-4
    Taylor polynomial of exp(dt D (A - gamma B B)); fixed nodes never move."""
    import oracle as O

    rng = np.random.default_rng(11)
    n = 14
    rp = [0]
    cols = []
    for i in range(n):
        nb = rng.choice([j for j in range(n) if j != i], size=int(rng.integers(2, 6)), replace=False)
        cols.extend(sorted(int(j) for j in nb))
        rp.append(len(cols))
    rp = np.array(rp, np.int64)
    col = np.array(cols, np.int32)
    w_lin = rng.normal(size=col.size)
    w_bh = rng.normal(size=col.size) if with_bh else None
    gamma = 0.3 if with_bh else 0.0
    fixed = np.zeros(n, np.int8)
    fixed[[0, 5, 13]] = 1
    u0 = rng.normal(size=n)
    dt, nsteps = 0.02, 7
    M = _csr_matrix(rp, col, w_lin)
    if with_bh:
        B = _csr_matrix(rp, col, w_bh)
        M = M - gamma * B @ B
    M = np.diag(1.0 - fixed) @ M
    Z = dt * M
    P = np.eye(n) + Z + Z @ Z / 2 + Z @ Z @ Z / 6 + Z @ Z @ Z @ Z / 24
    expect = np.linalg.matrix_power(P, nsteps) @ u0
    got = O.rk4(rp, col, w_lin, w_bh, gamma, dt, nsteps, u0, fixed=fixed)
    assert np.allclose(got, expect, rtol=0, atol=1e-12 * np.abs(expect).max())
    assert np.array_equal(got[fixed == 1], u0[fixed == 1])
    # no mask and an all-zero mask are the same integration
    a = O.rk4(rp, col, w_lin, w_bh, gamma, dt, nsteps, u0)
    b = O.rk4(rp, col, w_lin, w_bh, gamma, dt, nsteps, u0, fixed=np.zeros(n, np.int8))
    assert np.array_equal(a, b)
