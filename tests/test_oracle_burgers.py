"""Pins of the oracle's viscous Burgers' solver (Sec. 5.3) and of the exact
solution it is measured against.

* The Cole-Hopf series (with the decay exponent the transform gives) satisfies
  u_t + u u_x = u_xx / Re by finite differences and starts from sin(2 pi x).
* RK4 order: one step on a random nonlinear stencil system differs from a
  tight-tolerance integration by O(dt^5) (halving dt divides it by ~32).
* Difference form: constant fields are steady; without advection weights the
  solver is the linear RK4 on nu * lap.
* Periodic sawtooth (Re = 100, eps/dr = 0.2, h/dr = 2): the error against the
  exact solution falls with resolution at k = 4 and 6; v stays exactly zero.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from paper_1912_06441_amd import workloads as WL


def test_cole_hopf_series_solves_burgers():
    Re = 100.0
    x = np.linspace(0.03, 0.97, 11)
    assert np.abs(WL.burgers_cole_hopf(x, 0.0, Re) - np.sin(2 * math.pi * x)).max() < 1e-9
    for t in (0.05, 0.2, 0.6):
        e = 1e-4
        u = WL.burgers_cole_hopf(x, t, Re)
        ut = (WL.burgers_cole_hopf(x, t + e, Re) - WL.burgers_cole_hopf(x, t - e, Re)) / (2 * e)
        up = WL.burgers_cole_hopf(x + e, t, Re)
        um = WL.burgers_cole_hopf(x - e, t, Re)
        ux = (up - um) / (2 * e)
        uxx = (up - 2 * u + um) / (e * e)
        scale = np.abs(ut).max() + np.abs(u * ux).max()
        assert np.abs(ut + u * ux - uxx / Re).max() < 1e-4 * scale, t


def _random_system(n=10, seed=5):
    rng = np.random.default_rng(seed)
    rp, cols = [0], []
    for i in range(n):
        nb = rng.choice([j for j in range(n) if j != i], size=4, replace=False)
        cols.extend(sorted(int(j) for j in nb))
        rp.append(len(cols))
    rp = np.array(rp, np.int64)
    col = np.array(cols, np.int32)
    w = [rng.normal(size=col.size) for _ in range(4)]
    return rp, col, w, rng.normal(size=n), rng.normal(size=n)


def _ops(rp, col, w, f):
    n = rp.size - 1
    out = np.zeros(n)
    for i in range(n):
        for e in range(rp[i], rp[i + 1]):
            out[i] += w[e] * (f[col[e]] - f[i])
    return out


def test_burgers_rk4_local_error_is_fifth_order():
    """One RK4 step against solve_ivp (DOP853, rtol 1e-13) on the same right-hand
    side written from eq. (burgers): the local error shrinks ~32x per halving."""
    import oracle as O

    rp, col, w, u0, v0 = _random_system()
    nu = 0.3
    n = u0.size

    def rhs(t, z):
        u, v = z[:n], z[n:]
        du = -(u * _ops(rp, col, w[0], u) + v * _ops(rp, col, w[1], u)) + nu * _ops(rp, col, w[2], u) + _ops(rp, col, w[3], u)
        dv = -(u * _ops(rp, col, w[0], v) + v * _ops(rp, col, w[1], v)) + nu * _ops(rp, col, w[2], v) + _ops(rp, col, w[3], v)
        return np.concatenate([du, dv])

    errs = []
    for dt in (0.02, 0.01, 0.005):
        ref = solve_ivp(rhs, (0, dt), np.concatenate([u0, v0]), method="DOP853", rtol=1e-13, atol=1e-15).y[:, -1]
        u, v = O.burgers_rk4(rp, col, w[0], w[1], w[2], w[3], nu, dt, 1, u0, v0)
        errs.append(np.abs(np.concatenate([u, v]) - ref).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 20 < r1 < 45 and 20 < r2 < 45, errs


def test_constant_fields_are_steady_and_linear_limit():
    import oracle as O

    rp, col, w, u0, v0 = _random_system(seed=6)
    c = np.full(u0.size, 0.7)
    u, v = O.burgers_rk4(rp, col, w[0], w[1], w[2], w[3], 0.2, 0.01, 5, c, -c)
    assert np.array_equal(u, c) and np.array_equal(v, -c)
    zero = np.zeros_like(w[0])
    u, v = O.burgers_rk4(rp, col, zero, zero, w[2], None, 0.2, 0.01, 7, u0, v0)
    assert np.allclose(u, O.rk4(rp, col, 0.2 * w[2], None, 0.0, 0.01, 7, u0), rtol=0, atol=1e-14)
    assert np.allclose(v, O.rk4(rp, col, 0.2 * w[2], None, 0.0, 0.01, 7, v0), rtol=0, atol=1e-14)


def _sawtooth_error(O, k, side):
    cfg = WL.config("burgers")
    x, y, s = WL.jittered_lattice(side, eps=WL.paper_jitter(cfg["eps_paper"]), seed=cfg["seed"], periodic=True)
    dom = WL.unit_domain(True)
    order = np.full(x.size, k, np.int8)
    rp, col, R = O.neighbours(x, y, dom, 2.0 * cfg["h_over_dr"] * s, order, grow=True)
    w, st, _, _ = O.weights(x, y, dom, R, order, rp, col, family=cfg["abf"], rbf=cfg["rbf"], ops=7)
    assert np.all(st == O.ST_OK)
    h = cfg["h_over_dr"] * s
    nsteps = int(math.ceil(cfg["t_end"] / WL.burgers_dt(h, 1.0, cfg["Re"])))
    u, v = O.burgers_rk4(rp, col, w[0], w[1], w[2], None, 1.0 / cfg["Re"], cfg["t_end"] / nsteps, nsteps,
                         np.sin(2 * math.pi * x), np.zeros_like(x))
    assert np.all(v == 0.0)
    ex = WL.burgers_cole_hopf(x, cfg["t_end"], cfg["Re"])
    return np.linalg.norm(u - ex) / np.linalg.norm(ex)


@pytest.mark.parametrize("k,e81", [(4, 1e-2), (6, 3e-3)])
def test_periodic_sawtooth_converges(O, k, e81):
    e41, e81_ = _sawtooth_error(O, k, 41), _sawtooth_error(O, k, 81)
    assert e81_ < e81 and e41 / e81_ > 8.0, (e41, e81_)
