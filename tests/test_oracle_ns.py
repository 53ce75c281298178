"""Pins of the oracle's vorticity-streamfunction Navier-Stokes scheme (Sec. 5.4).

* Taylor-Green vortices (the paper's case): the vorticity decays as
  exp(-8 pi^2 t / Re) and the error falls as h^k (k = 2, 4).
* The Taylor-Green velocity is orthogonal to the vorticity gradient, so it
  cannot see the sign of u or v; a two-mode field, whose advection term is
  not zero, checks the right-hand side against its closed form (the stream
  function, velocity, advection and diffusion of the field written out).
"""
import math

import numpy as np
import pytest

from paper_1912_06441_amd import workloads as WL


def _set(O, k, side, seed=None):
    cfg = WL.config("taylor_green")
    seed = cfg["seed"] if seed is None else seed
    x, y, s = WL.jittered_lattice(side, eps=WL.paper_jitter(cfg["eps_paper"]), seed=seed, periodic=True)
    dom = WL.unit_domain(True)
    order = np.full(x.size, k, np.int8)
    rp, col, R = O.neighbours(x, y, dom, 2.0 * cfg["h_over_dr"] * s, order, grow=True)
    w, st, _, _ = O.weights(x, y, dom, R, order, rp, col, family=cfg["abf"], rbf=cfg["rbf"], ops=7)
    assert np.all(st == O.ST_OK)
    fixed = np.zeros(x.size, np.int8)
    fixed[0] = 1
    return dict(x=x, y=y, h=cfg["h_over_dr"] * s, rp=rp, col=col, w=w, fixed=fixed)


@pytest.mark.parametrize("k,rate", [(2, 2.0), (4, 4.0)])
def test_taylor_green_decay_orders(O, k, rate):
    from oracle import ns as NS

    cfg = WL.config("taylor_green")
    Re, t_end = cfg["Re"], cfg["t_end"]
    errs = []
    for side in cfg["sides"][:3]:
        S = _set(O, k, side)
        nsteps = int(math.ceil(t_end / WL.burgers_dt(S["h"], 1.0, Re)))
        om0 = WL.taylor_green_vorticity(S["x"], S["y"], 0.0, Re)
        om, _ = NS.vorticity_rk4(S["rp"], S["col"], S["w"][0], S["w"][1], S["w"][2], 1.0 / Re, t_end / nsteps, nsteps,
                                 om0, S["fixed"])
        ex = WL.taylor_green_vorticity(S["x"], S["y"], t_end, Re)
        errs.append(np.linalg.norm(om - ex) / np.linalg.norm(ex))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(rates) >= rate - 0.3, (errs, rates)


def test_two_mode_right_hand_side_closed_form(O):
    """omega = sin(2 pi x) sin(2 pi y) + cos(4 pi x) / 2:
    psi = sin sin / (8 pi^2) + cos(4 pi x) / (32 pi^2), u = psi_y, v = -psi_x,
    rhs = -(u omega_x + v omega_y) + nu lap omega.  One RK4 step of size dt
    from omega_0 gives (omega_1 - omega_0) / dt = rhs + O(dt); the order-6
    operators on a 64^2 set leave the spatial error far below the term."""
    from oracle import ns as NS

    S = _set(O, 6, 64, seed=3)
    x, y = S["x"], S["y"]
    tp = 2 * math.pi
    om0 = np.sin(tp * x) * np.sin(tp * y) + 0.5 * np.cos(2 * tp * x)
    u = np.sin(tp * x) * np.cos(tp * y) * tp / (8 * math.pi ** 2)
    v = -(np.cos(tp * x) * np.sin(tp * y) * tp / (8 * math.pi ** 2) - np.sin(2 * tp * x) * 2 * tp / (32 * math.pi ** 2))
    omx = tp * np.cos(tp * x) * np.sin(tp * y) - 2 * tp * 0.5 * np.sin(2 * tp * x)
    omy = tp * np.sin(tp * x) * np.cos(tp * y)
    lap = -2 * tp ** 2 * np.sin(tp * x) * np.sin(tp * y) - 0.5 * (2 * tp) ** 2 * np.cos(2 * tp * x)
    nu = 0.01
    rhs = -(u * omx + v * omy) + nu * lap
    adv = np.abs(u * omx + v * omy).max()
    assert adv > 0.1  # the advection term is not zero for this field
    dt = 1e-6
    om1, _ = NS.vorticity_rk4(S["rp"], S["col"], S["w"][0], S["w"][1], S["w"][2], nu, dt, 1, om0, S["fixed"])
    got = (om1 - om0) / dt
    assert np.abs(got - rhs).max() < 1e-3 * np.abs(rhs).max(), np.abs(got - rhs).max()
