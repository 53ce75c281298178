"""Seeded synthetic inputs: node sets, order maps, test fields.

This module holds none of the method's arithmetic; it only produces inputs
that both the HIP path and the oracle consume.

Node sets follow the paper's noisy Cartesian distribution (Sec. 4.1): a
lattice of spacing s, every node perturbed by at most eps*s.  Here the
lattice is cell-centred ((i + 1/2) s) and each coordinate is perturbed by
U(-eps s, +eps s); nodes are stored in Morton order of their lattice cell
so that neighbours are close in memory.

The noise level eps/dr quoted with the paper's own experiments maps to a
per-coordinate half-width of eps/2 (`paper_jitter`): Sec. 4.1 gives the
separation and fill distances of its eps/dr = 0.5 sets as about 0.29 dr and
0.86 dr, which per-coordinate U(-0.25 dr, 0.25 dr) reproduces (0.26-0.27 dr,
0.89-0.92 dr), while U(-0.5 dr, 0.5 dr) does not (0.02-0.05 dr, 1.1 dr).
"""
import math

import numpy as np

# ---------------------------------------------------------------------------
# node sets


def _morton_key(i, j):
    """Interleave the bits of two non-negative int arrays (i in even bits)."""
    key = np.zeros(np.broadcast(i, j).shape, dtype=np.uint64)
    i = i.astype(np.uint64)
    j = j.astype(np.uint64)
    for b in range(21):
        key |= ((i >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b)
        key |= ((j >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b + 1)
    return key


def jittered_lattice(nx, ny=None, eps=0.3, seed=0, periodic=False, morton=True):
    """Cell-centred nx*ny lattice on [0,1]^2 with per-coordinate jitter U(-eps s, eps s).

    Returns (x, y, s) with x, y float64 of length nx*ny.  On a periodic domain
    coordinates are wrapped into [0, 1)."""
    ny = nx if ny is None else ny
    sx, sy = 1.0 / nx, 1.0 / ny
    rng = np.random.default_rng(seed)
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    ii = ii.ravel()
    jj = jj.ravel()
    jx = rng.uniform(-eps, eps, ii.size)
    jy = rng.uniform(-eps, eps, ii.size)
    x = (ii + 0.5 + jx) * sx
    y = (jj + 0.5 + jy) * sy
    if periodic:
        x = np.mod(x, 1.0)
        y = np.mod(y, 1.0)
    if morton:
        perm = np.argsort(_morton_key(ii, jj), kind="stable")
        x, y = x[perm], y[perm]
    return np.ascontiguousarray(x), np.ascontiguousarray(y), min(sx, sy)


def wall_conforming_lattice(n, eps=0.3, seed=0, morton=True):
    """n*n nodes at (i/(n-1), j/(n-1)); interior nodes jittered in both
    coordinates, wall nodes only along the wall, corners fixed.  Used for the
    one-sided boundary stencil tests (nodes lie on the boundary as in the
    paper's bounded cases)."""
    s = 1.0 / (n - 1)
    rng = np.random.default_rng(seed)
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ii = ii.ravel()
    jj = jj.ravel()
    jx = rng.uniform(-eps, eps, ii.size)
    jy = rng.uniform(-eps, eps, ii.size)
    on_x = (ii == 0) | (ii == n - 1)
    on_y = (jj == 0) | (jj == n - 1)
    jx[on_x] = 0.0
    jy[on_y] = 0.0
    x = (ii + jx) * s
    y = (jj + jy) * s
    if morton:
        perm = np.argsort(_morton_key(ii, jj), kind="stable")
        x, y = x[perm], y[perm]
    return np.ascontiguousarray(x), np.ascontiguousarray(y), s


def paper_jitter(eps_over_dr):
    """Per-coordinate jitter half-width (in units of s) of the paper's noise
    level eps/dr (see the module docstring)."""
    return 0.5 * float(eps_over_dr)


def unit_domain(periodic=False):
    return {"lo": (0.0, 0.0), "hi": (1.0, 1.0), "periodic": (bool(periodic), bool(periodic))}


def order_map(x, y, k, band=0.0, k_boundary=None, periodic=False):
    """Per-node order: k everywhere; min(k, k_boundary) where the distance to
    the nearest wall of [0,1]^2 is below `band` (non-periodic domains)."""
    order = np.full(x.size, k, dtype=np.int8)
    if not periodic and band > 0.0 and k_boundary is not None:
        wall = np.minimum(np.minimum(x, 1.0 - x), np.minimum(y, 1.0 - y))
        order[wall < band] = min(k, k_boundary)
    return order


def interior_mask(x, y, band):
    wall = np.minimum(np.minimum(x, 1.0 - x), np.minimum(y, 1.0 - y))
    return wall >= band


# ---------------------------------------------------------------------------
# workload configurations (sizes and conventions of the measured workloads)

def config(name):
    """Workload parameters.  Radii are in units of the lattice spacing s."""
    cfgs = {
        # 32x32, order 4 everywhere, R0 = 2.85 s (mean N ~ 24), FP64 weights
        "c1": dict(n_side=32, eps=0.3, seed=1, k=4, k_boundary=4, R_s=2.85, periodic=False),
        # 512x512, order 8 interior / order 4 in a boundary band of width R0, R0 = 4.4 s (mean N ~ 60)
        "c2": dict(n_side=512, eps=0.3, seed=2, k=8, k_boundary=4, R_s=4.4, periodic=False),
        # 1024x1024 periodic, order 6, R = 4.0 s (mean N ~ 50), RK4 advection-diffusion with
        # composed nabla^8 hyperviscosity gamma = beta h^8 / dt.  dt = 0.1 s: at 0.2 s the RK4
        # step map of this node set grows (power iteration: x3.7 per step, a mode localised on
        # the stencils of largest amplification); at 0.1 s every mode decays.
        # batch of independent sets (seeds seed0 + s): n_s log-uniform in [n_min, n_max] (side
        # round(sqrt(n_s))), eps_s ~ U(0, eps_max), order k_s uniform over `orders`, R0 = R_s[k] s
        # (mean N about 10, 25, 48, 62) + growth, order min(k, 4) in the boundary band of width R0
        "c3": dict(nsets=64, seed0=3000, n_min=4096, n_max=262144, eps_max=0.4, orders=(2, 4, 6, 8),
                   R_s={2: 1.8, 4: 2.85, 6: 3.9, 8: 4.45}, k_boundary=4),
        # learned warm start, order 8 (p = 44) Hermite x Wendland C2, {dx, dy, lap}: training stencils
        # from periodic jittered lattices of side train_side, eps ~ U(0, eps_max) per lattice (seeds
        # train_seed0 + i), R0 = 4.4 s + growth; the network sees the nearest kmax = 64 neighbours.
        # Evaluation: 1024x1024, eps 0.3, seed 4 (the GPU tests use test_sets lattices and a
        # test_eval_side^2 evaluation set).
        "c4": dict(k=8, R_s=4.4, kmax=64, ops=7, dims=(192, 256, 256, 256, 132), train_side=96,
                   train_seed0=4000, eps_max=0.45, train_sets=218, eval_side=1024, eval_eps=0.3, eval_seed=4,
                   lr=1e-3, batch=512, test_sets=16, test_epochs=10, test_eval_side=96),
        "c5": dict(n_side=1024, eps=0.3, seed=5, k=6, k_boundary=6, R_s=4.0, periodic=True,
                   a=(1.0, 0.5), nu=1e-3, beta=1e-7, dt_s=0.1, nsteps=1000,
                   x0=(0.5, 0.5), width2=0.01),
        # heat equation u_t = kappa lap u, kappa = 1 (Sec. 5.1): quadratic RBF, ABF family
        # PAPER_D1 (= 2), h/dr = 2 (R = 4 dr, growth to the critical counts near walls),
        # eps/dr = 0.5 (paper's measure), dt = 0.05 h^2.  Dirichlet: wall-conforming lattice on
        # [0,1]^2, u = sin(pi x) on y = 0 and 0 on the other walls, steady state taken at
        # t* = 8 pi^2 t = 100; periodic: sin(2 pi x) sin(2 pi y) decaying to t* = 1.
        "heat": dict(abf=2, rbf=2, h_over_dr=2.0, eps_paper=0.5, dt_h2=0.05, tstar_ss=100.0,
                     tstar_periodic=1.0, seed=7, hH=(0.2, 0.1, 0.05, 0.025, 0.0125)),
        # viscous Burgers' equation (Sec. 5.3), periodic unit square: u0 = sin(2 pi x), v0 = 0
        # (Cole-Hopf solution), Re = 100, eps/dr = 0.2, h/dr = 2, quadratic x PAPER_D1,
        # dt = min(0.2 h / max|u|, 0.05 h^2 Re) (eq. tstep), resolutions h/H = 2/n_side;
        # the Re = 250 run adds -100 h^4 nabla^4 hyperviscosity (k = 6, eps/dr = 0.5, h/H = 2/81).
        # Poisson's equation lap phi = f (Sec. 5.2), phi = sin(2 pi x) sin(2 pi y): periodic unit
        # square with node 0 held at the exact value (the periodic problem fixes phi up to a
        # constant), and the unit square with phi = 0 on the walls; quadratic x PAPER_D1,
        # h/dr = 2 (3 for k = 7, 8), eps/dr = 0.5, BiCGStab to ||r|| <= 1e-10 ||F||.
        "poisson": dict(abf=2, rbf=2, eps_paper=0.5, seed=13, tol=1e-10, sides=(20, 40, 80, 160),
                        h_over_dr={2: 2.0, 3: 2.0, 4: 2.0, 5: 2.0, 6: 2.0, 7: 3.0, 8: 3.0}),
        # Taylor-Green vortices (Sec. 5.4), vorticity-streamfunction form on the periodic unit
        # square: omega = 4 pi sin(2 pi x) sin(2 pi y) exp(-8 pi^2 t / Re), Re = 100, quadratic x
        # PAPER_D1, h/dr = 2 and eps/dr = 0.5 (k = 2, 4, 6), dt by eq. (tstep) with max|u| = 1,
        # stream function pinned to 0 at node 0, Poisson tolerance 1e-10.
        "taylor_green": dict(abf=2, rbf=2, Re=100.0, h_over_dr=2.0, eps_paper=0.5, seed=17, tol=1e-10,
                             t_end=0.5, sides=(10, 20, 40, 80)),
        # three dimensions: periodic n^3 lattices, eps 0.3, Hermite (sigma 1.5) x Wendland C2, one
        # order per set, R0 by order for mean N about 14, 29, 51, 82, 111, 165 (k = 1..6; p = 3, 9, 19,
        # 34, 55, 83), no growth
        "c3d": dict(eps=0.3, seed=21, sigma=1.5, R_s={1: 1.5, 2: 1.9, 3: 2.3, 4: 2.7, 5: 3.0, 6: 3.4}, bench_side=64,
                    bench_k=4),
        "burgers": dict(abf=2, rbf=2, h_over_dr=2.0, Re=100.0, eps_paper=0.2, seed=11, t_end=0.4,
                        sides=(21, 41, 81, 161), Re_hv=250.0, hv_coef=100.0, hv_eps_paper=0.5, hv_side=81,
                        wave_ghost=6, wave_seed=13, wave_eps_paper=0.2),
    }
    return dict(cfgs[name])


def make_nodes(cfg, n_side=None, seed=None):
    """Node set + per-node order + initial radius for a config dict."""
    n_side = cfg["n_side"] if n_side is None else n_side
    seed = cfg["seed"] if seed is None else seed
    x, y, s = jittered_lattice(n_side, eps=cfg["eps"], seed=seed, periodic=cfg["periodic"])
    R0 = cfg["R_s"] * s
    order = order_map(x, y, cfg["k"], band=R0, k_boundary=cfg["k_boundary"], periodic=cfg["periodic"])
    R = np.full(x.size, R0)
    return dict(x=x, y=y, s=s, R0=R0, R=R, order=order, domain=unit_domain(cfg["periodic"]))


def batch_sets(cfg, nsets=None, n_min=None, n_max=None):
    """Node sets of the batched workload: list of dicts as make_nodes gives,
    plus the set's order k and jitter eps."""
    nsets = cfg["nsets"] if nsets is None else nsets
    n_min = cfg["n_min"] if n_min is None else n_min
    n_max = cfg["n_max"] if n_max is None else n_max
    out = []
    for t in range(nsets):
        seed = cfg["seed0"] + t
        rng = np.random.default_rng(seed)
        n = math.exp(rng.uniform(math.log(n_min), math.log(n_max)))
        side = max(4, int(round(math.sqrt(n))))
        eps = float(rng.uniform(0.0, cfg["eps_max"]))
        k = int(cfg["orders"][rng.integers(len(cfg["orders"]))])
        x, y, s = jittered_lattice(side, eps=eps, seed=seed, periodic=False)
        R0 = cfg["R_s"][k] * s
        order = order_map(x, y, k, band=R0, k_boundary=min(k, cfg["k_boundary"]), periodic=False)
        out.append(dict(x=x, y=y, s=s, R0=R0, R=np.full(x.size, R0), order=order, domain=unit_domain(False), k=k,
                        eps=eps))
    return out


# ---------------------------------------------------------------------------
# test fields with analytic derivatives (dx, dy, laplacian)

def sincos_field(x, y):
    """f = sin(2 pi x) cos(2 pi y)."""
    tp = 2.0 * math.pi
    f = np.sin(tp * x) * np.cos(tp * y)
    fx = tp * np.cos(tp * x) * np.cos(tp * y)
    fy = -tp * np.sin(tp * x) * np.sin(tp * y)
    lap = -2.0 * tp * tp * f
    return f, fx, fy, lap


def p6_field(x, y):
    """The paper's polynomial test function (Sec. 4.1 eq. p6), H = 1:
    1 + (xh yh)^4 + sum_{n=1..6} (xh^n + yh^n), xh = x - 0.1453, yh = y - 0.16401."""
    xh = x - 0.1453
    yh = y - 0.16401
    f = 1.0 + (xh * yh) ** 4
    fx = 4.0 * xh ** 3 * yh ** 4
    fy = 4.0 * xh ** 4 * yh ** 3
    lap = 12.0 * xh ** 2 * yh ** 4 + 12.0 * xh ** 4 * yh ** 2
    for n in range(1, 7):
        f = f + xh ** n + yh ** n
        fx = fx + n * xh ** (n - 1)
        fy = fy + n * yh ** (n - 1)
        if n >= 2:
            lap = lap + n * (n - 1) * (xh ** (n - 2) + yh ** (n - 2))
    return f, fx, fy, lap


def trig_poly(seed, deg=8):
    """Random trigonometric polynomial of degree <= deg on the unit torus:
    coefficients a, b ~ N(0,1)/(1 + m^2 + n^2) for |m|, |n| <= deg, (m,n) != 0."""
    rng = np.random.default_rng(seed)
    modes = [(m, n) for m in range(-deg, deg + 1) for n in range(-deg, deg + 1) if (m, n) != (0, 0)]
    modes = np.array(modes, dtype=np.float64)
    scale = 1.0 / (1.0 + modes[:, 0] ** 2 + modes[:, 1] ** 2)
    a = rng.standard_normal(len(modes)) * scale
    b = rng.standard_normal(len(modes)) * scale
    return modes, a, b


def trig_field(x, y, poly):
    modes, a, b = poly
    f = np.zeros_like(x)
    fx = np.zeros_like(x)
    fy = np.zeros_like(x)
    lap = np.zeros_like(x)
    tp = 2.0 * math.pi
    for (m, n), am, bm in zip(modes, a, b):
        ph = tp * (m * x + n * y)
        c, s_ = np.cos(ph), np.sin(ph)
        f += am * c + bm * s_
        fx += tp * m * (-am * s_ + bm * c)
        fy += tp * n * (-am * s_ + bm * c)
        lap += -(tp ** 2) * (m * m + n * n) * (am * c + bm * s_)
    return f, fx, fy, lap


def gaussian_pulse(x, y, x0=(0.5, 0.5), width2=0.01, periodic=True):
    """u0 = exp(-|x - x0|^2 / width2), minimum-image distance when periodic."""
    dx = x - x0[0]
    dy = y - x0[1]
    if periodic:
        dx = dx - np.round(dx)
        dy = dy - np.round(dy)
    return np.exp(-(dx * dx + dy * dy) / width2)


def advected_gaussian(x, y, t, a, nu, x0=(0.5, 0.5), width2=0.01, images=2):
    """Free-space solution of u_t + a.grad u = nu lap u from gaussian_pulse,
    summed over periodic images of the unit torus."""
    s2 = width2 + 4.0 * nu * t
    amp = width2 / s2
    cx = x0[0] + a[0] * t
    cy = x0[1] + a[1] * t
    u = np.zeros_like(x)
    for ix in range(-images, images + 1):
        for iy in range(-images, images + 1):
            dx = x - cx - ix
            dy = y - cy - iy
            u += amp * np.exp(-(dx * dx + dy * dy) / s2)
    return u


# ---------------------------------------------------------------------------
# heat equation (Sec. 5.1)


def heat_dirichlet_nodes(hH, eps_over_dr=0.5, seed=7):
    """Wall-conforming lattice with h/H = hH at h/dr = 2 (dr = hH / 2), paper
    noise level eps/dr.  Returns (x, y, s, wall) with wall a bool mask of the
    boundary nodes."""
    n = int(round(2.0 / hH)) + 1
    x, y, s = wall_conforming_lattice(n, eps=paper_jitter(eps_over_dr), seed=seed)
    wall = (x == 0.0) | (x == 1.0) | (y == 0.0) | (y == 1.0)
    return x, y, s, wall


def heat_periodic_nodes(hH, eps_over_dr=0.5, seed=3):
    """Periodic cell-centred lattice with h/H = hH at h/dr = 2."""
    n = int(round(2.0 / hH))
    return jittered_lattice(n, eps=paper_jitter(eps_over_dr), seed=seed, periodic=True)


def heat_boundary_values(x, y):
    """Dirichlet data of the steady-state case: sin(pi x) on y = 0, else 0."""
    return np.where(y == 0.0, np.sin(math.pi * x), 0.0)


def heat_steady_state(x, y):
    """u_ss = sinh(pi (1 - y)) sin(pi x) / sinh(pi) (Sec. 5.1, eq. heatss)."""
    return np.sinh(math.pi * (1.0 - y)) * np.sin(math.pi * x) / math.sinh(math.pi)


def heat_periodic_solution(x, y, t, kappa=1.0):
    """sin(2 pi x) sin(2 pi y) exp(-8 kappa pi^2 t) on the unit torus (Sec. 5.1)."""
    return np.sin(2 * math.pi * x) * np.sin(2 * math.pi * y) * math.exp(-8.0 * kappa * math.pi ** 2 * t)


# ---------------------------------------------------------------------------
# viscous Burgers' equation (Sec. 5.3)


def burgers_cole_hopf(x, t, Re, H=1.0, nterms=30):
    """Exact u(x, t) of u_t + u u_x = u_xx / Re from u(x, 0) = sin(2 pi x / H)
    (Cole-Hopf): with z = Re H / (4 pi), A_0 = e^-z I_0(z), A_n = 2 e^-z I_n(z),
    u = (4 pi / (H Re)) sum n A_n sin(2 n pi x / H) E_n / (A_0 + sum A_n cos(2 n pi x / H) E_n),
    E_n = exp(-4 n^2 pi^2 t / (H^2 Re)).  The printed decay exponent lacks the
    factor 4 that the heat equation behind the transform gives (modes
    cos(2 n pi x / H) decay at (2 n pi / H)^2 / Re); with it the series
    satisfies the equation."""
    from scipy.special import ive

    x = np.asarray(x, dtype=np.float64)
    z = Re * H / (4.0 * math.pi)
    n = np.arange(1, nterms + 1, dtype=np.float64)
    A0 = ive(0, z)
    An = 2.0 * ive(n, z)
    E = np.exp(-4.0 * n ** 2 * math.pi ** 2 * t / (H * H * Re))
    ang = 2.0 * math.pi * np.multiply.outer(x.ravel(), n) / H
    num = (np.sin(ang) * (n * An * E)).sum(axis=1)
    den = A0 + (np.cos(ang) * (An * E)).sum(axis=1)
    return (4.0 * math.pi / (H * Re) * num / den).reshape(x.shape)


def burgers_wave_nodes(M, ghost=6, eps_over_dr=0.2, seed=13, morton=True):
    """Node set of the travelling-wave case (Sec. 5.3): a cell-centred M x M
    lattice on [0,1]^2 (dr = 1/M) continued `ghost` layers outward on every
    side, per-coordinate jitter of the paper's noise level.  Returns
    (x, y, dr, fixed, domain): fixed = 1 on the nodes whose lattice cell lies
    outside the unit square (the analytic solution is prescribed there), and a
    non-periodic domain box that holds every node."""
    dr = 1.0 / M
    n1 = M + 2 * ghost
    rng = np.random.default_rng(seed)
    jj, ii = np.meshgrid(np.arange(n1), np.arange(n1), indexing="ij")
    ii = ii.ravel()
    jj = jj.ravel()
    eps = paper_jitter(eps_over_dr)
    x = (ii - ghost + 0.5 + rng.uniform(-eps, eps, ii.size)) * dr
    y = (jj - ghost + 0.5 + rng.uniform(-eps, eps, ii.size)) * dr
    fixed = ((ii < ghost) | (ii >= ghost + M) | (jj < ghost) | (jj >= ghost + M)).astype(np.int8)
    if morton:
        perm = np.argsort(_morton_key(ii, jj), kind="stable")
        x, y, fixed = x[perm], y[perm], fixed[perm]
    lo = -ghost * dr
    hi = 1.0 + ghost * dr
    dom = {"lo": (lo, lo), "hi": (hi, hi), "periodic": (False, False)}
    return np.ascontiguousarray(x), np.ascontiguousarray(y), dr, np.ascontiguousarray(fixed), dom


def _wave_arg(x, y, t, Re):
    return Re * (-t - 4.0 * np.asarray(x, np.float64) + 4.0 * np.asarray(y, np.float64)) / 32.0


def burgers_wave(x, y, t, Re):
    """Travelling-wave solution of Burgers' equation (Sec. 5.3):
    u = 3/4 - g, v = 3/4 + g with g = 1 / (4 (1 + e^z)), z = Re (-t - 4x + 4y) / 32,
    evaluated as g = (1 - tanh(z/2)) / 8."""
    g = (1.0 - np.tanh(0.5 * _wave_arg(x, y, t, Re))) / 8.0
    return 0.75 - g, 0.75 + g


def burgers_wave_dt(x, y, t, Re):
    """Time derivatives of burgers_wave: dg/dt = (Re / 128) e^z / (1 + e^z)^2,
    so du/dt = -dg/dt and dv/dt = dg/dt (e^z / (1 + e^z)^2 evaluated as
    e^-|z| / (1 + e^-|z|)^2)."""
    e = np.exp(-np.abs(_wave_arg(x, y, t, Re)))
    d = (Re / 128.0) * e / (1.0 + e) ** 2
    return -d, d


def burgers_dt(h, umax, Re):
    """Eq. (tstep): dt = min(0.2 h / max|u|, 0.05 h^2 Re)."""
    return min(0.2 * h / umax, 0.05 * h * h * Re)


# ---------------------------------------------------------------------------
# Poisson's equation (Sec. 5.2)


def poisson_solution(x, y):
    """phi = sin(2 pi x) sin(2 pi y); lap phi = -8 pi^2 phi."""
    return np.sin(2 * math.pi * x) * np.sin(2 * math.pi * y)


def poisson_source(x, y):
    return -8.0 * math.pi ** 2 * poisson_solution(x, y)


def poisson_system(x, y, fixed):
    """Right-hand side F of eq. (poisson_system): f on free rows, the exact
    value on Dirichlet rows; and the initial guess (exact value on Dirichlet
    rows, 0 elsewhere)."""
    phi = poisson_solution(x, y)
    fx = np.asarray(fixed) != 0
    F = np.where(fx, phi, poisson_source(x, y))
    x0 = np.where(fx, phi, 0.0)
    return F, x0


# ---------------------------------------------------------------------------
# Poisson's equation with Neumann walls (Sec. 5.2, eq. neu and the ghost rows)


def neumann_square_nodes(side, eps_over_dr=0.5, seed=13):
    """The unit square with Neumann walls at x = 0 and x = 1 and Dirichlet walls
    at y = 0 and y = 1 (corners Dirichlet): a wall-conforming (side+1)^2 lattice
    (interior nodes jittered at the paper's noise level, wall nodes only along
    their wall), and for every Neumann wall node b a ghost node at
    r_b - n_b dr outside the wall, n_b the inward unit normal.  Returns a dict:
    x, y, s (= dr), kind (0 interior, 1 Dirichlet wall, 2 Neumann wall, 3 ghost),
    parent (int32: the ghost's wall node, -1 elsewhere), nx, ny (at ghost rows:
    the parent's inward normal; 0 elsewhere), domain (the square widened by dr
    in x to hold the ghosts).  Ghosts follow the lattice nodes."""
    x, y, s = wall_conforming_lattice(side + 1, eps=paper_jitter(eps_over_dr), seed=seed)
    n = x.size
    kind = np.zeros(n, np.int8)
    onx = (x == 0.0) | (x == 1.0)
    ony = (y == 0.0) | (y == 1.0)
    kind[ony] = 1
    kind[onx & ~ony] = 2
    walls = np.nonzero(kind == 2)[0]
    nxw = np.where(x[walls] == 0.0, 1.0, -1.0)  # inward normal of each Neumann wall node
    gx = x[walls] - nxw * s
    gy = y[walls].copy()
    m = walls.size
    x = np.concatenate([x, gx])
    y = np.concatenate([y, gy])
    kind = np.concatenate([kind, np.full(m, 3, np.int8)])
    parent = np.concatenate([np.full(n, -1, np.int32), walls.astype(np.int32)])
    nx = np.concatenate([np.zeros(n), nxw])
    ny = np.zeros(n + m)
    dom = {"lo": (-s, 0.0), "hi": (1.0 + s, 1.0), "periodic": (False, False)}
    return dict(x=np.ascontiguousarray(x), y=np.ascontiguousarray(y), s=s, kind=kind, parent=parent,
                nx=nx, ny=ny, domain=dom)


def neumann_field(x, y):
    """phi = sin(2x + 1/2) cos(3y/2 + 1/5) and its gradient and Laplacian
    (-(4 + 9/4) phi): smooth, with non-zero Dirichlet and Neumann data."""
    phi = np.sin(2 * x + 0.5) * np.cos(1.5 * y + 0.2)
    px = 2 * np.cos(2 * x + 0.5) * np.cos(1.5 * y + 0.2)
    py = -1.5 * np.sin(2 * x + 0.5) * np.sin(1.5 * y + 0.2)
    return phi, px, py, -(4.0 + 2.25) * phi


def neumann_poly(k):
    """A polynomial of degree k (k = 2 or 4) with its gradient and Laplacian,
    as callables of (x, y): the discrete operators reproduce it exactly."""
    if k == 2:
        return (lambda x, y: 0.7 + 0.3 * x - 0.4 * y + 0.5 * x * x - 0.2 * x * y + 0.9 * y * y,
                lambda x, y: 0.3 + 1.0 * x - 0.2 * y,
                lambda x, y: -0.4 - 0.2 * x + 1.8 * y,
                lambda x, y: 1.0 + 1.8 + 0.0 * x)
    return (lambda x, y: 0.2 + x - 0.5 * y + 0.3 * x ** 2 * y ** 2 - 0.25 * x ** 4 + 0.6 * x ** 3 * y - 0.1 * y ** 4,
            lambda x, y: 1.0 + 0.6 * x * y ** 2 - x ** 3 + 1.8 * x ** 2 * y,
            lambda x, y: -0.5 + 0.6 * x ** 2 * y + 0.6 * x ** 3 - 0.4 * y ** 3,
            lambda x, y: 0.6 * y ** 2 - 3.0 * x ** 2 + 3.6 * x * y + 0.6 * x ** 2 - 1.2 * y ** 2)


def neumann_system(nodes, phi, grad_x, grad_y, lap):
    """Right-hand side of the enlarged eq. (poisson_system): f at interior and
    Neumann wall rows, the exact value at Dirichlet rows, and at each ghost row
    the parent's normal derivative n_b . grad phi (eq. neu); plus the initial
    guess (exact value on Dirichlet rows, 0 elsewhere) and the Dirichlet mask."""
    x, y, kind, parent = nodes["x"], nodes["y"], nodes["kind"], nodes["parent"]
    F = lap(x, y).astype(np.float64) * np.ones_like(x)
    d = kind == 1
    F[d] = phi(x[d], y[d])
    g = np.nonzero(kind == 3)[0]
    p = parent[g]
    F[g] = nodes["nx"][g] * grad_x(x[p], y[p]) + nodes["ny"][g] * grad_y(x[p], y[p])
    x0 = np.where(d, phi(x, y), 0.0)
    return F, x0, d.astype(np.int8)


# ---------------------------------------------------------------------------
# Taylor-Green vortices (Sec. 5.4)


def taylor_green_vorticity(x, y, t, Re, H=1.0):
    """omega = (4 pi / H) sin(2 pi x / H) sin(2 pi y / H) exp(-8 pi^2 t / (Re H^2))."""
    return (4.0 * math.pi / H) * np.sin(2 * math.pi * x / H) * np.sin(2 * math.pi * y / H) * \
        math.exp(-8.0 * math.pi ** 2 * t / (Re * H * H))


# ---------------------------------------------------------------------------
# three dimensions


def jittered_lattice3(n, eps=0.3, seed=0, periodic=True, morton=True):
    """Cell-centred n^3 lattice on [0,1]^3, per-coordinate jitter U(-eps s, eps s),
    nodes in Morton order of their cell.  Returns (x, y, z, s)."""
    s = 1.0 / n
    rng = np.random.default_rng(seed)
    kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()
    x = (ii + 0.5 + rng.uniform(-eps, eps, ii.size)) * s
    y = (jj + 0.5 + rng.uniform(-eps, eps, ii.size)) * s
    z = (kk + 0.5 + rng.uniform(-eps, eps, ii.size)) * s
    if periodic:
        x, y, z = np.mod(x, 1.0), np.mod(y, 1.0), np.mod(z, 1.0)
    if morton:
        key = np.zeros(ii.size, dtype=np.uint64)
        for b in range(21):
            for a, sh in ((ii, 0), (jj, 1), (kk, 2)):
                key |= ((a.astype(np.uint64) >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + sh)
        perm = np.argsort(key, kind="stable")
        x, y, z = x[perm], y[perm], z[perm]
    return np.ascontiguousarray(x), np.ascontiguousarray(y), np.ascontiguousarray(z), s


def unit_domain3(periodic=True):
    return {"lo": (0.0, 0.0, 0.0), "hi": (1.0, 1.0, 1.0), "periodic": (bool(periodic),) * 3}


def trig_field3(x, y, z):
    """f = sin(2 pi x) cos(2 pi y) sin(2 pi z + 1) and its x, y, z derivatives and Laplacian."""
    tp = 2 * math.pi
    sx, cx = np.sin(tp * x), np.cos(tp * x)
    sy, cy = np.sin(tp * y), np.cos(tp * y)
    sz, cz = np.sin(tp * z + 1.0), np.cos(tp * z + 1.0)
    f = sx * cy * sz
    return f, tp * cx * cy * sz, -tp * sx * sy * sz, tp * sx * cy * cz, -3 * tp * tp * f
