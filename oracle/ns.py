"""Oracle of the vorticity-streamfunction Navier-Stokes scheme (Sec. 5.4) --
test infrastructure only (tests, the smoke check and the benchmark's CPU
baseline use it; the library never does).

    d omega/dt = -(u d/dx + v d/dy) omega + nu lap omega,   nu = 1/Re,
    lap psi = -omega,   u = d psi/dy,   v = -d psi/dx,

every derivative by the local operators of eq. (general_do).  Classical RK4
(Sec. 5.1); at every stage the stream function comes from the global
Laplacian (eq. poisson_system) solved exactly (scipy's sparse LU), with the
nodes marked in `fixed` held at psi = 0 (the periodic problem fixes psi up to
a constant), and the velocity from its stencil derivatives.
"""
import numpy as np
import scipy.sparse.linalg as spl

import oracle as O
from oracle import poisson as P


def vorticity_rk4(row_ptr, col, wx, wy, wl, nu, dt, nsteps, omega0, fixed):
    """Returns (omega, psi) after nsteps steps."""
    A = P.laplacian_matrix(row_ptr, col, wl, fixed)
    lu = spl.splu(A.tocsc())
    fx = np.asarray(fixed) != 0

    def rhs(om):
        F = np.where(fx, 0.0, -om)
        psi = lu.solve(F)
        u = O.apply(row_ptr, col, wy, psi)
        v = -O.apply(row_ptr, col, wx, psi)
        k = -(u * O.apply(row_ptr, col, wx, om) + v * O.apply(row_ptr, col, wy, om)) + nu * O.apply(row_ptr, col, wl, om)
        return k, psi

    om = np.array(omega0, dtype=np.float64, copy=True)
    psi = np.zeros_like(om)
    for _ in range(nsteps):
        k1, psi = rhs(om)
        k2, _ = rhs(om + 0.5 * dt * k1)
        k3, _ = rhs(om + 0.5 * dt * k2)
        k4, _ = rhs(om + dt * k3)
        om = om + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return om, psi
