"""Training and evaluation stencils for the warm-start network, from the oracle.

Node sets come from the seeded generators of paper_1912_06441_amd.workloads;
neighbour lists, radii, moment matrices and ABF coefficients all come from
the oracle, so no training target is produced by the HIP path.
"""
import numpy as np

import oracle as O
from oracle import mlp as OM
from paper_1912_06441_amd import workloads as WL


def lattice_stencils(n_side, eps, seed, k, R_s, periodic=True):
    """One jittered lattice: positions, oracle radii and CSR."""
    x, y, s = WL.jittered_lattice(n_side, eps=eps, seed=seed, periodic=periodic)
    dom = WL.unit_domain(periodic)
    order = np.full(x.size, k, np.int8)
    rp, col, R = O.neighbours(x, y, dom, R_s * s, order, grow=True)
    return dict(x=x, y=y, R=R, rp=rp, col=col, order=order, domain=dom, s=s)


def padded_offsets(L):
    """Scaled offsets [n, Nmax] and row lengths of a lattice dict."""
    dxa, dya = OM.stencil_offsets(L["x"], L["y"], L["domain"], L["R"], L["rp"], L["col"])
    N = np.diff(L["rp"]).astype(np.int32)
    n, Nmax = N.size, int(N.max())
    pos = np.arange(L["rp"][-1]) - np.repeat(L["rp"][:-1], N)
    rows = np.repeat(np.arange(n), N)
    dx = np.zeros((n, Nmax))
    dy = np.zeros((n, Nmax))
    dx[rows, pos] = dxa
    dy[rows, pos] = dya
    return dx, dy, N


def targets(L, k, ops):
    """Oracle Psi [n, nops*p], moment matrices [n, p, p], status [n]."""
    dx, dy, N = padded_offsets(L)
    psi, st, res, M = O.stencils_psi(k, dx, dy, N, want_M=True, ops=ops)
    return psi.reshape(psi.shape[0], -1), M, st


def robust_scaling(psi):
    """Per-component median and 1.4826 * median absolute deviation."""
    mu = np.median(psi, axis=0)
    sd = 1.4826 * np.median(np.abs(psi - mu), axis=0)
    return mu, np.where(sd > 0, sd, 1.0)
