"""Plain FP64 CPU oracle for the LABFM hot path (ctypes wrapper over labfm_oracle.c).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library, and the library never imports it.

Method: King, Lind & Nasar, arXiv:1912.06441 -- Sec. 2 (operator, eq. general_do),
Sec. 3.1 (moment system, eqs. w_abf / disc_form / lsys), Sec. 3.2 and App. A
(ABFs), Sec. 4.2 (hyperviscosity targets), Sec. 5.1 (RK4).
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

ABF_HERMITE, ABF_PAPER, ABF_PAPER_D1 = 0, 1, 2
RBF_WENDLAND_C2, RBF_CONE, RBF_QUADRATIC, RBF_WENDLAND_C6, RBF_GAUSSIAN = 0, 1, 2, 3, 4
OP_DX, OP_DY, OP_LAP, OP_BIHARM, OP_TRIHARM = 1, 2, 4, 8, 16
OP_DZ = 32  # three dimensions only
ST_OK, ST_NOT_CONVERGED, ST_SINGULAR, ST_TOO_FEW, ST_DEGENERATE, ST_ORDER_TOO_LOW, ST_TOO_MANY = range(7)
NMAX = 128  # longest stencil row the weights accept (implementation limit; longer: ST_TOO_MANY)
NMAX3 = 256  # three dimensions (orders 5 and 6 need well over 100 neighbours)
MAXK = 8
MAXK3 = 6  # highest three-dimensional order


class _Domain(C.Structure):
    _fields_ = [("lo", C.c_double * 2), ("hi", C.c_double * 2), ("periodic", C.c_int * 2)]


class _Domain3(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3), ("periodic", C.c_int * 3)]


class _WOpts(C.Structure):
    _fields_ = [("family", C.c_int), ("rbf", C.c_int), ("sigma", C.c_double),
                ("ops", C.c_uint), ("tol_stop", C.c_double), ("max_iters", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        i8 = C.POINTER(C.c_int8)
        i32 = C.POINTER(C.c_int32)
        i64 = C.POINTER(C.c_int64)
        L.or_p_of_k.argtypes = [C.c_int]
        L.or_ncrit.argtypes = [C.c_int]
        L.or_index_table.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.or_monomials.argtypes = [C.c_int, C.c_double, C.c_double, dp]
        L.or_abfs.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_double, C.c_double, dp]
        L.or_rbf_derivs.argtypes = [C.c_int, C.c_double, dp]
        L.or_hermite.argtypes = [C.c_int, C.c_double, dp]
        for fn in (L.or_neighbours_brute, L.or_neighbours_cells):
            fn.argtypes = [C.c_int64, dp, dp, C.POINTER(_Domain), dp, i8, C.c_int, C.c_int, i64, i32]
            fn.restype = C.c_int64
        L.or_node_weights.argtypes = [C.c_int, C.c_int, dp, dp, C.POINTER(_WOpts), dp, dp,
                                      C.POINTER(C.c_int), dp, dp]
        L.or_weights.argtypes = [C.c_int64, dp, dp, C.POINTER(_Domain), dp, i8, i64, i32,
                                 C.POINTER(_WOpts), dp, i8, dp, i8]
        L.or_targets.argtypes = [C.c_uint, C.c_int, dp]
        L.or_p3_of_k.argtypes = [C.c_int]
        L.or_index_table3.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.or_monomials3.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, dp]
        L.or_abfs3.argtypes = [C.c_int, C.c_double, C.c_int, C.c_double, C.c_double, C.c_double, dp]
        L.or_neighbours3_brute.argtypes = [C.c_int64, dp, dp, dp, C.POINTER(_Domain3), dp, i64, i32]
        L.or_neighbours3_brute.restype = C.c_int64
        L.or_weights3.argtypes = [C.c_int64, dp, dp, dp, C.POINTER(_Domain3), dp, C.c_int, i64, i32,
                                  C.POINTER(_WOpts), dp, i8, dp, i8]
        L.or_stencils_psi.argtypes = [C.c_int64, C.c_int, C.c_int, i32, dp, dp, C.POINTER(_WOpts), dp, i8, dp, dp]
        L.or_stencils_psi.restype = None
        L.or_apply.argtypes = [C.c_int64, i64, i32, dp, dp, dp]
        L.or_combine.argtypes = [C.c_int64, C.c_int, dp, dp, dp]
        L.or_rk4.argtypes = [C.c_int64, i64, i32, dp, dp, C.c_double, C.c_double, C.c_int, dp, i8]
        L.or_burgers_rk4.argtypes = [C.c_int64, i64, i32, dp, dp, dp, dp, C.c_double, C.c_double, C.c_int, dp, dp,
                                     i8, dp]
        L.or_num_threads.restype = C.c_int
        L.or_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _dom(domain):
    d = _Domain()
    d.lo[0], d.lo[1] = domain["lo"]
    d.hi[0], d.hi[1] = domain["hi"]
    d.periodic[0], d.periodic[1] = [int(v) for v in domain["periodic"]]
    return d


def nops(ops):
    return bin(int(ops) & 31).count("1")


def p_of_k(k):
    return lib().or_p_of_k(int(k))


def ncrit(k):
    return lib().or_ncrit(int(k))


def index_table(k):
    p = p_of_k(k)
    ea = (C.c_int * p)()
    eb = (C.c_int * p)()
    lib().or_index_table(int(k), ea, eb)
    return list(zip(list(ea), list(eb)))


def monomials(k, dx, dy):
    X = np.zeros(p_of_k(k))
    lib().or_monomials(int(k), float(dx), float(dy), _p(X, C.c_double))
    return X


def abfs(k, dx, dy, family=ABF_HERMITE, rbf=RBF_WENDLAND_C2, sigma=1.0):
    W = np.zeros(p_of_k(k))
    rc = lib().or_abfs(int(family), int(rbf), float(sigma), int(k), float(dx), float(dy), _p(W, C.c_double))
    if rc != 0:
        raise ValueError("ABFs undefined at this offset (rc=%d)" % rc)
    return W


def rbf_derivs(rbf, q):
    f = np.zeros(4)
    lib().or_rbf_derivs(int(rbf), float(q), _p(f, C.c_double))
    return f


def hermite(nmax, t):
    H = np.zeros(nmax + 1)
    lib().or_hermite(int(nmax), float(t), _p(H, C.c_double))
    return H


def neighbours(x, y, domain, R, order, grow=True, max_grow=10, method="cells"):
    """Neighbour lists (CSR, ascending j).  Returns (row_ptr, col, R_grown)."""
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    n = x.size
    R = np.array(np.broadcast_to(np.asarray(R, np.float64), (n,)), dtype=np.float64)
    order = np.ascontiguousarray(np.broadcast_to(np.asarray(order, np.int8), (n,)), np.int8)
    rp = np.zeros(n + 1, np.int64)
    d = _dom(domain)
    fn = lib().or_neighbours_cells if method == "cells" else lib().or_neighbours_brute
    nnz = fn(n, _p(x, C.c_double), _p(y, C.c_double), C.byref(d), _p(R, C.c_double), _p(order, C.c_int8),
             int(bool(grow)), int(max_grow), _p(rp, C.c_int64), None)
    col = np.zeros(max(nnz, 1), np.int32)
    fn(n, _p(x, C.c_double), _p(y, C.c_double), C.byref(d), _p(R, C.c_double), _p(order, C.c_int8),
       0, 0, _p(rp, C.c_int64), _p(col, C.c_int32))
    return rp, col[:nnz], R


def wopts(family=ABF_HERMITE, rbf=RBF_WENDLAND_C2, sigma=1.0, ops=OP_DX | OP_DY | OP_LAP,
          tol_stop=1e-13, max_iters=5):
    return _WOpts(int(family), int(rbf), float(sigma), int(ops), float(tol_stop), int(max_iters))


def node_weights(k, dxh, dyh, **kw):
    """Scaled weights for one node from its scaled offsets.

    Returns dict(what [nops, N], status, resid, iters, M [p, p], cond1)."""
    o = wopts(**kw)
    dxh = np.ascontiguousarray(dxh, np.float64)
    dyh = np.ascontiguousarray(dyh, np.float64)
    N = dxh.size
    p = p_of_k(k)
    what = np.zeros((nops(o.ops), max(N, 1)))
    res = C.c_double()
    it = C.c_int()
    M = np.zeros((p, p))
    cond = C.c_double()
    st = lib().or_node_weights(int(k), N, _p(dxh, C.c_double), _p(dyh, C.c_double), C.byref(o),
                               _p(what, C.c_double), C.byref(res), C.byref(it), _p(M, C.c_double),
                               C.byref(cond))
    return dict(what=what[:, :N], status=st, resid=res.value, iters=it.value, M=M, cond1=cond.value)


def targets(ops, k):
    """Target vectors C^d (Sec. 2, Sec. 4.2) of the operators in `ops`, [nops, p]."""
    C_ = np.zeros((nops(ops), p_of_k(k)))
    if lib().or_targets(int(ops), int(k), _p(C_, C.c_double)) != 0:
        raise ValueError("order %d cannot express the requested operators" % k)
    return C_


def stencils_psi(k, dxh, dyh, N, want_M=False, **kw):
    """ABF coefficients Psi^d (eq. lsys, refined) of a batch of stencils.

    dxh, dyh: [n, Nmax] scaled offsets (rows padded beyond N[s]); N: [n].
    Returns (psi [n, nops, p], status [n], resid [n]) and, with want_M, the
    moment matrices [n, p, p] (row = monomial) as a fourth element."""
    o = wopts(**kw)
    dxh = np.ascontiguousarray(dxh, np.float64)
    dyh = np.ascontiguousarray(dyh, np.float64)
    n, Nmax = dxh.shape
    N = np.ascontiguousarray(N, np.int32)
    p = p_of_k(k)
    psi = np.zeros((n, nops(o.ops), p))
    st = np.zeros(n, np.int8)
    res = np.zeros(n)
    M = np.zeros((n, p, p)) if want_M else None
    lib().or_stencils_psi(n, int(k), int(Nmax), _p(N, C.c_int32), _p(dxh, C.c_double), _p(dyh, C.c_double),
                          C.byref(o), _p(psi, C.c_double), _p(st, C.c_int8), _p(res, C.c_double),
                          _p(M, C.c_double) if want_M else None)
    return (psi, st, res, M) if want_M else (psi, st, res)


def weights(x, y, domain, R, order, row_ptr, col, **kw):
    """Weights [nops, nnz] (physical units), status[n], resid[n], iters[n]."""
    o = wopts(**kw)
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    n = x.size
    R = np.ascontiguousarray(np.broadcast_to(np.asarray(R, np.float64), (n,)), np.float64)
    order = np.ascontiguousarray(np.broadcast_to(np.asarray(order, np.int8), (n,)), np.int8)
    row_ptr = np.ascontiguousarray(row_ptr, np.int64)
    col = np.ascontiguousarray(col, np.int32)
    nnz = int(row_ptr[-1])
    w = np.zeros((nops(o.ops), max(nnz, 1)))
    st = np.zeros(n, np.int8)
    res = np.zeros(n)
    its = np.zeros(n, np.int8)
    d = _dom(domain)
    lib().or_weights(n, _p(x, C.c_double), _p(y, C.c_double), C.byref(d), _p(R, C.c_double),
                     _p(order, C.c_int8), _p(row_ptr, C.c_int64), _p(col, C.c_int32), C.byref(o),
                     _p(w, C.c_double), _p(st, C.c_int8), _p(res, C.c_double), _p(its, C.c_int8))
    return w[:, :nnz], st, res, its


def apply(row_ptr, col, w, u):
    row_ptr = np.ascontiguousarray(row_ptr, np.int64)
    col = np.ascontiguousarray(col, np.int32)
    w = np.ascontiguousarray(w, np.float64)
    u = np.ascontiguousarray(u, np.float64)
    n = row_ptr.size - 1
    out = np.zeros(n)
    lib().or_apply(n, _p(row_ptr, C.c_int64), _p(col, C.c_int32), _p(w, C.c_double), _p(u, C.c_double),
                   _p(out, C.c_double))
    return out


def combine(w, coef):
    w = np.ascontiguousarray(w, np.float64)
    coef = np.ascontiguousarray(coef, np.float64)
    nsets, nnz = w.shape
    out = np.zeros(nnz)
    lib().or_combine(nnz, nsets, _p(w, C.c_double), _p(coef, C.c_double), _p(out, C.c_double))
    return out


def rk4(row_ptr, col, w_lin, w_bh, gamma, dt, nsteps, u0, fixed=None):
    """Classical RK4 on du/dt = L_lin u - gamma B(B u); nodes with fixed != 0
    keep their value (Dirichlet)."""
    row_ptr = np.ascontiguousarray(row_ptr, np.int64)
    col = np.ascontiguousarray(col, np.int32)
    w_lin = np.ascontiguousarray(w_lin, np.float64)
    u = np.array(u0, dtype=np.float64, copy=True)
    wb = None
    if w_bh is not None:
        w_bh = np.ascontiguousarray(w_bh, np.float64)
        wb = _p(w_bh, C.c_double)
    fx = None
    if fixed is not None:
        fixed = np.ascontiguousarray(fixed, np.int8)
        fx = _p(fixed, C.c_int8)
    n = row_ptr.size - 1
    lib().or_rk4(n, _p(row_ptr, C.c_int64), _p(col, C.c_int32), _p(w_lin, C.c_double), wb,
                 float(gamma), float(dt), int(nsteps), _p(u, C.c_double), fx)
    return u


def burgers_rk4(row_ptr, col, wx, wy, wl, whv, nu, dt, nsteps, u0, v0, fixed=None, boundary=None, t0=0.0):
    """Classical RK4 on the viscous Burgers' equation (Sec. 5.3):
    du/dt = -(u d/dx + v d/dy) u + nu lap u + L_hv u, the same for v; returns (u, v).

    Nodes with fixed != 0 hold their values, or, with boundary(t) -> (du/dt,
    dv/dt) (arrays over all nodes), follow those derivatives: stage q of the
    step from t takes them at t + c_q dt, c = (0, 1/2, 1/2, 1)."""
    row_ptr = np.ascontiguousarray(row_ptr, np.int64)
    col = np.ascontiguousarray(col, np.int32)
    ws = [np.ascontiguousarray(a, np.float64) for a in (wx, wy, wl)]
    hv = None if whv is None else np.ascontiguousarray(whv, np.float64)
    u = np.array(u0, dtype=np.float64, copy=True)
    v = np.array(v0, dtype=np.float64, copy=True)
    fx = None
    if fixed is not None:
        fixed = np.ascontiguousarray(fixed, np.int8)
        fx = _p(fixed, C.c_int8)
    n = row_ptr.size - 1
    args = (n, _p(row_ptr, C.c_int64), _p(col, C.c_int32), _p(ws[0], C.c_double), _p(ws[1], C.c_double),
            _p(ws[2], C.c_double), None if hv is None else _p(hv, C.c_double), float(nu), float(dt))
    if boundary is None:
        lib().or_burgers_rk4(*args, int(nsteps), _p(u, C.c_double), _p(v, C.c_double), fx, None)
        return u, v
    if fixed is None:
        raise ValueError("burgers_rk4: boundary derivatives need a fixed mask")
    dfix = np.zeros((2, 4, n), np.float64)
    for s in range(int(nsteps)):
        t = t0 + s * dt
        for q, c in enumerate((0.0, 0.5, 0.5, 1.0)):
            du, dv = boundary(t + c * dt)
            dfix[0, q] = du
            dfix[1, q] = dv
        lib().or_burgers_rk4(*args, 1, _p(u, C.c_double), _p(v, C.c_double), fx, _p(dfix, C.c_double))
    return u, v


def num_threads():
    return lib().or_num_threads()


def set_num_threads(t):
    lib().or_set_num_threads(int(t))


# ---------------------------------------------------------------------------
# three dimensions (HERMITE family)


def p3_of_k(k):
    return lib().or_p3_of_k(int(k))


def index_table3(k):
    p = p3_of_k(k)
    ea, eb, ec = (C.c_int * p)(), (C.c_int * p)(), (C.c_int * p)()
    lib().or_index_table3(int(k), ea, eb, ec)
    return list(zip(list(ea), list(eb), list(ec)))


def monomials3(k, dx, dy, dz):
    X = np.zeros(p3_of_k(k))
    lib().or_monomials3(int(k), float(dx), float(dy), float(dz), _p(X, C.c_double))
    return X


def abfs3(k, dx, dy, dz, rbf=RBF_WENDLAND_C2, sigma=1.0):
    W = np.zeros(p3_of_k(k))
    lib().or_abfs3(int(rbf), float(sigma), int(k), float(dx), float(dy), float(dz), _p(W, C.c_double))
    return W


def _dom3(domain):
    d = _Domain3()
    for a in range(3):
        d.lo[a] = float(domain["lo"][a])
        d.hi[a] = float(domain["hi"][a])
        d.periodic[a] = int(bool(domain["periodic"][a]))
    return d


def neighbours3(x, y, z, domain, R):
    """3-D neighbour lists by brute force (CSR, ascending j): (row_ptr, col)."""
    xs = [np.ascontiguousarray(a, np.float64) for a in (x, y, z)]
    n = xs[0].size
    R = np.ascontiguousarray(np.broadcast_to(np.asarray(R, np.float64), (n,)), np.float64)
    d = _dom3(domain)
    rp = np.zeros(n + 1, np.int64)
    ptrs = [_p(a, C.c_double) for a in xs]
    lib().or_neighbours3_brute(n, *ptrs, C.byref(d), _p(R, C.c_double), _p(rp, C.c_int64), None)
    col = np.zeros(max(int(rp[-1]), 1), np.int32)
    lib().or_neighbours3_brute(n, *ptrs, C.byref(d), _p(R, C.c_double), _p(rp, C.c_int64), _p(col, C.c_int32))
    return rp, col[:int(rp[-1])]


def weights3(x, y, z, domain, R, k, row_ptr, col, ops=OP_DX | OP_DY | OP_DZ | OP_LAP, rbf=RBF_WENDLAND_C2,
             sigma=1.0, tol_stop=1e-13, max_iters=5):
    """3-D weights [nops, nnz] (operators in bit order: dx, dy, lap, dz), status, resid, iters."""
    o = _WOpts(ABF_HERMITE, int(rbf), float(sigma), int(ops), float(tol_stop), int(max_iters))
    xs = [np.ascontiguousarray(a, np.float64) for a in (x, y, z)]
    n = xs[0].size
    R = np.ascontiguousarray(np.broadcast_to(np.asarray(R, np.float64), (n,)), np.float64)
    row_ptr = np.ascontiguousarray(row_ptr, np.int64)
    col = np.ascontiguousarray(col, np.int32)
    nnz = int(row_ptr[-1])
    nop = bin(int(ops) & 63).count("1")
    w = np.zeros((nop, max(nnz, 1)))
    st = np.zeros(n, np.int8)
    res = np.zeros(n)
    its = np.zeros(n, np.int8)
    d = _dom3(domain)
    lib().or_weights3(n, *[_p(a, C.c_double) for a in xs], C.byref(d), _p(R, C.c_double), int(k),
                      _p(row_ptr, C.c_int64), _p(col, C.c_int32), C.byref(o), _p(w, C.c_double),
                      _p(st, C.c_int8), _p(res, C.c_double), _p(its, C.c_int8))
    return w[:, :nnz], st, res, its
