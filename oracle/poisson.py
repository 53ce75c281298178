"""Oracle of the global Poisson solve (Sec. 5.2) -- test infrastructure only.

Only tests, the smoke check and the benchmark's CPU baseline use this module;
the library never does.

* `laplacian_matrix`: the global matrix A^L of eq. (poisson_system): row i
  holds the local weights w^L_ij at columns j and -sum_j w^L_ij on the
  diagonal; Dirichlet rows b (fixed[b] != 0) become identity rows
  (A_bb = 1, A_bj = 0), whose right-hand side is the boundary value.
* `neumann_matrix`: the same system enlarged by one ghost row per Neumann
  boundary node (Sec. 5.2, eq. neu): the ghost's row is its parent's discrete
  normal derivative, n_x w^x + n_y w^y in difference form.
* `bicgstab`: the stabilised bi-conjugate gradient method with a Jacobi
  (diagonal) preconditioner applied on the right, in the usual order of van
  der Vorst (1992): rho = (r0, r), beta = (rho/rho_old)(alpha/omega),
  p = r + beta (p - omega v), y = D^-1 p, v = A y, alpha = rho/(r0, v),
  s = r - alpha v, z = D^-1 s, t = A z, omega = (t, s)/(t, t),
  x += alpha y + omega z, r = s - omega t; stop when ||r|| <= tol ||b||.
"""
import numpy as np
import scipy.sparse as sps


def laplacian_matrix(row_ptr, col, w, fixed=None):
    n = row_ptr.size - 1
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    w = np.asarray(w, np.float64).copy()
    diag = -np.add.reduceat(w, row_ptr[:-1]) if w.size else np.zeros(n)
    diag[np.diff(row_ptr) == 0] = 0.0  # reduceat of an empty row repeats the next value
    if fixed is not None:
        fx = np.asarray(fixed) != 0
        w[fx[rows]] = 0.0
        diag[fx] = 1.0
    A = sps.csr_matrix((w, (rows, np.asarray(col, np.int64))), shape=(n, n)) + sps.diags(diag)
    return A.tocsr()


def neumann_matrix(row_ptr, col, w_x, w_y, w_lap, parent, nx, ny, fixed=None):
    """The enlarged global matrix of eq. (poisson_system) with the ghost rows of
    Sec. 5.2: row i with parent[i] < 0 is node i's Laplacian row (identity where
    fixed[i] != 0); ghost row g with parent p = parent[g] enforces eq. (neu) at
    p, A_gj = n_x w^x_pj + n_y w^y_pj for j in p's stencil and
    A_gp = -sum_j (n_x w^x_pj + n_y w^y_pj), with (n_x, n_y) = (nx[g], ny[g])
    the inward unit normal at p.  Row structure and weights come from the
    neighbour sets and local weights of every node, ghosts included."""
    n = row_ptr.size - 1
    A = laplacian_matrix(row_ptr, col, w_lap, fixed).tolil()
    for g in np.nonzero(np.asarray(parent) >= 0)[0]:
        p = int(parent[g])
        A.rows[g] = []
        A.data[g] = []
        acc = {}
        total = 0.0
        for q in range(row_ptr[p], row_ptr[p + 1]):
            wn = nx[g] * w_x[q] + ny[g] * w_y[q]
            j = int(col[q])
            acc[j] = acc.get(j, 0.0) + wn
            total += wn
        acc[p] = acc.get(p, 0.0) - total
        for j in sorted(acc):
            A[g, j] = acc[j]
    return A.tocsr()


def bicgstab(A, b, x0=None, tol=1e-10, max_iters=10000):
    """Returns (x, iterations, relative residual, converged)."""
    n = b.size
    d = A.diagonal()
    dinv = np.where(d != 0.0, 1.0 / np.where(d != 0.0, d, 1.0), 1.0)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A @ x
    r0 = r.copy()
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros(n), 0, 0.0, True
    rho_old = alpha = omega = 1.0
    p = np.zeros(n)
    v = np.zeros(n)
    it = 0
    res = np.linalg.norm(r) / bn
    while res > tol and it < max_iters:
        rho = r0 @ r
        if rho == 0.0:
            break
        beta = (rho / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        y = dinv * p
        v = A @ y
        rv = r0 @ v
        if rv == 0.0:
            break
        alpha = rho / rv
        s = r - alpha * v
        z = dinv * s
        t = A @ z
        tt = t @ t
        omega = (t @ s) / tt if tt > 0.0 else 0.0
        x = x + alpha * y + omega * z
        r = s - omega * t
        rho_old = rho
        it += 1
        res = np.linalg.norm(r) / bn
        if omega == 0.0 and res > tol:
            break
    return x, it, res, res <= tol
