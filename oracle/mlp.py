"""FP64 reference of the learned warm start for the order-8 weight solve.

Test infrastructure: only the tests, the entry point's smoke check and the
benchmark's CPU-baseline leg import this module; the library never does.

The network is not part of the paper.  It maps the scaled offsets of a
stencil's nearest neighbours to the ABF coefficients Psi^d of the moment
system M Psi^d = C^d (Sec. 3.1, eq. lsys), so that the weight refinement of
that section can start from its output instead of from a fresh solve.

Pieces, each written from its textbook definition:
  * stencil_features: neighbours ordered by (squared scaled distance, index),
    the nearest kmax kept, each as (dx/h, dy/h, 1); missing slots (0, 0, 0).
  * forward/backward: fully connected layers z = h W^T + b, SiLU
    (z * sigmoid(z)) between layers, a linear last layer; backward by the
    chain rule.
  * moment_loss: the network output y is de-normalised per component,
    Psi = mu + sd * y, and the loss is the batch mean of
    sum_d ||M_s Psi^d - C^d||^2, the squared residual of eq. (lsys).
  * adam_step: Adam with bias correction (Kingma & Ba, ICLR 2015, Alg. 1).
"""
import numpy as np


# ---------------------------------------------------------------- features

def stencil_offsets(x, y, domain, R, row_ptr, col):
    """Scaled offsets d = (r_j - r_i) / h_i, h_i = R_i / 2, minimum image on
    periodic axes.  Returns (dx, dy) [nnz] aligned with col."""
    n = x.size
    N = np.diff(row_ptr)
    rows = np.repeat(np.arange(n), N)
    dx = x[col] - x[rows]
    dy = y[col] - y[rows]
    L = (domain["hi"][0] - domain["lo"][0], domain["hi"][1] - domain["lo"][1])
    if domain["periodic"][0]:
        dx = dx - L[0] * np.round(dx / L[0])
    if domain["periodic"][1]:
        dy = dy - L[1] * np.round(dy / L[1])
    h = 0.5 * np.asarray(R, np.float64)[rows]
    return dx / h, dy / h


def stencil_features(x, y, domain, R, row_ptr, col, kmax=64, nodes=None):
    """[len(nodes), 3 * kmax] FP32 features (see module docstring)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    row_ptr = np.asarray(row_ptr, np.int64)
    col = np.asarray(col, np.int64)
    R = np.broadcast_to(np.asarray(R, np.float64), x.shape)
    dxa, dya = stencil_offsets(x, y, domain, R, row_ptr, col)
    nodes = np.arange(x.size) if nodes is None else np.asarray(nodes)
    out = np.zeros((nodes.size, kmax, 3), np.float32)
    for t, i in enumerate(nodes):
        s, e = row_ptr[i], row_ptr[i + 1]
        dx, dy, j = dxa[s:e], dya[s:e], col[s:e]
        d2 = dx * dx + dy * dy
        order = np.lexsort((j, d2))[:kmax]
        k = order.size
        out[t, :k, 0] = dx[order]
        out[t, :k, 1] = dy[order]
        out[t, :k, 2] = 1.0
    return out.reshape(nodes.size, 3 * kmax)


# ---------------------------------------------------------------- network

def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(dims, seed):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases; W[l] is
    [dims[l+1], dims[l]]."""
    rng = np.random.default_rng(seed)
    Ws = [rng.standard_normal((dims[l + 1], dims[l])) * np.sqrt(2.0 / dims[l]) for l in range(len(dims) - 1)]
    bs = [np.zeros(dims[l + 1]) for l in range(len(dims) - 1)]
    return Ws, bs


def forward(Ws, bs, X):
    """Returns (output, cache); cache = (layer inputs, pre-activations)."""
    H = np.asarray(X, np.float64)
    ins, zs = [], []
    L = len(Ws)
    for l in range(L):
        ins.append(H)
        Z = H @ Ws[l].T + bs[l]
        zs.append(Z)
        H = silu(Z) if l < L - 1 else Z
    return H, (ins, zs)


def backward(Ws, cache, dY):
    """Gradients (dWs, dbs) of a scalar loss with dLoss/dOutput = dY."""
    ins, zs = cache
    L = len(Ws)
    dWs, dbs = [None] * L, [None] * L
    dZ = np.asarray(dY, np.float64)
    for l in range(L - 1, -1, -1):
        dWs[l] = dZ.T @ ins[l]
        dbs[l] = dZ.sum(axis=0)
        if l > 0:
            dZ = (dZ @ Ws[l]) * silu_grad(zs[l - 1])
    return dWs, dbs


def moment_loss(y, M, C, mu, sd):
    """Batch mean of sum_d ||M_s (mu + sd * y_s)^d - C^d||^2.

    y [B, nops*p]; M [B, p, p]; C [nops, p]; mu, sd [nops*p].
    Returns (loss, dloss/dy)."""
    B = y.shape[0]
    nops, p = C.shape
    Psi = (mu + sd * y).reshape(B, nops, p)
    r = np.einsum("smq,sdq->sdm", M, Psi) - C[None, :, :]
    loss = float((r * r).sum() / B)
    g = 2.0 * np.einsum("smq,sdm->sdq", M, r).reshape(B, nops * p) * sd / B
    return loss, g


def adam_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t >= 1; returns (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
