"""Neighbour sets of the oracle against an O(n^2) brute force written here in
numpy (the definition of Sec. 2: all j != i with |r_j - r_i| < 2h)."""
import numpy as np
import pytest

from paper_1912_06441_amd import workloads as WL


def brute(x, y, R, periodic):
    n = x.size
    dx = x[None, :] - x[:, None]
    dy = y[None, :] - y[:, None]
    if periodic:
        dx = np.where(dx > 0.5, dx - 1.0, np.where(dx < -0.5, dx + 1.0, dx))
        dy = np.where(dy > 0.5, dy - 1.0, np.where(dy < -0.5, dy + 1.0, dy))
    d2 = dx * dx + dy * dy
    mask = d2 < (R * R)[:, None]
    np.fill_diagonal(mask, False)
    rows = [np.nonzero(mask[i])[0].astype(np.int32) for i in range(n)]
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum([r.size for r in rows])
    return rp, np.concatenate(rows) if rows else np.zeros(0, np.int32)


@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("side,Rs", [(24, 2.85), (40, 4.4), (7, 2.5), (3, 1.1)])
def test_cells_equal_brute_force(O, periodic, side, Rs):
    x, y, s = WL.jittered_lattice(side, eps=0.3, seed=side, periodic=periodic)
    dom = WL.unit_domain(periodic)
    R = np.full(x.size, Rs * s)
    rp, col, _ = O.neighbours(x, y, dom, R, 4, grow=False)
    rp2, col2, _ = O.neighbours(x, y, dom, R, 4, grow=False, method="brute")
    rp3, col3 = brute(x, y, R, periodic)
    assert np.array_equal(rp, rp3) and np.array_equal(col, col3)
    assert np.array_equal(rp2, rp3) and np.array_equal(col2, col3)


def test_rows_ascending_and_exclude_self(O):
    x, y, s = WL.jittered_lattice(32, eps=0.45, seed=3)
    rp, col, _ = O.neighbours(x, y, WL.unit_domain(), 3.0 * s, 4, grow=False)
    for i in range(x.size):
        row = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0)
        assert i not in row


@pytest.mark.parametrize("periodic", [False, True])
def test_growth_rule(O, periodic):
    """R_i <- 1.1 R_i (repeated, FP64) until N_i >= N_crit(k_i); the grown
    radius then gives the brute-force set."""
    x, y, s = WL.jittered_lattice(30, eps=0.3, seed=9, periodic=periodic)
    dom = WL.unit_domain(periodic)
    order = WL.order_map(x, y, 8, band=3.0 * s, k_boundary=4, periodic=periodic)
    R0 = np.full(x.size, 3.0 * s)
    rp, col, R = O.neighbours(x, y, dom, R0, order, grow=True, max_grow=10)
    ncrit = {4: 21, 8: 57}
    N = np.diff(rp)
    for i in range(x.size):
        g = 0
        r = R0[i]
        while g < 10:
            # the radius before R[i] must have been too small
            if r == R[i]:
                break
            r = r * 1.1
            g += 1
        assert r == R[i]
        assert N[i] >= ncrit[int(order[i])] or g == 10
    rp3, col3 = brute(x, y, R, periodic)
    assert np.array_equal(rp, rp3) and np.array_equal(col, col3)
    # grown nodes needed it: with the previous radius they had too few neighbours
    grown = np.nonzero(R > R0)[0]
    assert grown.size > 0
    rp4, _ = brute(x, y, R / 1.1, periodic)
    N4 = np.diff(rp4)
    assert np.all(N4[grown] < np.array([ncrit[int(k)] for k in order[grown]]))


def test_degenerate_sets(O):
    # single node, and all nodes coincident
    rp, col, _ = O.neighbours(np.array([0.5]), np.array([0.5]), WL.unit_domain(), 0.1, 4, grow=False)
    assert rp.tolist() == [0, 0] and col.size == 0
    x = np.full(5, 0.25)
    y = np.full(5, 0.75)
    rp, col, _ = O.neighbours(x, y, WL.unit_domain(), 0.1, 4, grow=False)
    assert np.diff(rp).tolist() == [4] * 5
