"""Pins of the oracle's delta functions and IBM operators (Sec. 2.2, Eqs. 9-13, 43-48):
the moment conditions that define the Peskin 4-point and Roma 3-point kernels, exact
interpolation of linear fields, conservation of force and torque by spreading, the
adjointness of interpolation and spreading, and the equality of the naive all-node
sums (Eqs. 43-44) with the point-to-node form (Eqs. 47-48)."""
import numpy as np
import pytest

import oracle

OFFSETS = [0.0, 0.1234, 0.5, 0.77, 0.999999, 0.31415926]


@pytest.mark.parametrize("r0", OFFSETS)
def test_peskin4_moments(r0):
    j = np.arange(-3, 5)
    v = np.array([oracle.phi(0, jj - r0) for jj in j])
    assert abs(v.sum() - 1) < 1e-15                 # partition of unity
    assert abs((v * (j - r0)).sum()) < 1e-15        # first moment
    assert abs((v * v).sum() - 3 / 8) < 1e-15       # sum of squares
    assert abs(v[j % 2 == 0].sum() - 0.5) < 1e-15   # even / odd split
    assert abs(v[j % 2 == 1].sum() - 0.5) < 1e-15
    assert np.all(v >= 0)


@pytest.mark.parametrize("r0", OFFSETS)
def test_roma3_moments(r0):
    j = np.arange(-3, 5)
    v = np.array([oracle.phi(1, jj - r0) for jj in j])
    assert abs(v.sum() - 1) < 1e-15
    assert abs((v * (j - r0)).sum()) < 1e-15
    assert abs((v * v).sum() - 0.5) < 1e-15
    assert np.all(v >= 0)


def test_kernels_continuous_and_compact():
    for r in (1.0, 2.0):
        assert abs(oracle.phi(0, r - 1e-12) - oracle.phi(0, r + 1e-12)) < 1e-11
    for r in (0.5, 1.5):
        assert abs(oracle.phi(1, r - 1e-12) - oracle.phi(1, r + 1e-12)) < 1e-11
    assert oracle.phi(0, 2.0) == 0.0 and oracle.phi(0, 2.5) == 0.0
    assert oracle.phi(1, 1.5) == 0.0
    assert abs(oracle.phi(0, 0.0) - 0.5) < 1e-16 and abs(oracle.phi(1, 0.0) - 2 / 3) < 1e-16


def _markers(dim, n, k, seed, margin=3.0):
    rng = np.random.default_rng(seed)
    X = np.zeros((k, 3))
    for a in range(dim):
        X[:, a] = rng.uniform(margin, n[a] - 1 - margin, k)
    return X


@pytest.mark.parametrize("dim,n", [(2, (16, 14, 1)), (3, (10, 9, 11))])
@pytest.mark.parametrize("kind", [0, 1])
def test_interp_linear_exact(dim, n, kind):
    N = int(np.prod(n))
    z, y, x = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    xs = [x.ravel(), y.ravel(), z.ravel()]
    A = np.array([[0.3, -1.1, 0.7], [2.0, 0.25, -0.5], [-0.4, 0.9, 1.3]])
    b = np.array([0.1, -0.2, 0.05])
    u = np.stack([b[c] + sum(A[c, a] * xs[a] for a in range(dim)) for c in range(dim)])
    X = _markers(dim, n, 20, 3)
    uh = oracle.ibm_interp(dim, n, (0, 0, 0), kind, u.ravel(), X)
    exact = b[:dim] + X[:, :dim] @ A[:dim, :dim].T
    assert np.allclose(uh[:, :dim], exact, atol=1e-12)


@pytest.mark.parametrize("dim,n", [(2, (16, 14, 1)), (3, (10, 9, 11))])
@pytest.mark.parametrize("kind", [0, 1])
def test_spread_conserves_force_and_torque(dim, n, kind):
    N = int(np.prod(n))
    X = _markers(dim, n, 15, 5)
    rng = np.random.default_rng(7)
    F = np.zeros((15, 3))
    F[:, :dim] = rng.normal(size=(15, dim))
    dV = rng.uniform(0.5, 2.0, 15)
    g = oracle.ibm_spread(dim, n, (0, 0, 0), kind, F, dV, X).reshape(dim, N)
    tot = (F[:, :dim] * dV[:, None]).sum(0)
    assert np.allclose(g.sum(1), tot, atol=1e-13)
    if dim == 2:
        z, y, x = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
        xs = np.stack([x.ravel(), y.ravel()]).astype(float)
        tq_grid = (xs[0] * g[1] - xs[1] * g[0]).sum()
        tq_pts = ((X[:, 0] * F[:, 1] - X[:, 1] * F[:, 0]) * dV).sum()
        assert abs(tq_grid - tq_pts) < 1e-11
    else:
        z, y, x = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
        xs = np.stack([x.ravel(), y.ravel(), z.ravel()]).astype(float)
        tq_grid = np.cross(xs.T, g.T).sum(0)
        tq_pts = (np.cross(X, F) * dV[:, None]).sum(0)
        assert np.allclose(tq_grid, tq_pts, atol=1e-11)


@pytest.mark.parametrize("dim,n", [(2, (12, 13, 1)), (3, (8, 9, 7))])
def test_adjointness(dim, n):
    N = int(np.prod(n))
    rng = np.random.default_rng(11)
    X = _markers(dim, n, 9, 13, margin=0.0)  # includes truncated stencils near walls
    u = rng.normal(size=dim * N)
    F = np.zeros((9, 3))
    F[:, :dim] = rng.normal(size=(9, dim))
    dV = rng.uniform(0.5, 2.0, 9)
    uh = oracle.ibm_interp(dim, n, (0, 0, 0), 0, u, X)
    g = oracle.ibm_spread(dim, n, (0, 0, 0), 0, F, dV, X)
    lhs = (uh[:, :dim] * F[:, :dim] * dV[:, None]).sum()
    rhs = (u * g).sum()
    assert abs(lhs - rhs) < 1e-12


@pytest.mark.parametrize("dim,n", [(2, (12, 13, 1)), (3, (7, 8, 6))])
@pytest.mark.parametrize("kind", [0, 1])
def test_naive_equals_point_to_node(dim, n, kind):
    """Eqs. 43-44 (every node) and Eqs. 47-48 (kernel support only) add the same
    nonzero terms in the same order, so they agree bit for bit."""
    N = int(np.prod(n))
    rng = np.random.default_rng(17)
    X = _markers(dim, n, 6, 19, margin=0.0)
    u = rng.normal(size=dim * N)
    F = np.zeros((6, 3))
    F[:, :dim] = rng.normal(size=(6, dim))
    dV = rng.uniform(0.5, 2.0, 6)
    a = oracle.ibm_interp(dim, n, (0, 0, 0), kind, u, X, naive=False)
    b = oracle.ibm_interp(dim, n, (0, 0, 0), kind, u, X, naive=True)
    assert np.array_equal(a, b)
    ga = oracle.ibm_spread(dim, n, (0, 0, 0), kind, F, dV, X, naive=False)
    gb = oracle.ibm_spread(dim, n, (0, 0, 0), kind, F, dV, X, naive=True)
    assert np.array_equal(ga, gb)


def test_periodic_wrap_partition():
    """On a periodic axis the support wraps: a constant field interpolates exactly
    even for points next to the seam."""
    n = (8, 8, 1)
    u = np.ones(2 * 64)
    X = np.array([[0.2, 7.6, 0.0], [7.9, 0.1, 0.0]])
    uh = oracle.ibm_interp(2, n, (1, 1, 0), 0, u, X)
    assert np.allclose(uh[:, :2], 1.0, atol=1e-15)
