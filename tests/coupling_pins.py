"""Pins of the oracle's particle coupling (Sec. 2.3, Eqs. 14-16), each against a value
that the mathematics fixes independently of the oracle's own code: closed forms of a
recurrence, exact integrals of the interior-volume indicator, geometric special cases,
and the mirror-image construction checked against the oracle's pair-force path.

Every pin takes an optional oracle library handle `L` (``oracle.load(path)``) so that
``test_oracle_mutations.py`` can run it against copies of the oracle with planted
mistakes; with L = None it checks the oracle itself.  A pin raises AssertionError when the
oracle disagrees."""
import math

import numpy as np
from scipy import integrate

import oracle

PI = math.pi


def _close(a, b, rtol, atol=0.0, what=""):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    err = np.abs(a - b).max()
    tol = rtol * max(np.abs(b).max(), 1e-300) + atol
    assert err <= tol, f"{what}: |diff| {err:.3e} > {tol:.3e} ({a} vs {b})"


# ---------------------------------------------------------------------------
# Newton-Euler (Eqs. 14-15)

def _state(X0, U0, Om0, P0):
    return dict(Pprev=np.array(P0, float), Lprev=np.zeros(3), Hprev=np.zeros(3), Gprev=np.zeros(3),
                X=np.array(X0, float), U=np.array(U0, float), Om=np.array(Om0, float))


def pin_newton_euler_constant_loads(L=None):
    """Constant loads from the first step: the hydrodynamic load H = F_h + (P - Pprev)
    enters as the mean of this and the previous step's value (zero before the first
    step), so U^1 = U^0 + (H/2 + B)/M and U^k = U^(k-1) + (H + B)/M afterwards, with
    B = F_c + (M - rho0 V) g; X follows the trapezoid rule; Omega the same recurrence with
    G = T_h + (L - Lprev) and I.  The interior momentum P grows by dP each step, so
    F_f = dP enters H with its sign."""
    for dim in (2, 3):
        rho0, M, V, I = 1.0, 2.3, 1.6, 0.71
        g = np.array([0.0, -1e-3, 0.0])
        Fh = np.array([3e-4, -2e-4, 1e-4 if dim == 3 else 0.0])
        Th = np.array([2e-4, -1e-4, 5e-5])
        Fc = np.array([-1e-4, 4e-4, 2e-4 if dim == 3 else 0.0])
        dP = np.array([1.5e-4, 2.5e-4, -1e-4 if dim == 3 else 0.0])
        dL = np.array([-3e-5, 4e-5, 6e-5])
        X0 = np.array([10.0, 20.0, 15.0 if dim == 3 else 0.0])
        U0 = np.array([1e-3, -2e-3, 5e-4 if dim == 3 else 0.0])
        Om0 = np.array([1e-4, 2e-4, -3e-4]) if dim == 3 else np.array([0.0, 0.0, -3e-4])
        P0 = np.array([0.2, -0.1, 0.05])
        st = _state(X0, U0, Om0, P0)
        st["Lprev"] = np.array([0.01, 0.02, -0.03])
        Lm0 = st["Lprev"].copy()
        nsteps = 7
        for k in range(1, nsteps + 1):
            P = P0 + k * dP
            Lm = Lm0 + k * dL
            oracle.newton_euler(dim, M, V, I, rho0, g, Fh, Th, Fc, P, Lm, st, L=L)
        d = slice(0, dim)
        H = Fh + dP
        B = Fc + (M - rho0 * V) * g
        b = (0.5 * H + B) / M          # first-step increment
        a = (H + B) / M                # later increments
        n = nsteps
        Un = U0 + b + (n - 1) * a
        # X^n = X0 + (U^0 + U^n)/2 + sum_{k=1}^{n-1} U^k
        sumU = (n - 1) * (U0 + b) + a * (n - 1) * (n - 2) / 2.0
        Xn = X0 + 0.5 * (U0 + Un) + sumU
        _close(st["U"][d], Un[d], 1e-12, what=f"{dim}-D U after {n} constant-load steps")
        _close(st["X"][d], Xn[d], 1e-13, what=f"{dim}-D X after {n} steps")
        G = Th + dL
        rot = [2] if dim == 2 else [0, 1, 2]
        Omn = Om0 + (0.5 * G + (n - 1) * G) / I
        _close(st["Om"][rot], Omn[rot], 1e-12, what=f"{dim}-D Omega after {n} steps")
        # the stored previous-step values are this step's
        _close(st["Hprev"][d], H[d], 1e-12, what="Hprev")
        _close(st["Pprev"], P0 + n * dP, 1e-15, what="Pprev")


def pin_newton_euler_rigid_interior(L=None):
    """Interior fluid moving rigidly with the body (P = rho0 V U): Eq. 14 becomes
    (M - rho0 V) dU/dt = F_c + (M - rho0 V) g, so the velocity increment per step tends to
    (F_c + (M - rho0 V) g)/(M - rho0 V) (density ratio 2 and 1.01)."""
    for ratio in (2.0, 1.01):
        dim, rho0, V = 2, 1.0, 50.0
        M = ratio * rho0 * V
        I = 0.5 * M * 16.0
        g = np.array([0.0, -1e-5, 0.0])
        Fc = np.array([2e-6, 0.0, 0.0])
        st = _state([30.0, 40.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0])
        prevU = st["U"].copy()
        steps = 200 if ratio > 1.5 else 20000
        for _ in range(steps):
            P = rho0 * V * st["U"]
            prevU = st["U"].copy()
            oracle.newton_euler(dim, M, V, I, rho0, g, np.zeros(3), np.zeros(3), Fc, P, np.zeros(3),
                                st, L=L)
        dU = st["U"] - prevU
        meff = M - rho0 * V
        _close(dU[:2], (Fc + meff * g)[:2] / meff, 1e-9, what=f"rigid-interior increment, ratio {ratio}")


# ---------------------------------------------------------------------------
# interior momentum (F_f and T_f of Eqs. 14-15)

def _chi_integrals(dim, R):
    """Exact integrals of chi = clamp(R + 1/2 - r, 0, 1): volume, and the second moment
    about the z axis (the rigid-rotation moment), from their radial profiles."""
    def chi(r):
        return min(1.0, max(0.0, R + 0.5 - r))
    if dim == 2:
        vol = PI * R * R + PI / 12.0  # closed form
        mom = PI * R ** 4 / 2.0 + PI * R * R / 4.0 + PI / 160.0
        return vol, mom
    vol = 4.0 / 3.0 * PI * R ** 3 + PI * R / 3.0
    # the sphere's moment about an axis: (2/3) of the radial second moment
    inner = 4.0 * PI * (R - 0.5) ** 5 / 5.0
    shell, _ = integrate.quad(lambda r: chi(r) * 4.0 * PI * r ** 4, R - 0.5, R + 0.5,
                              epsabs=1e-13, epsrel=1e-13)
    return vol, 2.0 / 3.0 * (inner + shell)


def _offsets(dim, K):
    g = (np.arange(K) + 0.5) / K
    if dim == 2:
        return [(a, b, 0.0) for a in g for b in g]
    return [(a, b, c) for a in g for b in g for c in g]


def pin_interior_volume_and_moment(L=None):
    """Averaged over centre offsets in the unit cell, the lattice sums of chi and of chi
    times the squared distance to the z axis equal their integrals (translation average
    of a lattice sum = integral): 2-D pi R^2 + pi/12 and pi R^4/2 + pi R^2/4 + pi/160,
    3-D 4 pi R^3/3 + pi R/3 and the quadrature of the shell.  The sums come from the
    oracle's momentum with a uniform field (P = rho0 U sum chi) and a rigid rotation
    about z (L_z = rho0 Omega sum chi r_perp^2)."""
    for dim, R, K, n in ((2, 7.0, 24, 32), (3, 5.0, 7, 24)):
        N = n ** dim
        shape = (n,) * dim
        # node coordinates in the order i = x + n (y + n z)
        lin = np.arange(N)
        x = lin % n
        y = (lin // n) % n
        rho0, Om, Ux = 1.3, 2e-3, 1e-2
        vols, moms = [], []
        for off in _offsets(dim, K):
            Xc = np.array([n / 2 - 0.5 + off[0], n / 2 - 0.5 + off[1],
                           (n / 2 - 0.5 + off[2]) if dim == 3 else 0.0])
            u = np.zeros((dim, N))
            u[0] = Ux
            P, _ = oracle.interior_momentum(dim, shape, Xc, R, rho0, u, L=L)
            vols.append(P[0] / (rho0 * Ux))
            # u = Om e_z x (x - Xc)
            u = np.zeros((dim, N))
            u[0] = -Om * (y - Xc[1])
            u[1] = Om * (x - Xc[0])
            _, Lm = oracle.interior_momentum(dim, shape, Xc, R, rho0, u, L=L)
            moms.append(Lm[2] / (rho0 * Om))
            assert abs(P[1]) < 1e-12 * abs(P[0]) + 1e-300
        vol, mom = _chi_integrals(dim, R)
        _close(np.mean(vols), vol, 1e-5 if dim == 2 else 5e-5, what=f"{dim}-D mean sum chi")
        _close(np.mean(moms), mom, 1e-5 if dim == 2 else 1e-4, what=f"{dim}-D mean sum chi r_perp^2")


# ---------------------------------------------------------------------------
# hydrodynamic load (F_h, T_h of Eqs. 14-15)

def pin_loads_closed_forms(L=None):
    """F_h = -sum F_k dV_k and T_h = -sum r_k x F_k dV_k: for N equally spaced points on
    a circle of radius R with a tangential force f each, F_h = 0 and T_h = -N R f dV e_z;
    with one uniform force F, F_h = -N F dV and T_h = 0; a point on the x axis pushed
    along z gives T_h = +R f dV e_y."""
    N, R, f, dV = 48, 6.5, 3e-3, 0.85
    th = 2 * PI * np.arange(N) / N
    r = np.stack([R * np.cos(th), R * np.sin(th), np.zeros(N)], 1)
    F = np.stack([-f * np.sin(th), f * np.cos(th), np.zeros(N)], 1)
    Fh, Th = oracle.particle_loads(r, F, np.full(N, dV), L=L)
    _close(Fh, np.zeros(3), 0.0, atol=1e-15, what="tangential F_h")
    _close(Th, [0.0, 0.0, -N * R * f * dV], 1e-14, what="tangential T_h")
    F0 = np.array([1e-3, -2e-3, 5e-4])
    Fh, Th = oracle.particle_loads(r, np.tile(F0, (N, 1)), np.full(N, dV), L=L)
    _close(Fh, -N * F0 * dV, 1e-14, what="uniform F_h")
    _close(Th, np.zeros(3), 0.0, atol=1e-16, what="uniform T_h")
    Fh, Th = oracle.particle_loads([[R, 0.0, 0.0]], [[0.0, 0.0, f]], [dV], L=L)
    _close(Th, [0.0, R * f * dV, 0.0], 1e-15, what="single-point T_h")


# ---------------------------------------------------------------------------
# wall images (Eq. 16 against the mirror particle)

def pin_wall_force_is_mirror_pair(L=None):
    """A particle at h from a wall plane feels the Eq. 16 force of its mirror image: the
    same as the pair force between it and a particle at distance 2h in open space (the
    oracle's pair path), directed away from the wall; zero once the surface gap h - D/2
    reaches zeta/2; and near a corner both walls act."""
    D, zeta, c, eps, E = 10.0, 1.0, 2e-3, 1e-3, 1e-4
    n = (40, 36, 30)
    per = (0, 0, 0)
    for dim in (2, 3):
        for h in (4.6, 5.0, 5.3, 5.49):
            for axis in range(dim):
                for side in (0, 1):
                    X = np.array([20.0, 18.0, 15.0 if dim == 3 else 0.0])
                    X[axis] = -0.5 + h if side == 0 else n[axis] - 0.5 - h
                    Fc = oracle.pair_forces(dim, n[:dim], per, [X], [D], [c],
                                            zeta, eps, E, np.zeros((0, 2)), L=L)[0]
                    # the pair in open space: two particles 2h apart along the axis
                    big = (400, 400, 400)
                    A = np.array([200.0, 200.0, 200.0 if dim == 3 else 0.0])
                    Bp = A.copy()
                    Bp[axis] -= 2 * h
                    Fp = oracle.pair_forces(dim, big[:dim], per, [A, Bp], [D, D], [c, c], zeta,
                                            eps, E, [[0, 1]], L=L)[0]
                    want = np.zeros(3)
                    want[axis] = Fp[axis] if side == 0 else -Fp[axis]
                    assert Fp[axis] > 0.0
                    _close(Fc, want, 1e-12, atol=1e-14, what=f"wall force dim={dim} h={h} axis={axis} side={side}")
        # beyond the range: surface gap h - D/2 >= zeta/2
        X = np.array([-0.5 + 0.5 * (D + zeta), 18.0, 15.0 if dim == 3 else 0.0])
        Fc = oracle.pair_forces(dim, n[:dim], per, [X], [D], [c], zeta, eps, E, np.zeros((0, 2)), L=L)[0]
        assert np.all(Fc == 0.0), Fc
    # a corner: both the -x and the +y walls push
    X = np.array([-0.5 + 5.2, n[1] - 0.5 - 5.3, 0.0])
    Fc = oracle.pair_forces(2, n[:2], per, [X], [D], [c], zeta, eps, E, np.zeros((0, 2)), L=L)[0]
    assert Fc[0] > 0.0 and Fc[1] < 0.0, Fc


# ---------------------------------------------------------------------------
# the gap feature of the learned forcing

def pin_gap_feature_geometry(L=None):
    """Two disks (D = 10 and 8) with a surface gap of 0.6 along x: the point of disk 0
    facing disk 1 has gap 0.6; the point facing away is clamped to zeta; a point 0.3
    from the -y wall has gap 0.3; without the pair in the list only the walls count; a
    disk at negative gap (overlap) clamps to 0.  In 3-D the same along z."""
    zeta = 1.0
    for dim in (2, 3):
        n = (60, 50, 40)[:dim]
        ax = 0 if dim == 2 else 2
        X0 = np.array([20.0, 25.0, 20.0 if dim == 3 else 0.0])
        X1 = X0.copy()
        X1[ax] += 5.0 + 4.0 + 0.6
        X = np.stack([X0, X1])
        D = np.array([10.0, 8.0])
        pairs = [[0, 1]]
        e = np.zeros(3)
        e[ax] = 1.0
        g = oracle.point_gap(dim, n, (0, 0, 0), zeta, X0 + 5.0 * e, 0, X, D, pairs, L=L)
        _close(g, 0.6, 1e-13, what=f"{dim}-D facing point")
        g = oracle.point_gap(dim, n, (0, 0, 0), zeta, X0 - 5.0 * e, 0, X, D, pairs, L=L)
        assert g == zeta, g
        g = oracle.point_gap(dim, n, (0, 0, 0), zeta, X1 - 4.0 * e, 1, X, D, pairs, L=L)
        _close(g, 0.6, 1e-13, what=f"{dim}-D facing point of the partner")
        g = oracle.point_gap(dim, n, (0, 0, 0), zeta, X0 + 5.0 * e, 0, X, D, np.zeros((0, 2)), L=L)
        assert g == zeta, g
        # a point 0.3 from the -y wall plane at -1/2
        Xw = np.array([30.0, -0.5 + 0.3, 20.0 if dim == 3 else 0.0])
        g = oracle.point_gap(dim, n, (0, 0, 0), zeta, Xw, 0, X, D, np.zeros((0, 2)), L=L)
        _close(g, 0.3, 1e-13, what=f"{dim}-D wall gap")
        # overlap: clamped to zero
        X2 = X.copy()
        X2[1, ax] = X0[ax] + 8.5
        g = oracle.point_gap(dim, n, (0, 0, 0), zeta, X0 + 5.0 * e, 0, X2, D, pairs, L=L)
        assert g == 0.0, g


# ---------------------------------------------------------------------------
# learned forcing: the prediction's output transform

def pin_learned_force_prediction(L=None):
    """The learned force F = F_prev + target mean + target std * y, y the network's
    output on the features normalised by their mean and std: with zero weights y is the
    output bias; with one path through the network y0 = c tanh(b tanh(a x0)) on the
    normalised first feature.  Components past the lattice dimension are zero."""
    NP = oracle.NPARAM
    rng = np.random.default_rng(5)
    n = 9
    feat = rng.normal(size=(n, 10))
    Fprev = rng.normal(size=(n, 3))
    norm = np.concatenate([rng.normal(size=10), rng.uniform(0.5, 2.0, 10),
                           [0.1, -0.2, 0.3], [2.0, 3.0, 0.5]])
    P = np.zeros(NP)
    P[NP - 3:] = [0.25, -0.5, 1.5]
    want = Fprev + norm[20:23] + norm[23:26] * np.array([0.25, -0.5, 1.5])
    _close(oracle.mlp_predict(P, norm, feat, Fprev, dim=3, L=L), want, 1e-14, 1e-15,
           what="output bias only")
    F2 = oracle.mlp_predict(P, norm, feat, Fprev, dim=2, L=L)
    _close(F2[:, :2], want[:, :2], 1e-14, 1e-15, what="2-D")
    assert np.array_equal(F2[:, 2], np.zeros(n))
    P = np.zeros(NP)
    P[0] = 0.7
    off_w2 = 10 * 64 + 64
    P[off_w2] = -1.3
    P[off_w2 + 64 * 64 + 64] = 2.1
    x0 = (feat[:, 0] - norm[0]) / norm[10]
    F = oracle.mlp_predict(P, norm, feat, Fprev, dim=3, L=L)
    y0 = 2.1 * np.tanh(-1.3 * np.tanh(0.7 * x0))
    _close(F[:, 0], Fprev[:, 0] + norm[20] + norm[23] * y0, 1e-13, 1e-14, what="one path")
    _close(F[:, 1:], Fprev[:, 1:] + norm[21:23], 1e-14, 1e-15, what="the other components")


ALL = [pin_newton_euler_constant_loads, pin_newton_euler_rigid_interior,
       pin_interior_volume_and_moment, pin_loads_closed_forms, pin_wall_force_is_mirror_pair,
       pin_gap_feature_geometry, pin_learned_force_prediction]
