"""Pins of the oracle's lattice, equilibrium (Eq. 4), macroscopic quantities (Eqs. 5-6)
and Guo forcing term (Eqs. 7-8) against the paper's tables, its unrolled Eqs. 21-36,
its symmetry relations Eqs. 37-40 and the moment identities these definitions imply."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "lattice_velocities.txt")
CS2 = 1.0 / 3.0


def _golden():
    rows = {}
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        lat, a, ex, ey, ez, w = line.split()
        rows.setdefault(lat, []).append(((int(ex), int(ey), int(ez)), float(Fraction(w))))
    return rows


@pytest.mark.parametrize("dim,name", [(2, "D2Q9"), (3, "D3Q19")])
def test_lattice_matches_paper_table(dim, name):
    e, w = oracle.lattice(dim)
    gold = _golden()[name]
    assert len(gold) == len(w)
    for a, (ev, wv) in enumerate(gold):
        assert tuple(e[a]) == ev
        assert w[a] == wv


@pytest.mark.parametrize("dim", [2, 3])
def test_lattice_isotropy(dim):
    e, w = oracle.lattice(dim)
    e = e[:, :dim].astype(float)
    q = len(w)
    assert abs(w.sum() - 1) < 1e-15
    assert np.allclose(np.einsum("a,ai->i", w, e), 0, atol=1e-15)
    assert np.allclose(np.einsum("a,ai,aj->ij", w, e, e), CS2 * np.eye(dim), atol=1e-15)
    assert np.allclose(np.einsum("a,ai,aj,ak->ijk", w, e, e, e), 0, atol=1e-15)
    d = np.eye(dim)
    iso4 = CS2 ** 2 * (np.einsum("ij,kl->ijkl", d, d) + np.einsum("ik,jl->ijkl", d, d)
                       + np.einsum("il,jk->ijkl", d, d))
    assert np.allclose(np.einsum("a,ai,aj,ak,al->ijkl", w, e, e, e, e), iso4, atol=1e-15)
    h = (q - 1) // 2
    for a in range(1, h + 1):  # e_alpha = -e_{alpha-(q-1)/2}
        assert np.array_equal(e[a + h], -e[a])


def _rand(seed, k, scale):
    return np.random.default_rng(seed).uniform(-scale, scale, k)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("rho0", [1.0, 1.3])
def test_feq_moments(dim, rho0):
    e, w = oracle.lattice(dim)
    e = e[:, :dim].astype(float)
    for s in range(5):
        u = _rand(s, dim, 0.05)
        p = _rand(100 + s, 1, 0.01)[0]
        f = oracle.feq(dim, rho0, p, u)
        assert abs(f.sum()) < 1e-15  # lambda_0 absorbs the rest mass: sum_all = 0
        assert np.allclose(e.T @ f, rho0 * u, atol=1e-16)
        M2 = np.einsum("a,ai,aj->ij", f, e, e)
        assert np.allclose(M2, p * np.eye(dim) + rho0 * np.outer(u, u), atol=1e-16)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("rho0", [1.0, 0.7])
def test_eq6_inverts_feq(dim, rho0):
    for s in range(5):
        u = _rand(s, dim, 0.05)
        p = _rand(50 + s, 1, 0.01)[0]
        f = oracle.feq(dim, rho0, p, u)
        pp, uu = oracle.macro(dim, rho0, f)
        assert abs(pp - p) < 1e-16
        assert np.allclose(uu[:dim], u, atol=1e-17)


def test_unrolled_feq_eqs_21_28():
    """The paper's unrolled D2Q9 equilibria (c = 1, 3 = 1/c_s^2) equal Eq. 4."""
    _, w = oracle.lattice(2)
    for s in range(5):
        ux, uy = _rand(s, 2, 0.05)
        p = _rand(9 + s, 1, 0.01)[0]
        r = 1.0 + 0.3 * s
        eq = [None,
              3 * w[1] * (p + r * (ux + ux * ux - 0.5 * uy * uy)),
              3 * w[2] * (p + r * (ux + uy + 3 * ux * uy + ux * ux + uy * uy)),
              3 * w[3] * (p + r * (uy - 0.5 * ux * ux + uy * uy)),
              3 * w[4] * (p + r * (-ux + uy - 3 * ux * uy + ux * ux + uy * uy)),
              3 * w[5] * (p + r * (-ux + ux * ux - 0.5 * uy * uy)),
              3 * w[6] * (p + r * (-ux - uy + 3 * ux * uy + ux * ux + uy * uy)),
              3 * w[7] * (p + r * (-uy - 0.5 * ux * ux + uy * uy)),
              3 * w[8] * (p + r * (ux - uy - 3 * ux * uy + ux * ux + uy * uy))]
        f = oracle.feq(2, r, p, [ux, uy])
        assert np.allclose(f[1:], eq[1:], rtol=1e-13, atol=1e-20)


def test_unrolled_force_eqs_29_36():
    """The paper's unrolled D2Q9 forcing terms equal Eq. 8."""
    _, w = oracle.lattice(2)
    for s in range(5):
        ux, uy = _rand(s, 2, 0.05)
        fx, fy = _rand(20 + s, 2, 1e-3)
        tau = 0.6 + 0.1 * s
        k = 3 * (1 - 1 / (2 * tau))
        uf = ux * fx + uy * fy
        c = [None,
             k * w[1] * (fx + 3 * ux * fx - uf),
             k * w[2] * ((fx + fy) + 3 * (ux * fy + uy * fx) + 2 * uf),
             k * w[3] * (fy + 3 * uy * fy - uf),
             k * w[4] * ((-fx + fy) - 3 * (ux * fy + uy * fx) + 2 * uf),
             k * w[5] * (-fx + 3 * ux * fx - uf),
             k * w[6] * (-(fx + fy) + 3 * (ux * fy + uy * fx) + 2 * uf),
             k * w[7] * (-fy + 3 * uy * fy - uf),
             k * w[8] * ((fx - fy) - 3 * (ux * fy + uy * fx) + 2 * uf)]
        F = oracle.guo_force(2, tau, [ux, uy], [fx, fy])
        assert np.allclose(F[1:], c[1:], rtol=1e-13, atol=1e-22)


@pytest.mark.parametrize("dim", [2, 3])
def test_symmetry_eqs_38_40(dim):
    """Opposite directions differ only in the odd term (Eqs. 37-40; Eq. 38 printed
    without rho0, which multiplies the odd term of Eq. 37)."""
    e, w = oracle.lattice(dim)
    q = len(w)
    h = (q - 1) // 2
    for s in range(4):
        u = _rand(s, dim, 0.05)
        f = _rand(30 + s, dim, 1e-3)
        rho0, tau, p = 1.2, 0.7, 0.003
        fe = oracle.feq(dim, rho0, p, u)
        F = oracle.guo_force(dim, tau, u, f)
        for a in range(1, h + 1):
            eu = e[a, :dim] @ u
            ef = e[a, :dim] @ f
            assert abs(fe[a + h] - (fe[a] - 2 * rho0 * w[a] * eu / CS2)) < 1e-17
            assert abs(F[a + h] - (F[a] - 2 * (1 - 1 / (2 * tau)) * w[a] * ef / CS2)) < 1e-19


@pytest.mark.parametrize("dim", [2, 3])
def test_force_moments(dim):
    e, w = oracle.lattice(dim)
    e = e[:, :dim].astype(float)
    for s in range(4):
        u = _rand(s, dim, 0.05)
        f = _rand(40 + s, dim, 1e-3)
        tau = 0.55 + 0.2 * s
        k = 1 - 1 / (2 * tau)
        F = oracle.guo_force(dim, tau, u, f)
        assert abs(F.sum()) < 1e-18
        assert np.allclose(e.T @ F, k * f, atol=1e-19)
        M2 = np.einsum("a,ai,aj->ij", F, e, e)
        assert np.allclose(M2, k * (np.outer(u, f) + np.outer(f, u)), atol=1e-19)
