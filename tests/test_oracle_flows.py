"""Pins of the oracle's collide-stream step (Eq. 1 with Eqs. 4-8, two-array streaming
Eqs. 17-18, half-way bounce-back walls) against closed-form flows, exact mass
conservation and the exact mass budget with forcing, and the bitwise equality of the
single-array swap scheme (Sec. 3.3) with two-array streaming."""
import math

import numpy as np
import pytest

import oracle
from paper_2002_08855_amd import inputs


def _steady(sim, tol=1e-15, chunk=500, max_steps=200000):
    last = None
    for _ in range(max_steps // chunk):
        sim.step(chunk)
        _, u, _ = sim.fields()
        if last is not None and np.max(np.abs(u - last)) < tol:
            return u
        last = u
    raise AssertionError("no steady state")


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.3])
def test_couette_2d_linear_profile(tau):
    ny, U = 12, 0.01
    wall = [[0, 0, 0] for _ in range(6)]
    wall[3] = [U, 0, 0]                        # +y wall moves along x
    p = inputs.default_params(2, (3, ny), tau=tau, periodic=(1, 0, 0), wall_u=wall)
    s = oracle.Sim(p)
    u = _steady(s, tol=1e-16)
    y = np.arange(ny)
    exact = U * (y + 0.5) / ny                 # walls at y = -1/2 and ny - 1/2
    ux = u[0].reshape(ny, 3)
    assert np.allclose(ux, exact[:, None], rtol=0, atol=1e-13)
    assert np.max(np.abs(u[1])) < 1e-15


def test_couette_3d_linear_profile():
    ny, U = 10, 0.02
    wall = [[0, 0, 0] for _ in range(6)]
    wall[3] = [0, 0, U]                        # +y wall moves along z
    p = inputs.default_params(3, (2, ny, 2), tau=0.9, periodic=(1, 0, 1), wall_u=wall)
    s = oracle.Sim(p)
    u = _steady(s, tol=1e-16)
    y = np.arange(ny)
    uz = u[2].reshape(2, ny, 2)
    assert np.allclose(uz, (U * (y + 0.5) / ny)[None, :, None], atol=1e-13)


def _poiseuille(dim, tau, ny, g):
    n = (2, ny) if dim == 2 else (2, ny, 2)
    per = (1, 0, 1) if dim == 3 else (1, 0, 0)
    p = inputs.default_params(dim, n, tau=tau, periodic=per, body_force=(g, 0, 0))
    s = oracle.Sim(p)
    u = _steady(s, tol=1e-17)
    nu = (tau - 0.5) / 3.0
    y = np.arange(ny)
    exact = g / (2 * nu) * (y + 0.5) * (ny - 0.5 - y)
    ux = u[0].reshape(-1, ny, 2)[0, :, 0] + g / 2.0   # Eq. 7: u = u* + f/(2 rho0)
    return ux, exact


@pytest.mark.parametrize("dim", [2, 3])
def test_poiseuille_exact_at_magic_tau(dim):
    """Half-way bounce-back puts the wall exactly half-way when (tau-1/2)^2 = 3/16.
    What remains is of order |u| |f|: Eq. 6 takes p from u* while Eqs. 4 and 8 use the
    corrected u, a small mass source (pinned exactly by the mass-budget test); at any
    other tau the wall-slip error is of order 1e-3."""
    ux, exact = _poiseuille(dim, 0.5 + math.sqrt(3) / 4, 12, 1e-6)
    assert np.max(np.abs(ux - exact)) < 1e-7 * np.max(exact)
    ux8, exact8 = _poiseuille(dim, 0.8, 12, 1e-6)
    assert np.max(np.abs(ux8 - exact8)) > 1e-3 * np.max(exact8)


def test_poiseuille_second_order():
    errs = []
    for ny in (8, 16, 32):
        g = 1e-6 * (8 / ny) ** 2
        ux, exact = _poiseuille(2, 0.8, ny, g)
        errs.append(np.sqrt(np.mean((ux - exact) ** 2)) / np.sqrt(np.mean(exact ** 2)))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


@pytest.mark.parametrize("dim,n", [(2, (9, 7)), (3, (6, 5, 7))])
def test_mass_conserved_closed_cavity(dim, n):
    p = inputs.default_params(dim, n, tau=0.7)
    s = oracle.Sim(p)
    s.set_pdfs(inputs.random_pdfs(1, 9 if dim == 2 else 19, int(np.prod(n))))
    m0 = s.mass()
    s.step(50)
    assert abs(s.mass() - m0) < 1e-13


@pytest.mark.parametrize("dim,n", [(2, (9, 7)), (3, (6, 5, 7))])
def test_mass_budget_with_force(dim, n):
    """With a force f, one step changes sum_{alpha>=1} f_alpha at a node by
    rho0 w0 (|u|^2-|u*|^2)/(2 cs^2 tau) + (1-1/(2 tau)) w0 u.f/cs^2 (Eqs. 1, 6, 7, 8);
    streaming with resting walls moves mass without changing the total."""
    tau, rho0 = 0.7, 1.0
    w0 = 4 / 9 if dim == 2 else 1 / 3
    force = (2e-4, -1e-4, 5e-5)[:dim] + (0.0,) * (3 - dim)
    p = inputs.default_params(dim, n, tau=tau, body_force=force, rho0=rho0)
    s = oracle.Sim(p)
    s.set_pdfs(inputs.random_pdfs(2, 9 if dim == 2 else 19, int(np.prod(n))))
    m0 = s.mass()
    _, us, _ = s.fields()
    f = np.array(force[:dim])[:, None]
    u = us + f / (2 * rho0)
    dm = (rho0 * w0 * ((u * u).sum(0) - (us * us).sum(0)) / (2 * tau / 3)
          + (1 - 1 / (2 * tau)) * w0 * (u * f).sum(0) * 3)
    s.step(1)
    assert abs((s.mass() - m0) - dm.sum()) < 1e-15


@pytest.mark.parametrize("dim,n,per", [(2, (7, 6), (0, 0, 0)), (2, (5, 4), (1, 0, 0)),
                                       (3, (5, 4, 6), (0, 0, 0)), (3, (4, 5, 3), (1, 0, 1))])
def test_swap_equals_two_array(dim, n, per):
    """The swap scheme moves the same post-collision values as two-array streaming
    (Sec. 3.3), including walls that move."""
    wall = [[0, 0, 0] for _ in range(6)]
    wall[3] = [0.01, 0, 0.005]
    wall[0] = [0, 0.003, 0]
    common = dict(tau=0.75, periodic=per, wall_u=wall, body_force=(1e-5, 2e-5, 0.0))
    q = 9 if dim == 2 else 19
    f0 = inputs.random_pdfs(5, q, int(np.prod(n)))
    a = oracle.Sim(inputs.default_params(dim, n, streaming=0, **common))
    b = oracle.Sim(inputs.default_params(dim, n, streaming=1, **common))
    a.set_pdfs(f0)
    b.set_pdfs(f0)
    a.step(7)
    b.step(7)
    assert np.array_equal(a.get_pdfs(), b.get_pdfs())


def _channel(dim, n, tau, U, periodic=(0, 0, 0), u_in=None):
    """Inflow (velocity, -y face) and outflow (pressure 0, +y face) by non-equilibrium
    extrapolation (Sec. 6.1); the other faces as given."""
    p = inputs.default_params(dim, n, tau=tau, storage="f64", mdf_iters=0, periodic=periodic)
    p["face_bc"] = (0, 0, 1, 2, 0, 0)
    wall = [[0.0, 0.0, 0.0] for _ in range(6)]
    wall[2] = list(u_in) if u_in is not None else [0.0, U, 0.0]
    p["wall_u"] = wall
    return p


@pytest.mark.parametrize("dim", [2, 3])
def test_uniform_stream_is_a_fixed_point_of_the_extrapolated_faces(dim):
    """A uniform stream at zero pressure between a velocity inlet and a pressure outlet
    (periodic across) is an equilibrium state with no gradients: the step must leave it
    unchanged."""
    n = (24, 40, 1) if dim == 2 else (10, 14, 8)
    per = (1, 0, 0) if dim == 2 else (1, 0, 1)
    u_in = [0.01, 0.03, 0.0] if dim == 2 else [0.01, 0.03, -0.02]
    p = _channel(dim, n[:dim], 0.7, 0.0, periodic=per, u_in=u_in)
    s = oracle.Sim(p)
    _, u = inputs.smooth_fields(0, dim, n, amp_u=0.0, amp_p=0.0)
    for a in range(dim):
        u[a] = u_in[a]
    s.set_equilibrium(None, u)
    f0 = s.get_pdfs().copy()
    s.step(50)
    assert np.abs(s.get_pdfs() - f0).max() < 1e-15


def test_channel_with_inflow_and_outflow_develops_poiseuille_flow():
    """Walls across x, inflow at the bottom and outflow at the top (Sec. 6.1): the steady
    flow has the same flux through every row, a uniform pressure across the section, the
    parabolic profile of the mean velocity ubar, and the Poiseuille pressure gradient
    dp/dy = -12 nu rho0 ubar / H^2 with H the wall distance (walls half-way outside the
    first and last nodes)."""
    nx, ny, tau, U = 16, 96, 0.8, 0.01
    s = oracle.Sim(_channel(2, (nx, ny), tau, U))
    _, u = inputs.smooth_fields(0, 2, (nx, ny, 1), amp_u=0.0, amp_p=0.0)
    u[1] = U
    s.set_equilibrium(None, u)
    s.step(6000)
    p, u, _ = s.fields()
    uy = u[1].reshape(ny, nx)
    pr = p.reshape(ny, nx)
    flux = uy[1:-1].sum(1)
    assert np.abs(flux - flux.mean()).max() < 1e-6 * flux.mean()
    ubar = uy[48].mean()
    assert 0.9 * U < ubar < 1.01 * U
    H, nu = float(nx), (tau - 0.5) / 3.0
    x = np.arange(nx) + 0.5
    par = 1.5 * ubar * (1.0 - ((x - H / 2) / (H / 2)) ** 2)
    assert np.abs(uy[48] - par).max() < 5e-3 * par.max()
    assert pr[48].std() < 1e-9 * abs(pr[48].mean()) + 1e-12
    dpdy = (pr[60].mean() - pr[36].mean()) / 24.0
    assert abs(dpdy / (-12.0 * nu * ubar / H ** 2) - 1.0) < 5e-3


def test_extrapolated_faces_must_share_one_axis():
    """Inflow and outflow faces on two different axes are refused."""
    p = _channel(2, (20, 20), 0.8, 0.01)
    p["face_bc"] = (2, 0, 1, 0, 0, 0)
    with pytest.raises(ValueError):
        oracle.Sim(p)
