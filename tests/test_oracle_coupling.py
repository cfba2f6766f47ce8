"""The oracle's particle coupling (Sec. 2.3, Eqs. 14-16) pinned piece by piece: the
Newton-Euler recurrence, the interior-fluid momentum behind F_f and T_f, the hydrodynamic
load and torque, the wall images of Eq. 16 and the gap feature (pins in
coupling_pins.py), and the paper's own particle-laden setting (Sec. 6.2, Table 7: the
3-point kernel, a shell of drs = 1.9, one forcing pass, density ratio 1.01) settling with
bounded velocities in the oracle."""
import numpy as np
import pytest

import coupling_pins as pins
import oracle
from paper_2002_08855_amd import inputs


@pytest.mark.parametrize("pin", pins.ALL, ids=lambda f: f.__name__)
def test_coupling_pin(pin):
    pin()


def _settle(dim, n, X, D, steps, every):
    """the paper's settling setting: 3-point kernel, drs = 1.9, one pass, ratio 1.01"""
    p = inputs.default_params(dim, n, tau=0.6, storage="f64", delta=1, drs=1.9, mdf_iters=1)
    o = oracle.Sim(p)
    o.add_particles(X, np.full(len(X), D), np.full(len(X), 1.01), n_markers=0)
    umax = []
    for _ in range(steps // every):
        o.step(every)
        pp = o.particles()
        assert np.all(np.isfinite(pp["U"])) and np.all(np.isfinite(pp["Omega"]))
        umax.append(float(np.abs(pp["U"]).max()))
    return umax, o


def test_paper_settling_setting_2d_stable():
    """Table 7 2-D (D = 16, 1000 disks in 2048^2, area fraction 4.8%) at the same area
    fraction in a 256^2 cavity (16 disks on a jittered grid of pitch 64): 500 steps, the
    particles accelerate smoothly from rest and stay far below one lattice unit per step
    (the terminal velocity of a disk of density ratio 1.01 under g = 1e-5 is of order
    1e-4)."""
    X = inputs.jittered_grid(seed=5, nx=4, ny=4, pitch=64.0, origin=32.0, jitter=8.0)
    umax, o = _settle(2, (256, 256), X, 16.0, 500, 50)
    print("max |U| every 50 steps", umax)
    assert max(umax) < 1e-4
    # the velocity grows monotonically while the particles accelerate from rest
    assert all(b >= a for a, b in zip(umax, umax[1:]))


def test_paper_settling_setting_2d_dense_stable():
    """Table 7 2-D at the dense end (area fraction 44%): 144 disks of D = 16 on a jittered
    square lattice of pitch 21.3 (surface gaps of at least 3.3 lu) in 256^2, 300 steps
    bounded."""
    X = inputs.jittered_grid(seed=7, nx=12, ny=12, pitch=256.0 / 12, origin=128.0 / 12, jitter=1.0)
    umax, _ = _settle(2, (256, 256), X, 16.0, 300, 50)
    print("max |U| every 50 steps", umax)
    assert max(umax) < 1e-3


def test_paper_settling_setting_3d_stable():
    """Table 7 3-D (D = 12 in 150^3, 100 spheres: volume fraction 2.7%) at a similar
    fraction in a 48^3 cavity (4 spheres), for the paper's 200 steps, bounded."""
    X = inputs.jittered_grid(seed=3, nx=2, ny=2, pitch=24.0, origin=12.0, jitter=2.0)
    X[:, 2] = 24.0
    umax, _ = _settle(3, (48, 48, 48), X, 12.0, 200, 50)
    print("max |U| every 50 steps", umax)
    assert max(umax) < 1e-4


def test_paper_settling_setting_3d_dense_stable():
    """Table 7 3-D towards its dense end: 27 spheres of D = 12 on the cubic lattice of the
    particle-count series (pitch 15, jitter 0.5, so surface gaps of at least 2 lu) in a
    60^3 cavity (volume fraction 0.11, between the series' 300 and 600 spheres), the
    paper's 200 steps, bounded."""
    X = inputs.lattice_pick(seed=8, dim=3, n=(60, 60, 60), count=27, diameter=12.0, pitch=15.0,
                            clearance=2.5, jitter=0.5)
    umax, _ = _settle(3, (60, 60, 60), X, 12.0, 200, 50)
    print("max |U| every 50 steps", umax)
    assert max(umax) < 1e-3
