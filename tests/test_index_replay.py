"""The kernels' index arithmetic (csrc/index_math.h) replayed on the host, built with
AddressSanitizer and UndefinedBehaviorSanitizer (float-cast-overflow included), over
particle states that reach every corner of it: the states of oracle runs that diverge
(the single thickened forcing pass at near contact, 2-D and 3-D, until positions become
huge, infinite or NaN), and constructed extremes (centres at +-1e18, +-inf, NaN, near
+-2^31 and +-2^24, outside the lattice by a few nodes, on the walls).  Every support
node must fall inside its LDS box, the lattice and the kernel's reach; cells, the
pair-search window and the interior box must stay inside their arrays."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2002_08855_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "index_replay.hip")


@pytest.fixture(scope="module")
def replay_bin(tmp_path_factory):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("replay") / "index_replay")
    # sanitizers on the host code only (the program runs no device code)
    cmd = ["hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xarch_host", "-fsanitize=address,undefined,float-cast-overflow",
           "-Xarch_host", "-fno-sanitize-recover=all", SRC, "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


def _cells(dim, n, D):
    """cell grid of Eqs. 49-50 as the library chooses it (the midpoint of the window)"""
    zeta = 1.0
    lo, hi = 0.5 * (D + zeta), D / math.sqrt(dim)
    H = 0.5 * (lo + hi) if lo < hi else 1.05 * lo
    nc = [max(1, int(math.floor(n[a] / H))) if a < dim else 1 for a in range(3)]
    invh = [nc[a] / n[a] if a < dim else 0.0 for a in range(3)]
    return nc, invh


def _write(path, dim, n, kind, cap, D, states, offsets):
    nc, invh = _cells(dim, n, D)
    with open(path, "w") as f:
        f.write(f"{dim} {n[0]} {n[1]} {n[2] if dim == 3 else 1} {kind} {cap} "
                f"{nc[0]} {nc[1]} {nc[2]} {invh[0]!r} {invh[1]!r} {invh[2]!r}\n")
        f.write(f"{len(states)}\n")
        for X in states:
            f.write(f"{len(X)}\n")
            for x in X:
                f.write(" ".join(repr(float(v)) for v in x) + f" {0.5 * D!r} {len(offsets)}\n")
                f.write(" ".join(repr(float(v)) for v in offsets.ravel()) + "\n")


def _run(binpath, path):
    r = subprocess.run([binpath, path], capture_output=True, text=True, timeout=600)
    print(r.stdout, r.stderr[-2000:])
    assert r.returncode == 0, r.stderr[-2000:]
    sup, nodes, skipped = (int(v) for v in r.stdout.split()[1:4])
    return sup, nodes, skipped


EXTREMES = [1e18, -1e18, math.inf, -math.inf, math.nan, 2.0 ** 31 - 2.5, -(2.0 ** 31) + 1.5,
            2.0 ** 31 + 7.0, 2.0 ** 24 - 3.25, -(2.0 ** 24) + 2.75, 2.0 ** 24 + 0.5]


def _extreme_states(dim, n, D):
    R = 0.5 * D
    base = np.array([n[0] / 2, n[1] / 2, n[2] / 2 if dim == 3 else 0.0])
    states = []
    for v in EXTREMES:
        for axis in range(dim):
            X = base.copy()
            X[axis] = v
            states.append([X])
        states.append([np.where(np.arange(3) < dim, v, 0.0)])
    # a few nodes outside the lattice, on the walls, and at the far corner
    for axis in range(dim):
        for v in (-R - 3.0, -0.5 + R, -0.5, n[axis] - 0.5 - R, n[axis] - 0.5, n[axis] + R + 2.0,
                  n[axis] - 1e-12):
            X = base.copy()
            X[axis] = v
            states.append([X])
    return states


def _diverging_states(dim, n, D, X0, steps):
    p = inputs.default_params(dim, n, tau=0.6, storage="f64", delta=1, drs=1.9, mdf_iters=1,
                              gravity=(0.0, -1e-5, 0.0))
    o = oracle.Sim(p)
    o.add_particles(X0, np.full(len(X0), D), np.full(len(X0), 1.5), n_markers=0)
    offsets = o.markers()["r"][: o.markers()["owner"].tolist().count(0)]
    states = []
    for s in range(steps):
        o.step(1)
        X = o.particles()["X"]
        states.append(X.copy())
    return states, offsets


def test_replay_2d_diverging_and_extreme_states(replay_bin, tmp_path):
    """2-D: the 256^2 analogue of the dense thickened-shell workload (40% area fraction,
    D = 20, gaps of 0.5 lu), whose oracle run diverges within 60 steps, then the
    constructed extremes; 3-point and 4-point supports."""
    n = (256, 256)
    D = 20.0
    count = int(round(0.40 * n[0] * n[1] / (math.pi * D * D / 4)))
    X0 = inputs.rsa(seed=2, dim=2, n=n, count=count, diameter=D, gap=0.5, clearance=2.5)
    states, offsets = _diverging_states(2, n, D, X0, 60)
    last = states[-1]
    assert not np.all(np.isfinite(last)) or np.abs(last).max() > 1e3, "the run did not diverge"
    states += _extreme_states(2, n, D)
    for kind in (1, 0):
        path = str(tmp_path / f"s2_{kind}.txt")
        _write(path, 2, n, kind, 2 * 4096, D, states, offsets)
        sup, nodes, _ = _run(replay_bin, path)
        assert sup > 0 and nodes > 0


def test_replay_3d_diverging_and_extreme_states(replay_bin, tmp_path):
    """3-D: spheres of D = 12 packed with gaps of 0.5 lu in a 48^3 cavity under the single
    thickened pass, followed until the oracle run diverges, then the extremes."""
    n = (48, 48, 48)
    D = 12.0
    X0 = inputs.rsa(seed=4, dim=3, n=n, count=20, diameter=D, gap=0.5, clearance=2.5)
    states, offsets = _diverging_states(3, n, D, X0, 40)
    states += _extreme_states(3, n, D)
    for kind in (1, 0):
        path = str(tmp_path / f"s3_{kind}.txt")
        _write(path, 3, n, kind, 24 * 24 * 24, D, states, offsets)
        sup, nodes, _ = _run(replay_bin, path)
        assert sup > 0 and nodes > 0
