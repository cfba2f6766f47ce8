"""Seeded synthetic inputs for the IB-LBM step: parameter presets, particle placement
and random initial states.

This module holds none of the method's arithmetic.  It produces numbers (positions,
random PDF deviations, parameter sets) that are handed unchanged to both the GPU
library and the CPU oracle.  All randomness comes from one SplitMix64 stream per seed
(Steele, Lea & Flood 2014: state += 0x9E3779B97F4A7C15, then two xor-shift-multiply
rounds), so placements are reproducible on any machine.

The paper's workload is particles settling in a closed cavity (Sec. 6.2): a synthetic
setup with no dataset.  The presets below carry the sizes of the five workloads the
IB-LBM step is measured on; their derivation is described next to each.
"""
from __future__ import annotations

import math

import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


class SplitMix64:
    """Counter-based SplitMix64 generator (vectorised over numpy uint64)."""

    def __init__(self, seed: int):
        self.state = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)

    def next_u64(self, n: int) -> np.ndarray:
        with np.errstate(over="ignore"):
            k = np.arange(1, n + 1, dtype=np.uint64)
            s = self.state + k * np.uint64(0x9E3779B97F4A7C15)
            self.state = s[-1] if n > 0 else self.state
            z = s
            z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
            z = z ^ (z >> np.uint64(31))
        return z

    def uniform(self, n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
        u = (self.next_u64(n) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
        return lo + (hi - lo) * u


# ---------------------------------------------------------------------------
# parameter presets

def default_params(dim: int, n, **kw) -> dict:
    p = dict(
        dim=dim,
        n=tuple(list(n) + [1] * (3 - len(n))),
        tau=0.8,
        rho0=1.0,
        body_force=(0.0, 0.0, 0.0),
        periodic=(0, 0, 0),
        wall_u=[[0.0, 0.0, 0.0] for _ in range(6)],
        delta=0,            # Peskin 4-point
        drs=1.0,
        mdf_iters=3,
        gravity=(0.0, -1e-5, 0.0),
        zeta=1.0,
        eps_pp=1e-3,
        E_pp=1e-4,
        cell_h=0.0,
        storage="f64",
        f16_scale=1024.0,
        forcing=0,
        slip_tol=1e30,
        fallback_iters=5,
    )
    p.update(kw)
    return p


def workload(name: str) -> dict:
    """Parameters and particle set of a named workload.

    cavity128_f64     : 2-D 128^2 D2Q9 cavity, FP64, tau 0.8, 16 disks D=10, 32 points,
                        density ratio 1.5, MDF-3, jittered 4x4 grid, 1000 steps.
    cavity2048_f32    : 2-D 2048^2, FP32, tau 0.6, area fraction 0.40: 5340 disks D=20,
                        64 points, ratio 1.5, random sequential addition, 500 steps.
    cavity2048_free   : the same cavity without particles.
    cavity2048_sparse : 2-D 2048^2, FP32, tau 0.8: the 128^2 layout tiled 16 x 16 (4096
                        disks D=10 on a jittered grid of pitch 32, 32 points, ratio 1.5,
                        area fraction 0.077).
    cavity8192_free   : 2-D 8192^2 FP32 cavity without particles (2.1 GB of PDFs, far
                        beyond the last-level cache: the collide-stream kernel against HBM).
    cavity256_free    : 3-D 256^3 FP32 cavity without particles.
    cavity256_f32     : 3-D 256^3 D3Q19, FP32, tau 0.7, volume fraction 0.20: 1565
                        spheres D=16, 804 points, ratio 2.0, 200 steps.
    cavity384_bf16/_f16: 3-D 384^3, volume fraction 0.40: 25033 spheres D=12, 452 points,
                        ratio 2.0, BF16/FP16 PDF storage, 200 steps (FCC + deletion).
    cavity256_learned : 3-D 256^3, volume fraction 0.30: 2347 spheres D=16, learned
                        forcing, 200 steps (FCC + deletion).
    cavity256_train   : the training source of the learned forcing: cavity256_f32's shape
                        (1565 spheres, 0.20, random sequential addition) with seed 103,
                        plain MDF-5.
    cavity256_train30 : the second training source: 2347 spheres D=16 (0.30) on a
                        10-cell FCC lattice thinned with seed 105, plain MDF-5.
    np2d_<Np> / np3d_<Np>: the particle-count series of Table 7: 2048^2 FP32 with Np
                        disks D=16 (Np <= 10^4), 150^3 FP32 with Np spheres D=12 (Np <= 600),
                        round(pi D) / round(pi D^2) points, ratio 1.5, MDF-3, on a thinned
                        square or cubic lattice (pitch 20 / 15, jitter 1).
    np2d_<Np>_paper / np3d_<Np>_paper: the same series in the paper's setting of Sec. 6.2:
                        3-point kernel, drs = 1.9, one forcing pass, density ratio 1.01
                        (3-D jitter 0.5, so that surface gaps stay at 2 lu or more).
    res2d_<D> / res3d_<D>: the resolution series of Sec. 6.2.2: a 40 D square with 400
                        disks (20 x 20 grid, pitch 2 D) / a 5 D cube with 27 spheres (pitch
                        5 D / 3), diameter D, FP32, ratio 1.5, MDF-3.
    channel2d_<n> / channel3d_<n>: the particle-free flow of Sec. 6.1 on n^2 / n^3 nodes,
                        FP32, tau 0.6: inflow at the bottom (uniform 0.01 lattice units
                        per step) and outflow at the top (pressure 0) by non-equilibrium
                        extrapolation, bounce-back walls on the other faces.
    <name>_btdf       : the workload <name> with the single-pass boundary-thickened direct
                        forcing of Sec. 2.2: the 3-point kernel, shell thickness drs = 1.9
                        lattice units, one forcing pass (the paper's setting for its
                        particle-laden runs, Sec. 6.2).
    """
    if name.startswith("np2d_") or name.startswith("np3d_"):
        # the particle-count series of Table 7 (Sec. 6.2.1): 2048^2 with D = 16 up to 10^4
        # disks, 150^3 with D = 12 up to 600 spheres; plain MDF-3, density ratio 1.5.
        # With the suffix _paper: the paper's own setting of Sec. 6.2 (the 3-point kernel,
        # a shell of drs = 1.9, one forcing pass, density ratio 1.01), on lattices whose
        # surface gaps stay at 2 lu or more (3-D jitter 0.5)
        dim = 2 if name.startswith("np2d_") else 3
        paper = name.endswith("_paper")
        count = int(name.split("_")[1])
        if dim == 2:
            p = default_params(2, (2048, 2048), tau=0.6, storage="f32", mdf_iters=3)
            X = lattice_pick(seed=7, dim=2, n=(2048, 2048), count=count, diameter=16.0,
                             pitch=20.0, clearance=2.5, jitter=1.0)
            D = 16.0
        else:
            p = default_params(3, (150, 150, 150), tau=0.7, storage="f32", mdf_iters=3)
            X = lattice_pick(seed=8, dim=3, n=(150, 150, 150), count=count, diameter=12.0,
                             pitch=15.0, clearance=2.5, jitter=0.5 if paper else 1.0)
            D = 12.0
        rho = 1.5
        if paper:
            p.update(delta=1, drs=1.9, mdf_iters=1)
            rho = 1.01
        parts = dict(center=X, diameter=np.full(count, D), density=np.full(count, rho),
                     n_markers=0)
        return dict(params=p, particles=parts, steps=1000 if dim == 2 else 200)
    if name.startswith("res2d_") or name.startswith("res3d_"):
        # the resolution series of Sec. 6.2.2: a 40 D square / 5 D cube with the particle
        # diameter D in lattice units; the number of particles (400 / 27) and so the
        # volume fraction (0.20 / 0.11) stay fixed
        dim = 2 if name.startswith("res2d_") else 3
        D = float(name.split("_")[1])
        if dim == 2:
            n = int(round(40 * D))
            p = default_params(2, (n, n), tau=0.6, storage="f32", mdf_iters=3)
            X = jittered_grid(seed=9, nx=20, ny=20, pitch=2 * D, origin=D, jitter=1.0)
        else:
            n = int(round(5 * D))
            p = default_params(3, (n, n, n), tau=0.7, storage="f32", mdf_iters=3)
            X = jittered_grid(seed=10, nx=3, ny=3, pitch=5 * D / 3, origin=5 * D / 6,
                              jitter=1.0, nz=3)
        parts = dict(center=X, diameter=np.full(len(X), D), density=np.full(len(X), 1.5),
                     n_markers=0)
        return dict(params=p, particles=parts, steps=200)
    if name.startswith("channel2d_") or name.startswith("channel3d_"):
        dim = 2 if name.startswith("channel2d_") else 3
        n = int(name.split("_")[1])
        p = default_params(dim, (n,) * dim, tau=0.6, storage="f32", mdf_iters=0)
        p["face_bc"] = (0, 0, 1, 2, 0, 0)
        wall = [[0.0, 0.0, 0.0] for _ in range(6)]
        wall[2] = [0.0, 0.01, 0.0]
        p["wall_u"] = wall
        return dict(params=p, particles=None, steps=200)
    if name.endswith("_btdf"):
        w = workload(name[:-len("_btdf")])
        w["params"] = dict(w["params"], delta=1, drs=1.9, mdf_iters=1)
        return w
    if name == "cavity128_f64":
        p = default_params(2, (128, 128), tau=0.8, storage="f64", mdf_iters=3)
        X = jittered_grid(seed=1, nx=4, ny=4, pitch=32.0, origin=16.0, jitter=5.0)
        parts = dict(center=X, diameter=np.full(len(X), 10.0), density=np.full(len(X), 1.5),
                     n_markers=32)
        return dict(params=p, particles=parts, steps=1000)
    if name in ("cavity2048_f32", "cavity2048_free"):
        p = default_params(2, (2048, 2048), tau=0.6, storage="f32", mdf_iters=3)
        if name == "cavity2048_free":
            return dict(params=p, particles=None, steps=500)
        X = rsa(seed=2, dim=2, n=(2048, 2048), count=5340, diameter=20.0, gap=0.5,
                clearance=2.5)
        parts = dict(center=X, diameter=np.full(len(X), 20.0), density=np.full(len(X), 1.5),
                     n_markers=64)
        return dict(params=p, particles=parts, steps=500)
    if name == "cavity2048_sparse":
        p = default_params(2, (2048, 2048), tau=0.8, storage="f32", mdf_iters=3)
        X = jittered_grid(seed=6, nx=64, ny=64, pitch=32.0, origin=16.0, jitter=5.0)
        parts = dict(center=X, diameter=np.full(len(X), 10.0), density=np.full(len(X), 1.5),
                     n_markers=32)
        return dict(params=p, particles=parts, steps=500)
    if name == "cavity8192_free":
        return dict(params=default_params(2, (8192, 8192), tau=0.6, storage="f32", mdf_iters=3),
                    particles=None, steps=200)
    if name == "cavity256_free":
        return dict(params=default_params(3, (256, 256, 256), tau=0.7, storage="f32", mdf_iters=3),
                    particles=None, steps=200)
    if name == "cavity256_f32":
        p = default_params(3, (256, 256, 256), tau=0.7, storage="f32", mdf_iters=3)
        X = rsa(seed=3, dim=3, n=(256, 256, 256), count=1565, diameter=16.0, gap=0.5,
                clearance=2.5)
        parts = dict(center=X, diameter=np.full(len(X), 16.0), density=np.full(len(X), 2.0),
                     n_markers=804)
        return dict(params=p, particles=parts, steps=200)
    if name in ("cavity384_bf16", "cavity384_f16"):
        st = "bf16" if name.endswith("bf16") else "f16"
        p = default_params(3, (384, 384, 384), tau=0.7, storage=st, mdf_iters=3)
        X = fcc_fill(seed=4, n=384, cells=19, diameter=12.0, count=25033, clearance=1.0,
                     jitter=0.2)
        parts = dict(center=X, diameter=np.full(len(X), 12.0), density=np.full(len(X), 2.0),
                     n_markers=452)
        return dict(params=p, particles=parts, steps=200)
    if name == "cavity256_train":
        # the training runs of the learned forcing: the 256^3 plain workload's shape (volume
        # fraction 0.20, random sequential addition) with its own seed, plain MDF-5
        p = default_params(3, (256, 256, 256), tau=0.7, storage="f32", mdf_iters=5)
        X = rsa(seed=103, dim=3, n=(256, 256, 256), count=1565, diameter=16.0, gap=0.5,
                clearance=2.5)
        parts = dict(center=X, diameter=np.full(len(X), 16.0), density=np.full(len(X), 2.0),
                     n_markers=804)
        return dict(params=p, particles=parts, steps=200)
    if name == "cavity256_train30":
        # a second training packing at the evaluation's volume fraction 0.30: a finer FCC
        # lattice (10 cells, nearest-neighbour gap about 2 lu instead of 4) thinned with
        # its own seed, so that no training sphere sits on an evaluation site pattern
        p = default_params(3, (256, 256, 256), tau=0.7, storage="f32", mdf_iters=5)
        X = fcc_fill(seed=105, n=256, cells=10, diameter=16.0, count=2347, clearance=1.0,
                     jitter=0.5)
        parts = dict(center=X, diameter=np.full(len(X), 16.0), density=np.full(len(X), 2.0),
                     n_markers=804)
        return dict(params=p, particles=parts, steps=200)
    if name == "cavity256_learned":
        p = default_params(3, (256, 256, 256), tau=0.7, storage="f32", mdf_iters=5, forcing=1)
        # with the 0.5 gap and the wall clearance, random sequential addition at 0.30 is
        # close to jamming; a thinned FCC lattice reaches it at once
        X = fcc_fill(seed=5, n=256, cells=9, diameter=16.0, count=2347, clearance=1.0,
                     jitter=0.5)
        parts = dict(center=X, diameter=np.full(len(X), 16.0), density=np.full(len(X), 2.0),
                     n_markers=804)
        return dict(params=p, particles=parts, steps=200)
    raise KeyError(name)


# ---------------------------------------------------------------------------
# placements (centres in FP64, lattice units; walls at -1/2 and n - 1/2)

def jittered_grid(seed, nx, ny, pitch, origin, jitter, nz=None):
    rng = SplitMix64(seed)
    pts = []
    for j in range(ny):
        for i in range(nx):
            if nz is None:
                pts.append((origin + pitch * i, origin + pitch * j, 0.0))
            else:
                for k in range(nz):
                    pts.append((origin + pitch * i, origin + pitch * j, origin + pitch * k))
    X = np.array(pts, dtype=np.float64)
    dims = 2 if nz is None else 3
    X[:, :dims] += rng.uniform(len(X) * dims, -jitter, jitter).reshape(len(X), dims)
    return X


def lattice_pick(seed, dim, n, count, diameter, pitch, clearance, jitter):
    """`count` sites drawn without replacement (seeded) from a square or cubic lattice of
    the given pitch inside the wall-cleared box, each jittered uniformly by up to
    `jitter` per axis (pitch - diameter >= 2 jitter keeps the particles apart)."""
    rng = SplitMix64(seed)
    R = 0.5 * diameter
    lo = -0.5 + R + clearance + jitter
    axes = []
    for a in range(dim):
        hi = n[a] - 0.5 - R - clearance - jitter
        m = int(math.floor((hi - lo) / pitch)) + 1
        axes.append(lo + pitch * np.arange(m) + 0.5 * ((hi - lo) - pitch * (m - 1)))
    grid = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, dim)
    if count > len(grid):
        raise ValueError("not enough lattice sites")
    order = np.argsort(rng.uniform(len(grid)), kind="stable")[:count]
    X = np.zeros((count, 3))
    X[:, :dim] = grid[np.sort(order)] + rng.uniform(count * dim, -jitter, jitter).reshape(count, dim)
    return X


def rsa(seed, dim, n, count, diameter, gap, clearance, max_attempts=50_000_000):
    """Random sequential addition of equal particles: uniform candidates, kept when
    the surface gap to every kept particle is >= gap and to every wall >= clearance."""
    rng = SplitMix64(seed)
    R = 0.5 * diameter
    lo = -0.5 + R + clearance
    hi = np.array([n[a] - 0.5 - R - clearance for a in range(dim)])
    dmin2 = (diameter + gap) ** 2
    cell = diameter + gap
    ncell = [max(1, int(math.ceil((n[a] + 1) / cell))) for a in range(dim)]
    grid: dict = {}
    out = np.zeros((count, 3))
    m = 0
    batch = 4096
    attempts = 0
    while m < count:
        cand = rng.uniform(batch * dim).reshape(batch, dim)
        cand = lo + cand * (hi - lo)
        for c in cand:
            attempts += 1
            key = tuple(int((c[a] + 0.5) // cell) for a in range(dim))
            ok = True
            rngs = [range(max(0, key[a] - 1), min(ncell[a], key[a] + 2)) for a in range(dim)]
            if dim == 2:
                neigh = ((i, j) for i in rngs[0] for j in rngs[1])
            else:
                neigh = ((i, j, k) for i in rngs[0] for j in rngs[1] for k in rngs[2])
            for nk in neigh:
                for idx in grid.get(nk, ()):
                    d = out[idx, :dim] - c
                    if float(d @ d) < dmin2:
                        ok = False
                        break
                if not ok:
                    break
            if ok:
                out[m, :dim] = c
                grid.setdefault(key, []).append(m)
                m += 1
                if m == count:
                    break
        if attempts > max_attempts:
            raise RuntimeError(f"RSA stalled at {m} of {count} particles")
    return out


def fcc_fill(seed, n, cells, diameter, count, clearance, jitter):
    """Face-centred cubic sites, `cells` conventional cells per axis fitted between
    the walls (wall clearance of the surfaces >= clearance), thinned to `count` by a
    seeded random deletion, then jittered by up to `jitter` per axis."""
    rng = SplitMix64(seed)
    R = 0.5 * diameter
    lo = -0.5 + R + clearance + jitter
    hi = n - 0.5 - R - clearance - jitter
    a = (hi - lo) / (cells - 0.5)
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    idx = np.stack(np.meshgrid(np.arange(cells), np.arange(cells), np.arange(cells),
                               indexing="ij"), -1).reshape(-1, 3)
    sites = (idx[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a + lo
    keys = rng.uniform(len(sites))
    keep = np.sort(np.argsort(keys, kind="stable")[:count])
    X = sites[keep]
    X = X + rng.uniform(X.size, -jitter, jitter).reshape(X.shape)
    return X


# ---------------------------------------------------------------------------
# random states

def random_pdfs(seed, q, N, amplitude=1e-3):
    """Random PDF deviations from the rest state, (q-1) x N, uniform in
    [-amplitude, amplitude]."""
    rng = SplitMix64(seed)
    return rng.uniform((q - 1) * N, -amplitude, amplitude).reshape(q - 1, N)


def smooth_fields(seed, dim, n, amp_u=1e-2, amp_p=1e-3):
    """Smooth random pressure and velocity: a few low Fourier modes with seeded
    amplitudes and phases.  Returns p (N), u (dim x N)."""
    rng = SplitMix64(seed)
    nz = n[2] if dim == 3 else 1
    z, y, x = np.meshgrid(np.arange(nz), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    coords = [x.ravel().astype(float), y.ravel().astype(float), z.ravel().astype(float)]

    def field(amp):
        out = np.zeros(coords[0].size)
        for _ in range(3):
            c = rng.uniform(4)
            kx, ky, kz = 1 + int(3 * c[0]), 1 + int(3 * c[1]), 1 + int(3 * c[2])
            ph = 2 * math.pi * c[3]
            arg = (2 * math.pi * kx * coords[0] / n[0] + 2 * math.pi * ky * coords[1] / n[1]
                   + (2 * math.pi * kz * coords[2] / nz if dim == 3 else 0.0) + ph)
            out += amp * np.sin(arg)
        return out

    p = field(amp_p)
    u = np.stack([field(amp_u) for _ in range(dim)])
    return p, u
