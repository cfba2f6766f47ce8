"""Plain FP64 CPU oracle of the IB-LBM time step (arXiv 2002.08855).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It wraps the C library
built from ``iblbm_ref.c`` (FP64, ``-ffp-contract=off``) and shares no code with the GPU
library in ``paper_2002_08855_amd``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libiblbm_ref.so")

NPARAM = 10 * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3


CFLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-Wall", "-Wno-unknown-pragmas"]


def compiler_version() -> str:
    r = subprocess.run(["gcc", "--version"], capture_output=True, text=True)
    return r.stdout.splitlines()[0] if r.returncode == 0 and r.stdout else "gcc"


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (always recompiles)."""
    src = os.path.join(HERE, "iblbm_ref.c")
    cmd = ["gcc", *CFLAGS, src, "-o", LIB_PATH + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class RefConfig(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("n", C.c_int32 * 3), ("tau", C.c_double), ("rho0", C.c_double),
        ("body_force", C.c_double * 3), ("periodic", C.c_int32 * 3),
        ("wall_u", (C.c_double * 3) * 6), ("delta", C.c_int32), ("drs", C.c_double),
        ("mdf_iters", C.c_int32), ("gravity", C.c_double * 3), ("zeta", C.c_double),
        ("eps_pp", C.c_double), ("E_pp", C.c_double), ("cell_h", C.c_double),
        ("streaming", C.c_int32), ("forcing", C.c_int32), ("slip_tol", C.c_double),
        ("fallback_iters", C.c_int32), ("face_bc", C.c_int32 * 6), ("face_p", C.c_double * 6),
    ]


_lib = None
_P = C.POINTER
_d = _P(C.c_double)
_i32 = _P(C.c_int32)


def load(path):
    """A ctypes handle of an oracle library at `path`, with the signatures set."""
    L = C.CDLL(path)
    if True:
        sig = {
            "ref_lattice": (C.c_int32, [C.c_int32, _i32, _d]),
            "ref_feq": (None, [C.c_int32, C.c_double, C.c_double, _d, _d]),
            "ref_guo_force": (None, [C.c_int32, C.c_double, _d, _d, _d]),
            "ref_macro": (None, [C.c_int32, C.c_double, _d, _d, _d]),
            "ref_phi": (C.c_double, [C.c_int32, C.c_double]),
            "ref_pair_force": (C.c_double, [C.c_double] * 6),
            "ref_ibm_interp": (None, [C.c_int32, _i32, _i32, C.c_int32, _d, C.c_int32, _d, _d,
                                      C.c_int32]),
            "ref_ibm_spread": (None, [C.c_int32, _i32, _i32, C.c_int32, _d, _d, C.c_int32, _d, _d,
                                      C.c_int32]),
            "ref_half_search": (C.c_int64, [C.c_int32, C.c_int32, _d, _d, C.c_double, _i32,
                                            C.c_int64]),
            "ref_grid_search": (C.c_int64, [C.c_int32, _i32, C.c_int32, _d, _d, C.c_double,
                                            C.c_double, _i32, C.c_int64]),
            "ref_create": (C.c_void_p, [_P(RefConfig)]),
            "ref_destroy": (None, [C.c_void_p]),
            "ref_set_equilibrium": (C.c_int32, [C.c_void_p, _d, _d]),
            "ref_set_pdfs": (C.c_int32, [C.c_void_p, _d]),
            "ref_get_pdfs": (C.c_int32, [C.c_void_p, _d]),
            "ref_add_particles": (C.c_int32, [C.c_void_p, C.c_int32, _d, _d, _d, _d, _d,
                                              C.c_int32]),
            "ref_step": (C.c_int32, [C.c_void_p, C.c_int32]),
            "ref_get_fields": (C.c_int32, [C.c_void_p, _d, _d, _d]),
            "ref_get_particles": (C.c_int32, [C.c_void_p, _d, _d, _d, _d, _d, _d]),
            "ref_get_markers": (C.c_int32, [C.c_void_p, _d, _d, _i32, _d]),
            "ref_num_markers": (C.c_int32, [C.c_void_p]),
            "ref_get_pairs": (C.c_int64, [C.c_void_p, _i32, C.c_int64]),
            "ref_get_cells": (C.c_int32, [C.c_void_p, _i32, _i32, _d]),
            "ref_mass": (C.c_double, [C.c_void_p]),
            "ref_slip_rms": (C.c_double, [C.c_void_p]),
            "ref_truncated": (C.c_int64, [C.c_void_p]),
            "ref_fallbacks": (C.c_int32, [C.c_void_p]),
            "ref_judged_slip": (C.c_double, [C.c_void_p]),
            "ref_mlp_forward": (None, [_d, C.c_int64, _d, _d]),
            "ref_mlp_predict": (None, [_d, _d, C.c_int64, C.c_int32, _d, _d, _d]),
            "ref_mlp_loss_grad": (C.c_double, [_d, C.c_int64, _d, _d, _d]),
            "ref_set_mlp": (C.c_int32, [C.c_void_p, _d, _d]),
            "ref_capture_samples": (C.c_int32, [C.c_void_p, _d, _d]),
            "ref_particle_loads": (None, [C.c_int32, _d, _d, _d, _d, _d]),
            "ref_interior_momentum": (None, [C.c_int32, _i32, _d, C.c_double, C.c_double, _d, _d,
                                             _d]),
            "ref_newton_euler": (None, [C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double]
                                 + [_d] * 13),
            "ref_pair_forces": (None, [C.c_int32, _i32, _i32, C.c_int32, _d, _d, _d, C.c_double,
                                       C.c_double, C.c_double, _i32, C.c_int64, _d]),
            "ref_point_gap": (C.c_double, [C.c_int32, _i32, _i32, C.c_double, _d, C.c_int32, _d,
                                           _d, _i32, C.c_int64]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = load(LIB_PATH)
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(_d)


def _ip(a):
    return None if a is None else a.ctypes.data_as(_i32)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


# ---- pure functions --------------------------------------------------------

def lattice(dim):
    q = 9 if dim == 2 else 19
    e = np.zeros((q, 3), np.int32)
    w = np.zeros(q)
    lib().ref_lattice(dim, _ip(e), _dp(w))
    return e, w


def feq(dim, rho0, p, u):
    q = 9 if dim == 2 else 19
    out = np.zeros(q)
    u = _f64(np.resize(np.asarray(u, float), 3))
    lib().ref_feq(dim, rho0, p, _dp(u), _dp(out))
    return out


def guo_force(dim, tau, u, f):
    q = 9 if dim == 2 else 19
    out = np.zeros(q)
    u = _f64(np.resize(np.asarray(u, float), 3))
    f = _f64(np.resize(np.asarray(f, float), 3))
    lib().ref_guo_force(dim, tau, _dp(u), _dp(f), _dp(out))
    return out


def macro(dim, rho0, f):
    f = _f64(f)
    p = C.c_double()
    u = np.zeros(3)
    lib().ref_macro(dim, rho0, _dp(f), C.byref(p), _dp(u))
    return p.value, u


def phi(kind, r):
    return lib().ref_phi(kind, float(r))


def pair_force(d, D, zeta, c, eps_pp, E_pp):
    return lib().ref_pair_force(d, D, zeta, c, eps_pp, E_pp)


def ibm_interp(dim, n, periodic, kind, u, X, naive=False):
    n = np.asarray(n, np.int32)
    per = np.asarray(periodic, np.int32)
    u = _f64(u)
    X = _f64(X, (-1, 3))
    out = np.zeros((X.shape[0], 3))
    lib().ref_ibm_interp(dim, _ip(n), _ip(per), kind, _dp(u), X.shape[0], _dp(X), _dp(out),
                         int(naive))
    return out


def ibm_spread(dim, n, periodic, kind, F, dV, X, naive=False):
    n = np.asarray(n, np.int32)
    per = np.asarray(periodic, np.int32)
    F = _f64(F, (-1, 3))
    dV = _f64(dV)
    X = _f64(X, (-1, 3))
    N = int(np.prod(n))
    g = np.zeros(dim * N)
    lib().ref_ibm_spread(dim, _ip(n), _ip(per), kind, _dp(F), _dp(dV), X.shape[0], _dp(X),
                         _dp(g), int(naive))
    return g


def half_search(dim, X, D, zeta):
    X = _f64(X, (-1, 3))
    D = _f64(D)
    cap = 16
    while True:
        ij = np.zeros((cap, 2), np.int32)
        m = lib().ref_half_search(dim, X.shape[0], _dp(X), _dp(D), zeta, _ip(ij), cap)
        if m <= cap:
            return ij[:m].copy()
        cap = int(m)


def grid_search(dim, n, X, D, zeta, H):
    X = _f64(X, (-1, 3))
    D = _f64(D)
    n = np.asarray(n, np.int32)
    cap = 16 * max(1, X.shape[0])
    ij = np.zeros((cap, 2), np.int32)
    m = lib().ref_grid_search(dim, _ip(n), X.shape[0], _dp(X), _dp(D), zeta, H, _ip(ij), cap)
    if m < 0:
        return None
    assert m <= cap
    return ij[:m].copy()


def mlp_forward(params, x):
    params = _f64(params)
    x = _f64(x, (-1, 10))
    y = np.zeros((x.shape[0], 3))
    lib().ref_mlp_forward(_dp(params), x.shape[0], _dp(x), _dp(y))
    return y


def mlp_predict(params, norm, feat, Fprev, dim=3, L=None):
    """the learned force F = F_prev + target mean + target std * MLP(normalised features)"""
    params = _f64(params)
    norm = _f64(norm)
    feat = _f64(feat, (-1, 10))
    Fprev = _f64(Fprev, (-1, 3))
    F = np.zeros((feat.shape[0], 3))
    (L or lib()).ref_mlp_predict(_dp(params), _dp(norm), feat.shape[0], dim, _dp(feat),
                                 _dp(Fprev), _dp(F))
    return F


def mlp_loss_grad(params, x, t):
    params = _f64(params)
    x = _f64(x, (-1, 10))
    t = _f64(t, (-1, 3))
    g = np.zeros(NPARAM)
    loss = lib().ref_mlp_loss_grad(_dp(params), x.shape[0], _dp(x), _dp(t), _dp(g))
    return loss, g


# ---- particle coupling (Sec. 2.3) ---------------------------------------------
# Each takes an optional library handle L (from load()); the default is this package's.

def particle_loads(r, F, dV, L=None):
    r = _f64(r, (-1, 3))
    F = _f64(F, (-1, 3))
    dV = _f64(dV)
    Fh, Th = np.zeros(3), np.zeros(3)
    (L or lib()).ref_particle_loads(r.shape[0], _dp(r), _dp(F), _dp(dV), _dp(Fh), _dp(Th))
    return Fh, Th


def interior_momentum(dim, n, Xc, R, rho0, u, L=None):
    n = np.asarray(list(n) + [1] * (3 - len(n)), np.int32)
    Xc = _f64(np.resize(np.asarray(Xc, float), 3))
    u = _f64(u)
    P, Lm = np.zeros(3), np.zeros(3)
    (L or lib()).ref_interior_momentum(dim, _ip(n), _dp(Xc), float(R), float(rho0), _dp(u), _dp(P),
                                       _dp(Lm))
    return P, Lm


def newton_euler(dim, M, V, I, rho0, g, Fh, Th, Fc, P, Lm, state, L=None):
    """One step of Eqs. 14-15 for one particle.  `state` is a dict of 3-vectors Pprev,
    Lprev, Hprev, Gprev, X, U, Om, updated in place (and returned)."""
    args = [_f64(np.resize(np.asarray(a, float), 3)) for a in (g, Fh, Th, Fc, P, Lm)]
    for k in ("Pprev", "Lprev", "Hprev", "Gprev", "X", "U", "Om"):
        state[k] = _f64(np.resize(np.asarray(state[k], float), 3)).copy()
    (L or lib()).ref_newton_euler(dim, float(M), float(V), float(I), float(rho0),
                                  *[_dp(a) for a in args],
                                  *[_dp(state[k]) for k in ("Pprev", "Lprev", "Hprev", "Gprev", "X",
                                                            "U", "Om")])
    return state


def pair_forces(dim, n, periodic, X, D, c, zeta, eps_pp, E_pp, pairs, L=None):
    n = np.asarray(list(n) + [1] * (3 - len(n)), np.int32)
    per = np.asarray(periodic, np.int32)
    X = _f64(X, (-1, 3))
    ij = np.ascontiguousarray(np.asarray(pairs, np.int32).reshape(-1, 2))
    Fc = np.zeros((X.shape[0], 3))
    (L or lib()).ref_pair_forces(dim, _ip(n), _ip(per), X.shape[0], _dp(X), _dp(_f64(D)),
                                 _dp(_f64(c)), zeta, eps_pp, E_pp, _ip(ij), ij.shape[0], _dp(Fc))
    return Fc


def point_gap(dim, n, periodic, zeta, Xk, p, X, D, pairs, L=None):
    n = np.asarray(list(n) + [1] * (3 - len(n)), np.int32)
    per = np.asarray(periodic, np.int32)
    Xk = _f64(np.resize(np.asarray(Xk, float), 3))
    X = _f64(X, (-1, 3))
    ij = np.ascontiguousarray(np.asarray(pairs, np.int32).reshape(-1, 2))
    return (L or lib()).ref_point_gap(dim, _ip(n), _ip(per), zeta, _dp(Xk), int(p), _dp(X),
                                      _dp(_f64(D)), _ip(ij), ij.shape[0])


# ---- the time-stepping context ----------------------------------------------

def make_config(p: dict) -> RefConfig:
    """Fill the oracle's config struct from a plain parameter dict (see
    ``paper_2002_08855_amd.inputs.default_params``)."""
    c = RefConfig()
    c.dim = int(p["dim"])
    for a in range(3):
        c.n[a] = int(p["n"][a]) if a < len(p["n"]) else 1
        c.body_force[a] = float(p.get("body_force", (0, 0, 0))[a])
        c.periodic[a] = int(p.get("periodic", (0, 0, 0))[a])
        c.gravity[a] = float(p.get("gravity", (0, 0, 0))[a])
    for fce in range(6):
        for a in range(3):
            c.wall_u[fce][a] = float(p.get("wall_u", [[0, 0, 0]] * 6)[fce][a])
    c.tau = float(p["tau"])
    c.rho0 = float(p.get("rho0", 1.0))
    c.delta = int(p.get("delta", 0))
    c.drs = float(p.get("drs", 1.0))
    c.mdf_iters = int(p.get("mdf_iters", 3))
    c.zeta = float(p.get("zeta", 1.0))
    c.eps_pp = float(p.get("eps_pp", 1e-3))
    c.E_pp = float(p.get("E_pp", 1e-4))
    c.cell_h = float(p.get("cell_h", 0.0))
    c.streaming = int(p.get("streaming", 0))
    c.forcing = int(p.get("forcing", 0))
    c.slip_tol = float(p.get("slip_tol", 1e30))
    c.fallback_iters = int(p.get("fallback_iters", 5))
    for fce in range(6):
        c.face_bc[fce] = int(p.get("face_bc", (0,) * 6)[fce])
        c.face_p[fce] = float(p.get("face_p", (0.0,) * 6)[fce])
    return c


class Sim:
    """One oracle context."""

    def __init__(self, params: dict):
        self.params = dict(params)
        self.cfg = make_config(params)
        self.dim = self.cfg.dim
        self.n = tuple(self.cfg.n[a] if a < self.dim else 1 for a in range(3))
        self.N = int(np.prod(self.n))
        self.q = 9 if self.dim == 2 else 19
        self.h = lib().ref_create(C.byref(self.cfg))
        if not self.h:
            raise ValueError("oracle rejected the configuration")
        self.np = 0

    def close(self):
        if self.h:
            lib().ref_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_equilibrium(self, p=None, u=None):
        lib().ref_set_equilibrium(self.h, _dp(_f64(p)), _dp(_f64(u)))

    def set_pdfs(self, f):
        f = _f64(f)
        assert f.size == (self.q - 1) * self.N
        lib().ref_set_pdfs(self.h, _dp(f))

    def get_pdfs(self):
        f = np.zeros((self.q - 1, self.N))
        lib().ref_get_pdfs(self.h, _dp(f))
        return f

    def add_particles(self, center, diameter, density, velocity=None, omega=None, n_markers=0):
        center = _f64(center, (-1, 3))
        n = center.shape[0]
        rc = lib().ref_add_particles(self.h, n, _dp(center), _dp(_f64(diameter)),
                                     _dp(_f64(density)), _dp(_f64(velocity, (-1, 3))),
                                     _dp(_f64(omega, (-1, 3))), int(n_markers))
        if rc != 0:
            raise ValueError("oracle rejected the particles")
        self.np += n

    def step(self, n=1):
        lib().ref_step(self.h, int(n))

    def fields(self):
        p = np.zeros(self.N)
        u = np.zeros((self.dim, self.N))
        f = np.zeros((self.dim, self.N))
        lib().ref_get_fields(self.h, _dp(p), _dp(u), _dp(f))
        return p, u, f

    def particles(self):
        out = [np.zeros((self.np, 3)) for _ in range(6)]
        lib().ref_get_particles(self.h, *[_dp(a) for a in out])
        return dict(zip(["X", "U", "Omega", "F_h", "T_h", "F_c"], out))

    def markers(self):
        m = lib().ref_num_markers(self.h)
        F = np.zeros((m, 3))
        r = np.zeros((m, 3))
        own = np.zeros(m, np.int32)
        dV = np.zeros(m)
        lib().ref_get_markers(self.h, _dp(F), _dp(r), _ip(own), _dp(dV))
        return dict(F=F, r=r, owner=own, dV=dV)

    def pairs(self):
        cap = 16
        while True:
            ij = np.zeros((cap, 2), np.int32)
            m = lib().ref_get_pairs(self.h, _ip(ij), cap)
            if m <= cap:
                return ij[:m].copy()
            cap = int(m)

    def cells(self):
        cell = np.zeros((self.np, 3), np.int32)
        dims = np.zeros(3, np.int32)
        h = np.zeros(3)
        lib().ref_get_cells(self.h, _ip(cell), _ip(dims), _dp(h))
        return cell, dims, h

    def mass(self):
        return lib().ref_mass(self.h)

    def slip_rms(self):
        return lib().ref_slip_rms(self.h)

    def truncated(self):
        return lib().ref_truncated(self.h)

    def fallbacks(self):
        return lib().ref_fallbacks(self.h)

    def judged_slip(self):
        """the slip the last learned prediction left, which the fallback tolerance judges"""
        return lib().ref_judged_slip(self.h)

    def set_mlp(self, params, norm):
        lib().ref_set_mlp(self.h, _dp(_f64(params)), _dp(_f64(norm)))

    def capture_samples(self):
        m = lib().ref_num_markers(self.h)
        feat = np.zeros((m, 10))
        tgt = np.zeros((m, 3))
        lib().ref_capture_samples(self.h, _dp(feat), _dp(tgt))
        return feat, tgt
