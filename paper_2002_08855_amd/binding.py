"""ctypes binding of the C ABI in ``include/iblbm.h`` (argument marshalling only).

Every computation runs in the HIP library ``libiblbm.so`` built from ``csrc/``; this
module only converts numpy arrays to host pointers, fills the config struct, and hands
PyTorch's caching allocator and current HIP stream to the library.  Importing it fails
loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libiblbm.so")

STORAGE = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3}
STATUS = {0: "OK", 1: "E_ARG", 2: "E_NOMEM", 3: "E_DEVICE", 4: "E_STATE", 5: "E_UNSTABLE",
          6: "E_CAPACITY", 7: "E_CELL_OVERFLOW"}
NPARAM = 10 * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3
TIMERS = ["collide", "band", "interp", "spread", "interior", "particle", "mlp", "other"]

_ALLOC = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Config(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("dim", C.c_int32), ("n", C.c_int32 * 3),
        ("tau", C.c_double), ("rho0", C.c_double), ("body_force", C.c_double * 3),
        ("periodic", C.c_int32 * 3), ("wall_u", (C.c_double * 3) * 6),
        ("storage", C.c_int32), ("f16_scale", C.c_double), ("delta", C.c_int32),
        ("drs", C.c_double), ("mdf_iters", C.c_int32), ("gravity", C.c_double * 3),
        ("zeta", C.c_double), ("eps_pp", C.c_double), ("E_pp", C.c_double),
        ("cell_h", C.c_double), ("forcing", C.c_int32), ("slip_tol", C.c_double),
        ("fallback_iters", C.c_int32), ("stats_every", C.c_int32), ("stream", C.c_void_p),
        ("dev_alloc", _ALLOC), ("dev_free", _FREE), ("alloc_user", C.c_void_p),
        ("face_bc", C.c_int32 * 6), ("face_p", C.c_double * 6),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("slip_rms", C.c_double), ("truncated", C.c_int64),
        ("n_pairs", C.c_int64), ("flags", C.c_int32), ("fallbacks", C.c_int32),
        ("band_nodes", C.c_int64), ("time_ms", C.c_double * 8), ("launches", C.c_int64 * 8),
        ("band_lattice", C.c_int32), ("reserved", C.c_int32),
    ]


class TrainOpts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("seed", C.c_uint64), ("check_fp32", C.c_int32)]


class IblbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None
_P = C.POINTER
_d = _P(C.c_double)
_f = _P(C.c_float)
_i32 = _P(C.c_int32)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        sig = {
            "iblbm_create": (C.c_int, [_P(Config), _P(vp)]),
            "iblbm_destroy": (None, [vp]),
            "iblbm_last_error": (C.c_char_p, [vp]),
            "iblbm_set_equilibrium": (C.c_int, [vp, _d, _d]),
            "iblbm_set_pdfs": (C.c_int, [vp, _d]),
            "iblbm_get_pdfs": (C.c_int, [vp, _d]),
            "iblbm_add_particles": (C.c_int, [vp, C.c_int32, _d, _d, _d, _d, _d, C.c_int32]),
            "iblbm_step": (C.c_int, [vp, C.c_int32]),
            "iblbm_get_fields": (C.c_int, [vp, _d, _d, _d]),
            "iblbm_get_forces": (C.c_int, [vp, _d, _d, _d, _d, _d, _d, _d]),
            "iblbm_get_pairs": (C.c_int, [vp, _i32, C.c_int64, _P(C.c_int64)]),
            "iblbm_get_cells": (C.c_int, [vp, _i32, _i32]),
            "iblbm_get_stats": (C.c_int, [vp, _P(Stats)]),
            "iblbm_num_particles": (C.c_int, [vp, _i32, _i32]),
            "iblbm_set_timing": (C.c_int, [vp, C.c_int32]),
            "iblbm_reset_stats": (C.c_int, [vp]),
            "iblbm_set_graph": (C.c_int, [vp, C.c_int32]),
            "iblbm_set_option": (C.c_int, [vp, C.c_int32, C.c_int32]),
            "iblbm_plan_units": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_int32,
                                           C.c_int32, _i32, _i32, _i32, _P(C.c_int64)]),
            "iblbm_set_mlp": (C.c_int, [vp, _f, _f]),
            "iblbm_capture_samples": (C.c_int, [vp, _f, _f]),
            "iblbm_nn_train": (C.c_int, [_f, _f, C.c_int64, _f, _P(TrainOpts), _f]),
            "iblbm_nn_grad": (C.c_int, [_f, _f, C.c_int64, _f, _f, _f]),
            "iblbm_nn_forward": (C.c_int, [_f, C.c_int64, _f, _f]),
            "iblbm_nn_grad_noalloc": (C.c_int, [vp, vp, C.c_int64, vp, vp, vp, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(_d)


def _fp(a):
    return None if a is None else a.ctypes.data_as(_f)


def _ip(a):
    return None if a is None else a.ctypes.data_as(_i32)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


def _f32(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a if shape is None else a.reshape(shape)


def make_config(p: dict, stream=None, use_torch_alloc=True):
    """Fill the C config struct from a parameter dict; returns (config, keepalive)."""
    c = Config()
    c.struct_size = C.sizeof(Config)
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
    c.storage = STORAGE[p.get("storage", "f64")]
    c.f16_scale = float(p.get("f16_scale", 1024.0))
    c.delta = int(p.get("delta", 0))
    c.drs = float(p.get("drs", 1.0))
    c.mdf_iters = int(p.get("mdf_iters", 3))
    c.zeta = float(p.get("zeta", 1.0))
    c.eps_pp = float(p.get("eps_pp", 1e-3))
    c.E_pp = float(p.get("E_pp", 1e-4))
    c.cell_h = float(p.get("cell_h", 0.0))
    c.forcing = int(p.get("forcing", 0))
    c.slip_tol = float(p.get("slip_tol", 1e30))
    c.fallback_iters = int(p.get("fallback_iters", 5))
    c.stats_every = int(p.get("stats_every", 0))
    for fce in range(6):
        c.face_bc[fce] = int(p.get("face_bc", (0,) * 6)[fce])
        c.face_p[fce] = float(p.get("face_p", (0.0,) * 6)[fce])
    keep = []
    if stream is not None:
        c.stream = stream
    if use_torch_alloc:
        import torch

        dev = torch.cuda.current_device()
        alloc_fn = torch.cuda.caching_allocator_alloc
        free_fn = torch.cuda.caching_allocator_delete
        finalizing = sys.is_finalizing

        def _alloc(nbytes, user):
            return alloc_fn(int(nbytes), dev)

        def _free(ptr, user):
            # A context still alive at interpreter exit is destroyed after torch's
            # modules are torn down; the process is ending and the driver reclaims
            # its memory, so the block is left to it.
            if not finalizing():
                free_fn(ptr)

        fa, ff = _ALLOC(_alloc), _FREE(_free)
        c.dev_alloc = fa
        c.dev_free = ff
        keep += [fa, ff]
    return c, keep


class Sim:
    """One GPU context.  Uses PyTorch's current HIP stream and caching allocator."""

    def __init__(self, params: dict, use_torch=True):
        self.params = dict(params)
        stream = None
        if use_torch:
            import torch

            if not torch.cuda.is_available():
                raise RuntimeError("no GPU: the IB-LBM library needs an MI355X (gfx950)")
            stream = torch.cuda.current_stream().cuda_stream
        self.cfg, self._keep = make_config(params, stream=stream, use_torch_alloc=use_torch)
        self.dim = self.cfg.dim
        self.n = tuple(self.cfg.n[a] if a < self.dim else 1 for a in range(3))
        self.N = int(np.prod(self.n))
        self.q = 9 if self.dim == 2 else 19
        h = C.c_void_p()
        self._check(lib().iblbm_create(C.byref(self.cfg), C.byref(h)), None)
        self.h = h

    def _check(self, st, h="self"):
        if st != 0:
            hh = self.h if h == "self" else h
            msg = lib().iblbm_last_error(hh).decode() if hh else "create failed"
            raise IblbmError(st, msg)

    def close(self):
        if getattr(self, "h", None):
            lib().iblbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_equilibrium(self, p=None, u=None):
        self._check(lib().iblbm_set_equilibrium(self.h, _dp(_f64(p)), _dp(_f64(u))))

    def set_pdfs(self, f):
        f = _f64(f)
        assert f.size == (self.q - 1) * self.N
        self._check(lib().iblbm_set_pdfs(self.h, _dp(f)))

    def get_pdfs(self):
        f = np.zeros((self.q - 1, self.N))
        self._check(lib().iblbm_get_pdfs(self.h, _dp(f)))
        return f

    def add_particles(self, center, diameter, density, velocity=None, omega=None, n_markers=0):
        center = _f64(center, (-1, 3))
        self._check(lib().iblbm_add_particles(
            self.h, center.shape[0], _dp(center), _dp(_f64(diameter)), _dp(_f64(density)),
            _dp(_f64(velocity, (-1, 3))), _dp(_f64(omega, (-1, 3))), int(n_markers)))

    def step(self, n=1):
        self._check(lib().iblbm_step(self.h, int(n)))

    def fields(self):
        p = np.zeros(self.N)
        u = np.zeros((self.dim, self.N))
        f = np.zeros((self.dim, self.N))
        self._check(lib().iblbm_get_fields(self.h, _dp(p), _dp(u), _dp(f)))
        return p, u, f

    def counts(self):
        a, b = C.c_int32(), C.c_int32()
        self._check(lib().iblbm_num_particles(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def particles(self):
        np_, nmk = self.counts()
        out = [np.zeros((np_, 3)) for _ in range(6)]
        mf = np.zeros((nmk, 3))
        self._check(lib().iblbm_get_forces(self.h, *[_dp(a) for a in out], _dp(mf)))
        d = dict(zip(["X", "U", "Omega", "F_h", "T_h", "F_c"], out))
        d["marker_F"] = mf
        return d

    def pairs(self):
        n = C.c_int64()
        self._check(lib().iblbm_get_pairs(self.h, None, 0, C.byref(n)))
        ij = np.zeros((max(1, n.value), 2), np.int32)
        self._check(lib().iblbm_get_pairs(self.h, _ip(ij), n.value, C.byref(n)))
        return ij[:n.value].copy()

    def cells(self):
        np_, _ = self.counts()
        cell = np.zeros((np_, 3), np.int32)
        dims = np.zeros(3, np.int32)
        self._check(lib().iblbm_get_cells(self.h, _ip(cell), _ip(dims)))
        return cell, dims

    def stats(self):
        s = Stats()
        self._check(lib().iblbm_get_stats(self.h, C.byref(s)))
        d = {k: getattr(s, k) for k, _ in Stats._fields_
             if k not in ("time_ms", "launches", "reserved")}
        d["time_ms"] = dict(zip(TIMERS, list(s.time_ms)))
        d["launches"] = dict(zip(TIMERS, list(s.launches)))
        return d

    def set_timing(self, mask=-1):
        """-1 (default) every kernel group, 0 off, else a bit mask over TIMERS (bit g for
        TIMERS[g])."""
        self._check(lib().iblbm_set_timing(self.h, int(mask)))

    def reset_stats(self):
        self._check(lib().iblbm_reset_stats(self.h))

    def set_option(self, option, value):
        self._check(lib().iblbm_set_option(self.h, int(option), int(value)))

    def set_ibm_lds(self, on=True):
        self.set_option(1, int(on))

    def set_stats_every(self, n):
        """compute the slip statistic every n steps (0: never)"""
        self.set_option(3, int(n))

    def set_band_pass(self, on=True):
        """band u* in its own lattice pass (True) or in the first interpolation (False)"""
        self.set_option(2, int(on))

    def set_timing_every(self, k):
        """with timing on, time the launches of every k-th step only"""
        self.set_option(4, int(k))

    def set_timing_kernel(self, on=True):
        """collide, interpolation and spreading groups: time the kernel itself (events
        recorded with its launch) instead of bracketing the group's launches"""
        self.set_option(5, int(on))

    def set_graph(self, on=True):
        self._check(lib().iblbm_set_graph(self.h, int(on)))

    def set_mlp(self, params, norm):
        self._check(lib().iblbm_set_mlp(self.h, _fp(_f32(params)), _fp(_f32(norm))))

    def capture_samples(self):
        _, nmk = self.counts()
        feat = np.zeros((nmk, 10), np.float32)
        tgt = np.zeros((nmk, 3), np.float32)
        self._check(lib().iblbm_capture_samples(self.h, _fp(feat), _fp(tgt)))
        return feat, tgt


def _raise(st, what):
    if st != 0:
        raise IblbmError(st, what)


def plan_units(dim, storage, diameter, n_points=0, lds_bytes=0):
    """Work units of the per-particle kernels for one particle (host-side planning):
    a list of (first point, point count, box-node bound); empty when the particle takes
    the point-wise kernels."""
    st = STORAGE[storage] if isinstance(storage, str) else int(storage)
    n = C.c_int32()
    _raise(lib().iblbm_plan_units(dim, st, lds_bytes, float(diameter), n_points, 0, C.byref(n),
                                  None, None, None), "iblbm_plan_units")
    first = np.zeros(n.value, np.int32)
    count = np.zeros(n.value, np.int32)
    nodes = np.zeros(n.value, np.int64)
    _raise(lib().iblbm_plan_units(dim, st, lds_bytes, float(diameter), n_points, n.value,
                                  C.byref(n), _ip(first), _ip(count),
                                  nodes.ctypes.data_as(_P(C.c_int64))), "iblbm_plan_units")
    return list(zip(first.tolist(), count.tolist(), nodes.tolist()))


def nn_forward(params, x):
    x = _f32(x, (-1, 10))
    y = np.zeros((x.shape[0], 3), np.float32)
    _raise(lib().iblbm_nn_forward(_fp(x), x.shape[0], _fp(_f32(params)), _fp(y)), "nn_forward")
    return y


def nn_grad(params, x, t):
    x = _f32(x, (-1, 10))
    t = _f32(t, (-1, 3))
    g = np.zeros(NPARAM, np.float32)
    loss = np.zeros(1, np.float32)
    _raise(lib().iblbm_nn_grad(_fp(x), _fp(t), x.shape[0], _fp(_f32(params)), _fp(loss), _fp(g)),
           "nn_grad")
    return float(loss[0]), g


def nn_grad_noalloc(x_ptr, t_ptr, n, params_ptr, loss_ptr, grad_ptr, stream=None):
    """iblbm_nn_grad_noalloc on device addresses (ints, e.g. torch tensor data_ptr());
    enqueued on `stream` (a hipStream_t as int, None for the null stream)."""
    _raise(lib().iblbm_nn_grad_noalloc(x_ptr, t_ptr, int(n), params_ptr, loss_ptr, grad_ptr,
                                       stream), "nn_grad_noalloc")


def nn_train(x, t, params, epochs=10, batch=4096, lr=1e-3, seed=0, check_fp32=False):
    x = _f32(x, (-1, 10))
    t = _f32(t, (-1, 3))
    P = _f32(params).copy()
    o = TrainOpts(epochs=epochs, batch=batch, lr=lr, beta1=0.9, beta2=0.999, eps=1e-8,
                  seed=seed, check_fp32=int(check_fp32))
    curve = np.zeros(epochs, np.float32)
    _raise(lib().iblbm_nn_train(_fp(x), _fp(t), x.shape[0], _fp(P), C.byref(o), _fp(curve)),
           "nn_train")
    return P, curve
