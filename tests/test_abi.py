"""The C-ABI library builds for gfx950, loads without a GPU, and exports every function
that include/iblbm.h declares; the oracle library exports what its header declares."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header, prefix):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(" + prefix + r"[a-z0-9_]+)\s*\(", text)))


def test_library_exports_header_symbols():
    from paper_2002_08855_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libiblbm.so not built")
    lib = ctypes.CDLL(binding.LIB_PATH)
    names = _declared(os.path.join(ROOT, "include", "iblbm.h"), "iblbm_")
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    binding.lib()  # every signature in the binding resolves


def test_oracle_exports_header_symbols():
    import oracle
    lib = ctypes.CDLL(oracle.LIB_PATH)
    names = _declared(os.path.join(ROOT, "oracle", "iblbm_ref.h"), "ref_")
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_config_struct_matches_header():
    """The binding's struct layout equals the C compiler's (struct_size check)."""
    from paper_2002_08855_amd import binding
    import subprocess
    import tempfile
    src = '#include "iblbm.h"\n#include <stdio.h>\nint main(){printf("%zu %zu %zu\\n", sizeof(iblbm_config), sizeof(iblbm_stats), sizeof(iblbm_train_opts));return 0;}\n'
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "t")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    assert int(out[0]) == ctypes.sizeof(binding.Config)
    assert int(out[1]) == ctypes.sizeof(binding.Stats)
    assert int(out[2]) == ctypes.sizeof(binding.TrainOpts)


def test_create_rejects_bad_config_without_gpu():
    """Validation happens before any device call: a bad config is refused on any host."""
    from paper_2002_08855_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libiblbm.so not built")
    from paper_2002_08855_amd import inputs
    for bad in (dict(tau=0.5), dict(tau=0.3), dict(storage="f64", dim=4)):
        p = inputs.default_params(2, (8, 8))
        p.update(bad)
        if p["dim"] not in (2, 3):
            cfg, _ = binding.make_config(dict(p, dim=2), use_torch_alloc=False)
            cfg.dim = p["dim"]
        else:
            cfg, _ = binding.make_config(p, use_torch_alloc=False)
        h = ctypes.c_void_p()
        st = binding.lib().iblbm_create(ctypes.byref(cfg), ctypes.byref(h))
        assert st == 1 and not h.value
    cfg, _ = binding.make_config(inputs.default_params(2, (8, 8)), use_torch_alloc=False)
    cfg.struct_size = 8
    h = ctypes.c_void_p()
    assert binding.lib().iblbm_create(ctypes.byref(cfg), ctypes.byref(h)) == 1


def _plan(*args, **kw):
    from paper_2002_08855_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libiblbm.so not built")
    return binding.plan_units(*args, **kw)


@pytest.mark.parametrize("dim,storage,D,npts,units", [
    # 21^3 box of FP32 sums: fits one workgroup's 160 KB but not two, so two bands
    (3, "f32", 16.0, 804, [(0, 402), (402, 402)]),
    # 17^3 box fits twice: one unit (16-bit storage computes in FP32 too)
    (3, "f32", 12.0, 452, [(0, 452)]),
    (3, "bf16", 12.0, 452, [(0, 452)]),
    (3, "f64", 12.0, 452, [(0, 226), (226, 226)]),
    (3, "f64", 10.0, 314, [(0, 157), (157, 157)]),
    # more points than a workgroup's 1024 lanes
    (2, "f64", 40.0, 2000, [(0, 1000), (1000, 1000)]),
    (2, "f32", 20.4, 64, [(0, 64)]),
    # FP64 bands of a D = 36 sphere stay wider than one workgroup's LDS: point-wise kernels
    (3, "f64", 36.0, 0, []),
])
def test_plan_units_cases(dim, storage, D, npts, units):
    """Host-side plan of the per-particle work units: whole particles, two bands, runs
    of at most a workgroup's points, or no plan."""
    assert [(f, c) for f, c, _ in _plan(dim, storage, D, npts)] == units


@pytest.mark.parametrize("dim,storage,D,npts", [
    (3, "f32", 16.0, 804), (3, "f64", 28.0, 0), (3, "f32", 30.0, 0), (3, "f64", 12.0, 452),
    (2, "f64", 40.0, 2000), (2, "f32", 48.0, 0), (3, "f32", 20.0, 0)])
def test_plan_units_cover_every_support(dim, storage, D, npts):
    """The units split the points into consecutive runs that cover each point once; each
    unit's box fits one workgroup's LDS; and it holds the union of the 4-point supports
    (Eqs. 47-48) of its points, placed by the oracle's own point generator, for centres
    at several sub-node offsets."""
    import oracle
    from paper_2002_08855_amd import inputs
    plan = _plan(dim, storage, D, npts)
    n = npts or int(np.floor((np.pi * D if dim == 2 else np.pi * D * D) + 0.5))
    assert plan and plan[0][0] == 0
    for (f0, c0, _), (f1, _, _) in zip(plan, plan[1:]):
        assert f1 == f0 + c0
    assert plan[-1][0] + plan[-1][1] == n
    cs = 8 if storage == "f64" else 4
    assert all(nodes * (dim * cs + 3) + 1024 <= 160 * 1024 for _, _, nodes in plan)
    side = int(D) + 24
    p = inputs.default_params(dim, (side,) * dim, storage="f64")
    rng = np.random.default_rng(5)
    for trial in range(3):
        c = np.array([side / 2 + rng.uniform(-0.5, 0.5) for _ in range(dim)] + [0.0] * (3 - dim))
        o = oracle.Sim(p)
        o.add_particles(c[None, :], [D], [1.5], n_markers=n)
        X = (c[None, :] + o.markers()["r"])[:, :dim]  # r: offsets from the centre
        o.close()
        for f, cnt, nodes in plan:
            pts = X[f:f + cnt]
            width = np.floor(pts.max(0)) - np.floor(pts.min(0)) + 4
            assert np.prod(width) <= nodes, (f, cnt, width, nodes)


def test_plan_units_rejects_bad_arguments():
    from paper_2002_08855_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libiblbm.so not built")
    n = ctypes.c_int32()
    L = binding.lib()
    for args in ((4, 1, 0, 10.0, 0), (3, 7, 0, 10.0, 0), (3, 1, 0, 0.0, 0), (3, 1, 0, -2.0, 0),
                 (3, 1, 0, 10.0, -1), (3, 1, 512, 10.0, 0), (2, 0, 0, float("nan"), 0)):
        assert L.iblbm_plan_units(*args, 0, ctypes.byref(n), None, None, None) == 1, args
    assert L.iblbm_plan_units(3, 1, 0, 10.0, 0, 0, None, None, None, None) == 1
