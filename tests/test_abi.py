"""The C-ABI library builds for gfx950, loads without a GPU, and exports every function
that include/iblbm.h declares; the oracle library exports what its header declares."""
import ctypes
import os
import re

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
