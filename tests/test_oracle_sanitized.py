"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (float-cast-
overflow included, no recovery) and driven through every path the other tests use:
two-array and swap streaming on walls, moving walls, periodic axes and inflow/outflow
faces; the IB forcing with both kernels, point-wise and naive; particles in 2-D and 3-D
with pairs and wall images; the coupling pins; the MLP and the learned forcing step.
Any out-of-bounds access, overflow or undefined conversion ends the child process."""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

CHILD = r'''
import sys
sys.path.insert(0, ROOT); sys.path.insert(0, HERE)
import numpy as np
import oracle
oracle.LIB_PATH = LIB
from paper_2002_08855_amd import inputs
import coupling_pins

for pin in coupling_pins.ALL:
    pin()
# fluid: walls with moving lids, periodic axes, both streaming schemes, faces
for dim, n, per in ((2, (23, 19), (0, 0, 0)), (2, (20, 16), (1, 0, 0)), (3, (9, 8, 7), (0, 1, 1))):
    for streaming in (0, 1):
        w = [[0.0, 0.0, 0.0] for _ in range(6)]
        w[3] = [0.01, 0.0, 0.003]
        p = inputs.default_params(dim, n, tau=0.7, periodic=per, wall_u=w, streaming=streaming,
                                  body_force=(1e-6, -2e-6, 1e-6))
        s = oracle.Sim(p)
        s.set_pdfs(inputs.random_pdfs(1, s.q, s.N))
        s.step(3)
        s.fields(); s.mass()
for dim, n in ((2, (12, 16)), (3, (8, 10, 9))):
    p = inputs.default_params(dim, n, tau=0.6, face_bc=(0, 0, 1, 2, 0, 0), face_p=(0, 0, 0, 0.001, 0, 0))
    p["wall_u"][2] = [0.0, 0.01, 0.0]
    s = oracle.Sim(p); s.step(3)
# particles: 2-D workload, both kernels and the thickened shell
for name in ("cavity128_f64", "cavity128_f64_btdf"):
    w = inputs.workload(name)
    s = oracle.Sim(w["params"])
    pr = w["particles"]
    s.add_particles(pr["center"], pr["diameter"], pr["density"], n_markers=pr["n_markers"])
    s.step(3)
    s.pairs(); s.cells(); s.markers(); s.particles()
# 3-D spheres near the walls and each other (pairs, wall images, truncated stencils)
p = inputs.default_params(3, (30, 28, 26), tau=0.7, mdf_iters=2)
s = oracle.Sim(p)
X = np.array([[6.2, 6.0, 6.4], [17.5, 6.3, 6.1], [12.0, 20.0, 19.3]])
s.add_particles(X, [10.0, 10.0, 12.0], [1.5, 2.0, 1.5], n_markers=0)
s.step(3)
# IB operators, naive and point-to-node, on both kernels
rng = np.random.default_rng(0)
for kind in (0, 1):
    u = rng.normal(size=2 * 20 * 18)
    Xp = np.column_stack([rng.uniform(-0.5, 19.5, 7), rng.uniform(-0.5, 17.5, 7), np.zeros(7)])
    for naive in (False, True):
        oracle.ibm_interp(2, (20, 18, 1), (0, 0, 0), kind, u, Xp, naive)
        oracle.ibm_spread(2, (20, 18, 1), (0, 0, 0), kind, rng.normal(size=(7, 3)), np.ones(7), Xp, naive)
oracle.grid_search(2, (64, 64, 1), rng.uniform(5, 58, size=(12, 3)) * [1, 1, 0], np.full(12, 6.0), 1.0, 7.0)
# MLP and the learned forcing step
P = rng.normal(0, 0.2, oracle.NPARAM)
x = rng.normal(size=(40, 10)); t = rng.normal(size=(40, 3))
oracle.mlp_forward(P, x); oracle.mlp_loss_grad(P, x, t)
p = inputs.default_params(3, (30, 28, 26), tau=0.7, mdf_iters=3, forcing=1, slip_tol=1e-30, fallback_iters=2)
s = oracle.Sim(p)
s.add_particles(X, [10.0, 10.0, 12.0], [1.5, 2.0, 1.5], n_markers=0)
norm = np.concatenate([np.zeros(10), np.ones(10), np.zeros(3), np.full(3, 1e-4)])
s.set_mlp(P, norm)
s.step(2)
s.capture_samples()
print("SANITIZED_OK", s.fallbacks())
'''


def test_oracle_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    if not (os.path.isabs(asan) and os.path.isabs(ubsan)):
        pytest.skip("sanitizer runtimes not found")
    lib = str(tmp_path / "libiblbm_ref_san.so")
    src = os.path.join(ROOT, "oracle", "iblbm_ref.c")
    subprocess.run(["gcc", "-O1", "-g", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                    "-fno-fast-math", "-fopenmp", "-Wno-unknown-pragmas",
                    "-fsanitize=address,undefined,float-cast-overflow", "-fno-sanitize-recover=all",
                    src, "-o", lib, "-lm"], check=True)
    env = dict(os.environ, LD_PRELOAD=f"{asan} {ubsan}", ASAN_OPTIONS="detect_leaks=0",
               OMP_NUM_THREADS="2")
    code = f"ROOT = {ROOT!r}\nHERE = {HERE!r}\nLIB = {lib!r}\n" + CHILD
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=600)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0 and "SANITIZED_OK" in r.stdout, r.stderr[-4000:]
